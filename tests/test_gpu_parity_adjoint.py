"""GPU adjoint through the C ABI, checked against central finite differences of the
plain FP64 oracle run with the same frozen cell orders and time steps.

The adjoint differentiates a stage with the forward's final orders and dt held
fixed, so the reference is the oracle's forced-order stage (Sec. "Stepwise
implementation" with the detection replaced by the recorded orders) at the GPU's
dt: d/d(eps) <lambda, S(U + eps v)> by a central difference.  The bar is the
spec 1e-4 relative; the differences seen are far smaller except where a
direction crosses an HLLC branch switch.
"""
import sys

import numpy as np
import pytest

import gpmood_inputs as gi
import oracle

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


@pytest.mark.parametrize("n,bc,s", [(32, (1, 1), 0), (32, (1, 1), 1), (28, (0, 0), 2), (30, (1, 0), 1)])
def test_stage_vjp_matches_oracle_fd(torch_cuda, n, bc, s):
    torch = torch_cuda
    from paper_2110_08683_amd import GPMood
    cascade = (3, 2, 1, 0)
    _note(f"stage vjp f64 n={n} bc={bc} s={s}")
    o = oracle.Oracle(n, n, bc=bc, cascade=cascade)
    U = o.run(gi.quadrants(n, n, seed=7), cfl=0.8, nsteps=2)[0]
    dt = o.dt(U, 0.8)
    U1 = o.stage(0, U, U, dt)[0]
    U2 = o.stage(1, U, U1, dt)[0]
    Us_h = (U, U1, U2)[s]
    g = GPMood(n, n, bc=bc, prec="f64", cascade=cascade, device="cuda:0")
    Un, Us = _dev(torch, U, torch.float64), _dev(torch, Us_h, torch.float64)
    out = torch.empty_like(Us)
    g.gpm_set_dt(dt)
    g.gpm_stage_dev(s, Un, Us, out)
    order = g.gpm_order_ptr().clone()
    mask = order.cpu().numpy().astype(np.int32)
    rng = np.random.default_rng(11 + s)
    lam = rng.standard_normal((4, n, n))
    lam_d = _dev(torch, lam, torch.float64)
    lUs = torch.empty_like(Us)
    lUn = torch.zeros_like(Us)
    dl = g.gpm_stage_vjp(s, Un, Us, order, dt, lam_d, lUs, lUn if s > 0 else None)
    lUs, lUn = lUs.cpu().numpy(), lUn.cpu().numpy()

    def phi(dUs=0.0, dUn=0.0, orc=o):
        if s == 0:
            a = U + dUs
            return float((lam * orc.stage_forced(0, a, a, dt, mask)).sum())
        return float((lam * orc.stage_forced(s, U + dUn, Us_h + dUs, dt, mask)).sum())

    scale = np.abs(Us_h).mean(axis=(1, 2), keepdims=True)
    eps = 1e-6
    for t in range(2):
        v = rng.standard_normal((4, n, n)) * scale
        fd = (phi(dUs=eps * v) - phi(dUs=-eps * v)) / (2 * eps)
        ad = float((lUs * v).sum())
        _note(f"  U_s direction {t}: fd {fd:.12e} adjoint {ad:.12e}")
        assert abs(fd - ad) <= 1e-4 * abs(fd)
        if s > 0:
            fd = (phi(dUn=eps * v) - phi(dUn=-eps * v)) / (2 * eps)
            ad = float((lUn * v).sum())
            _note(f"  U^n direction {t}: fd {fd:.12e} adjoint {ad:.12e}")
            assert abs(fd - ad) <= 1e-6 * abs(fd)  # linear in U^n
    h = 1e-5 * o.ell
    op = oracle.Oracle(n, n, bc=bc, cascade=cascade, ell=o.ell + h)
    om = oracle.Oracle(n, n, bc=bc, cascade=cascade, ell=o.ell - h)
    fd = (phi(orc=op) - phi(orc=om)) / (2 * h)
    _note(f"  ell: fd {fd:.12e} adjoint {dl:.12e}")
    assert abs(fd - dl) <= 1e-4 * abs(fd)
    g.close()


def _loss_box(n):
    """Box of the loss: the cells of the middle quarter of the domain."""
    a, b = n // 4, 3 * n // 4
    return slice(a, b), slice(a, b)


def _oracle_rollout_loss(o, U0, dts, masks, area, box):
    U = U0.copy()
    k = 0
    for dt in dts:
        U1 = o.stage_forced(0, U, U, dt, masks[k])
        U2 = o.stage_forced(1, U, U1, dt, masks[k + 1])
        U = o.stage_forced(2, U, U2, dt, masks[k + 2])
        k += 3
    return float((U[0][box] ** 2).sum() * area)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_rollout_gradient_vs_oracle_fd(torch_cuda, prec):
    """Vortex + Gaussian density bump, 48^2 on [0,10]^2 periodic, 7 steps with a
    checkpoint every 3: dL/d(rho^0) and dL/d(ell) of L = sum_box rho^2 dx dy."""
    torch = torch_cuda
    from paper_2110_08683_amd import GPMood
    from paper_2110_08683_amd.adjoint import _step, rollout
    n, nsteps = 48, 7
    _note(f"rollout {prec} n={n} steps={nsteps}")
    cascade = (3, 2, 1, 0)
    dtype = torch.float64 if prec == "f64" else torch.float32
    U0 = gi.vortex_bump(n, n, seed=5)
    g = GPMood(n, n, hi=(10.0, 10.0), bc=(0, 0), prec=prec, cascade=cascade, device="cuda:0")
    box = _loss_box(n)
    area = (10.0 / n) ** 2
    U0_d = _dev(torch, U0, dtype).requires_grad_(True)
    ell = torch.tensor(g.ell, dtype=torch.float64, requires_grad=True)
    UT = rollout(g, U0_d, nsteps, cfl=0.8, checkpoint_every=3, ell=ell)
    loss = (UT[0][box[0], box[1]].double() ** 2).sum() * area
    loss.backward()
    grad = U0_d.grad.double().cpu().numpy()
    dldell = float(ell.grad)
    # the forward's dt and orders, for the oracle with the same frozen choices
    dts, masks = [], []
    with torch.cuda.stream(g.stream):
        U = _dev(torch, U0, dtype)
        for _ in range(nsteps):
            U, dt, _, orders = _step(g, U, 0.8, keep=True)
            dts.append(dt)
            masks += [m.cpu().numpy().astype(np.int32) for m in orders]
    assert all((m == 3).all() for m in masks)  # the smooth flow keeps the top order
    o = oracle.Oracle(n, n, hi=(10.0, 10.0), bc=(0, 0), cascade=cascade)
    rng = np.random.default_rng(21)
    tol = 1e-4 if prec == "f64" else 2e-3
    for t in range(2):
        v = np.zeros((4, n, n))
        v[0] = rng.standard_normal((n, n)) * 0.01  # density only (rho u, rho v, E fixed)
        eps = 1e-4
        fd = (_oracle_rollout_loss(o, U0 + eps * v, dts, masks, area, box)
              - _oracle_rollout_loss(o, U0 - eps * v, dts, masks, area, box)) / (2 * eps)
        ad = float((grad * v).sum())
        _note(f"  rho direction {t}: fd {fd:.10e} adjoint {ad:.10e} rel {abs(fd - ad) / abs(fd):.2e}")
        assert abs(fd - ad) <= tol * abs(fd)
    h = 1e-5 * o.ell
    op = oracle.Oracle(n, n, hi=(10.0, 10.0), bc=(0, 0), cascade=cascade, ell=o.ell + h)
    om = oracle.Oracle(n, n, hi=(10.0, 10.0), bc=(0, 0), cascade=cascade, ell=o.ell - h)
    fd = (_oracle_rollout_loss(op, U0, dts, masks, area, box) - _oracle_rollout_loss(om, U0, dts, masks, area, box)) / (2 * h)
    _note(f"  ell: fd {fd:.10e} adjoint {dldell:.10e} rel {abs(fd - dldell) / abs(fd):.2e}")
    assert abs(fd - dldell) <= tol * abs(fd)
    g.close()
