"""GP-MOOD oracle: plain FP64 CPU reference.  TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  The product library (paper_2110_08683_amd) never imports it and
shares no code with it; the two meet only through the seeded inputs of
gpmood_inputs and the values they return.

Parts:
  weights_mp.py     GP prediction vectors and u2 curvature weights in mpmath
                    (80 digits, rounded to double), eqs. (SE-pred), (SE-cov),
                    (gp_reconstructor), (normalized_z), App. B.
  gpmood_oracle.c   the stage: GP reconstruction, HLLC, candidate, MOOD loop
                    (Steps 3-10), SSP-RK3, dt, totals; plain loops in FP64; the
                    derivatives of a stage with frozen orders and dt (JVP with
                    dual numbers, and its transpose, the VJP).
  weights3d_mp.py   the same weights in 3D (L1-ball stencil, tensor Gauss nodes).
  gpmood_oracle3d.c the 3D stage (five variables), same steps.
  exact_riemann.py  Toro's exact Riemann solver for the 1D shock-tube pins.

Pins: see tests/test_oracle_*.py.  Every function here is pinned by at least
one test against something the paper or the mathematics fixes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import weights_mp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpmood_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC3 = os.path.join(_HERE, "gpmood_oracle3d.c")
_LIB3 = os.path.join(_HERE, "liboracle3d.so")

ORC_CSD, ORC_PLATEAU, ORC_U2, ORC_RSCAD = 1, 2, 4, 8
ORC_ALL = ORC_CSD | ORC_PLATEAU | ORC_U2 | ORC_RSCAD


def _compile(src, out, force):
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(force=True):
    """Compile the 2D and 3D oracles with gcc (plain -O2, no FP contraction, no fast-math)."""
    _compile(_SRC3, _LIB3, force)
    return _compile(_SRC, _LIB, force)


_lib = None


def rk4_stages():
    """The five-stage 4th-order SSP-RK of eqs. (rk4) and (rk4_substeps) as general
    stages U_out = a B + b (Us - cf dt F(Us)).  Sub-step i (i = 1..4):
    U(i) = alpha_i U^n + beta_i U(i-1) - gamma_i dt F(U(i-1)), so a = alpha_i,
    b = beta_i, cf = gamma_i / beta_i.  Reading: the last combination has both
    dt F terms subtracted, as every sub-step (the printed "+" on the U(3) term
    would not be 4th order); it is U^{n+1} = W + b5 (U(4) - cf5 dt F(U(4)))
    with W = c2 U(2) + c3 U(3) - d3 dt F(U(3)), where dt F(U(3)) is recovered
    from sub-step 4, dt F(U(3)) = (beta_4 U(3) + alpha_4 U^n - U(4)) / gamma_4,
    so W = w2 U(2) + w3 U(3) + w4 U(4) + wn U^n."""
    alpha = [0.0, 0.444370493651235, 0.620101851488403, 0.178079954393132]
    beta = [1.0, 0.555629506348765, 0.379898148511597, 0.821920045606868]
    gam = [0.391752226571890, 0.368410593050371, 0.251891774271694, 0.544974750228521]
    c2, c3, d3 = 0.517231671970585, 0.096059710526147, 0.063692468666290
    b5, d4 = 0.386708617503269, 0.226007483236906
    sub = [(alpha[i], beta[i], gam[i] / beta[i]) for i in range(4)]
    w = (c2, c3 - d3 * beta[3] / gam[3], d3 / gam[3], -d3 * alpha[3] / gam[3])
    return {"sub": sub, "w": w, "last": (1.0, b5, d4 / b5)}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        cp = ctypes.POINTER(_Cfg)
        L.orc_stage.argtypes = [cp, ctypes.c_int, dp, dp, ctypes.c_double, dp, ip,
                                ctypes.POINTER(ctypes.c_longlong)]
        L.orc_stage.restype = ctypes.c_int
        L.orc_stage_coef.argtypes = [cp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, dp, ip, ctypes.POINTER(ctypes.c_longlong)]
        L.orc_stage_coef.restype = ctypes.c_int
        L.orc_stage_forced.argtypes = [cp, ctypes.c_int, dp, dp, ctypes.c_double, ip, dp]
        L.orc_candidate.argtypes = [cp, dp, ctypes.c_double, ip, dp, ip]
        L.orc_criteria.argtypes = [cp, dp, dp, ip, ip, ctypes.POINTER(ctypes.c_uint), ip]
        L.orc_relax.argtypes = [cp, dp, dp]
        L.orc_dt.argtypes = [cp, dp, ctypes.c_double]
        L.orc_dt.restype = ctypes.c_double
        L.orc_run.argtypes = [cp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp,
                              ctypes.POINTER(ctypes.c_longlong), ip]
        L.orc_totals.argtypes = [cp, dp, dp]
        L.orc_hllc.argtypes = [ctypes.c_double, dp, dp, ctypes.c_int, dp]
        L.orc_hll.argtypes = [ctypes.c_double, dp, dp, ctypes.c_int, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_stage_jvp.argtypes = [cp, ctypes.c_int, dp, dp, dp, ctypes.c_double, ip, dp]
        L.orc_stage_vjp.argtypes = [cp, ctypes.c_int, dp, ctypes.c_double, ip, dp, dp, dp]
        _lib = L
    return _lib


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("bcx", ctypes.c_int), ("bcy", ctypes.c_int),
        ("gamma", ctypes.c_double),
        ("nlev", ctypes.c_int),
        ("rad", ctypes.c_int * 4),
        ("nst", ctypes.c_int * 4),
        ("off", ctypes.POINTER(ctypes.c_int) * 4),
        ("nq", ctypes.c_int * 4),
        ("qw", ctypes.POINTER(ctypes.c_double) * 4),
        ("z", ctypes.POINTER(ctypes.c_double) * 4),
        ("w2", ctypes.POINTER(ctypes.c_double)),
        ("off1", ctypes.POINTER(ctypes.c_int)),
        ("sigma_v", ctypes.c_double), ("sigma_p", ctypes.c_double),
        ("flags", ctypes.c_uint),
        ("solver", ctypes.c_int),
        ("slit", ctypes.c_int), ("slit_i0", ctypes.c_int), ("slit_i1", ctypes.c_int),
        ("slit_u", ctypes.c_double * 4), ("slit_u2", ctypes.c_double * 4),
    ]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class Oracle:
    """2D GP-MOOD oracle on a uniform grid [lo, hi] with nx-by-ny cells.

    bc: (bcx, bcy), 0 periodic / 1 outflow / 2 reflecting wall (mirror image with
    the normal momentum reversed; at least 4 cells, the ghost depth).  cascade: radii, strictly decreasing,
    ending in 0 (FOG).  ell: physical GP length scale.  shape: "diamond" (the
    blocky diamond), "cross" (the cross-shaped stencils of Sec. "Isentropic
    vortex") or "poly3" (POL-MOOD3: radius 1 with the polynomial weights).
    solver: "hllc" (the default) or "hll" (the paper's solver for the Mach jets).
    slit: None, or (sides, x0, x1, (rho, u, v, p)[, (rho, u, v, p) top]), an inflow
    slit on the y boundaries (bit 0 bottom, bit 1 top) over the cells with centres
    in [x0, x1]; the top side takes the second state if given.
    """

    def __init__(self, nx, ny, lo=(0.0, 0.0), hi=(1.0, 1.0), bc=(0, 0), cascade=(3, 2, 1, 0),
                 ell=None, gamma=1.4, sigma_v=5.0, sigma_p=5.0, flags=ORC_ALL, shape="diamond", solver="hllc",
                 slit=None):
        self.nx, self.ny = int(nx), int(ny)
        self.dx = (hi[0] - lo[0]) / nx
        self.dy = (hi[1] - lo[1]) / ny
        if ell is None:
            ell = 12.0 * min(self.dx, self.dy)
        self.ell = ell
        self.cascade = tuple(cascade)
        ax, ay = ell / self.dx, ell / self.dy
        self._keep = []
        c = _Cfg()
        c.nx, c.ny, c.dx, c.dy = self.nx, self.ny, self.dx, self.dy
        c.bcx, c.bcy = int(bc[0]), int(bc[1])
        for b, n in ((c.bcx, self.nx), (c.bcy, self.ny)):
            if b not in (0, 1, 2) or (b == 2 and n < 4):
                raise ValueError("bc 0 (periodic), 1 (outflow) or 2 (reflecting, >= 4 cells)")
        c.gamma = gamma
        c.nlev = len(cascade)
        if shape == "poly3" and max(cascade) > 1:
            raise ValueError("POL-MOOD3 has radius 1 (then FOG) only")
        for l, R in enumerate(cascade):
            if shape == "poly3" and R == 1:
                st = np.array(weights_mp.stencil(1), dtype=np.int32).reshape(-1)
                z = np.array(weights_mp.poly3_weights(), dtype=np.float64).reshape(-1)
            else:
                st = np.array(weights_mp.stencil(R, shape), dtype=np.int32).reshape(-1)
                z = np.array(weights_mp.weights(R, ax, ay, shape), dtype=np.float64).reshape(-1)
            q = weights_mp.nq(R)
            _, qw = weights_mp.gauss_rule_float(q)
            qw = np.array(qw, dtype=np.float64)
            self._keep += [st, z, qw]
            c.rad[l] = R
            c.nst[l] = len(st) // 2
            c.off[l] = _ip(st)
            c.nq[l] = q
            c.qw[l] = _dp(qw)
            c.z[l] = _dp(z)
        w2 = np.array(weights_mp.d2_weights(ax, ay, ell), dtype=np.float64).reshape(-1)
        off1 = np.array(weights_mp.stencil(1), dtype=np.int32).reshape(-1)
        self._keep += [w2, off1]
        c.w2 = _dp(w2)
        c.off1 = _ip(off1)
        c.sigma_v, c.sigma_p = sigma_v, sigma_p
        c.flags = flags
        if solver not in ("hllc", "hll"):
            raise ValueError("solver is 'hllc' or 'hll'")
        c.solver = 1 if solver == "hll" else 0
        if slit is not None:
            # slit = (sides, x0, x1, (rho, u, v, p)): sides bit 0 bottom, bit 1 top;
            # the cells whose centres lie in [x0, x1]; an outflow y axis elsewhere
            sides, x0, x1, prim = slit[:4]
            prim_top = slit[4] if len(slit) > 4 else prim
            if c.bcy != 1 or not 0 < sides < 4:
                raise ValueError("an inflow slit sits on outflow y boundaries")
            xc = lo[0] + (np.arange(self.nx) + 0.5) * self.dx
            inside = np.nonzero((xc >= x0) & (xc <= x1))[0]
            c.slit, c.slit_i0, c.slit_i1 = int(sides), int(inside[0]), int(inside[-1]) + 1
            for field, pr in ((c.slit_u, prim), (c.slit_u2, prim_top)):
                r, u, v, p = (float(x) for x in pr)
                field[:] = [r, r * u, r * v, p / (gamma - 1.0) + 0.5 * r * (u * u + v * v)]
        self.cfg = c
        self.gamma = gamma

    # -- helpers
    def _arr(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (4, self.ny, self.nx), U.shape
        return U

    def stage(self, s, Un, Us, dt):
        """One stage with the full MOOD loop.  Returns (Uout, order, counts, iters)."""
        Un, Us = self._arr(Un), self._arr(Us)
        out = np.empty_like(Us)
        order = np.empty((self.ny, self.nx), dtype=np.int32)
        counts = np.zeros(len(self.cascade), dtype=np.int64)
        it = lib().orc_stage(ctypes.byref(self.cfg), int(s), _dp(Un), _dp(Us), float(dt), _dp(out),
                             _ip(order), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
        return out, order, counts, it

    def stage_coef(self, B, Us, dt, a, b, cf):
        """General SSP-RK stage: U_out = a B + b U*, U* = Us - (cf dt) F(Us), with the
        full MOOD loop on U*.  Returns (Uout, order, counts, iters)."""
        B, Us = self._arr(B), self._arr(Us)
        out = np.empty_like(Us)
        order = np.empty((self.ny, self.nx), dtype=np.int32)
        counts = np.zeros(len(self.cascade), dtype=np.int64)
        it = lib().orc_stage_coef(ctypes.byref(self.cfg), _dp(B), _dp(Us), float(dt), float(a), float(b),
                                  float(cf), _dp(out), _ip(order),
                                  counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
        return out, order, counts, it

    def rk4_step(self, U, dt):
        """One step of the five-stage SSP-RK4 of eqs. (rk4) and (rk4_substeps),
        every stage with its own MOOD loop (rk4_stages).  Returns (U_next, iters)."""
        U = self._arr(U)
        st = rk4_stages()
        Ui = U
        keep = {}
        iters = []
        for i, (a, b, cf) in enumerate(st["sub"]):
            Ui, _, _, it = self.stage_coef(U, Ui, dt, a, b, cf)
            keep[i + 1] = Ui
            iters.append(it)
        k2, k3, k4, kn = st["w"]
        W = k2 * keep[2] + k3 * keep[3] + k4 * keep[4] + kn * U
        a, b, cf = st["last"]
        Un1, _, _, it = self.stage_coef(W, keep[4], dt, a, b, cf)
        iters.append(it)
        return Un1, iters

    def stage_forced(self, s, Un, Us, dt, order):
        Un, Us = self._arr(Un), self._arr(Us)
        order = np.ascontiguousarray(order, dtype=np.int32)
        out = np.empty_like(Us)
        lib().orc_stage_forced(ctypes.byref(self.cfg), int(s), _dp(Un), _dp(Us), float(dt),
                               _ip(order), _dp(out))
        return out

    def stage_jvp(self, s, Us, dUs, dUn, dt, order):
        """Directional derivative of the stage with the orders `order` and dt fixed
        (stage_forced): dU_out for tangents dUs of U_s and dUn of U^n (s = 0: U^n is
        U_s, dUn ignored)."""
        Us, dUs = self._arr(Us), self._arr(dUs)
        dUn = self._arr(dUn) if dUn is not None else np.zeros_like(Us)
        order = np.ascontiguousarray(order, dtype=np.int32)
        out = np.empty_like(Us)
        lib().orc_stage_jvp(ctypes.byref(self.cfg), int(s), _dp(Us), _dp(dUs), _dp(dUn), float(dt), _ip(order),
                            _dp(out))
        return out

    def stage_vjp(self, s, Us, dt, order, lam_out):
        """Transpose of stage_jvp: (lam_Us, lam_Un) for the adjoint lam_out of U_out
        (lam_Un is None for s = 0, where U^n is U_s)."""
        Us, lam_out = self._arr(Us), self._arr(lam_out)
        order = np.ascontiguousarray(order, dtype=np.int32)
        lus = np.empty_like(Us)
        lun = np.zeros_like(Us)
        lib().orc_stage_vjp(ctypes.byref(self.cfg), int(s), _dp(Us), float(dt), _ip(order), _dp(lam_out), _dp(lus),
                            _dp(lun))
        return lus, (lun if s > 0 else None)

    def candidate(self, Us, dt, order):
        Us = self._arr(Us)
        order = np.ascontiguousarray(order, dtype=np.int32)
        out = np.empty_like(Us)
        rs = np.empty((self.ny, self.nx), dtype=np.int32)
        lib().orc_candidate(ctypes.byref(self.cfg), _dp(Us), float(dt), _ip(order), _dp(out), _ip(rs))
        return out, rs

    def criteria(self, Us, Ustar, order, rsbad=None):
        Us, Ustar = self._arr(Us), self._arr(Ustar)
        order = np.ascontiguousarray(order, dtype=np.int32)
        bits = np.empty((self.ny, self.nx), dtype=np.uint32)
        tr = np.empty((self.ny, self.nx), dtype=np.int32)
        rsp = _ip(np.ascontiguousarray(rsbad, dtype=np.int32)) if rsbad is not None else None
        if rsbad is not None:
            rsbad = np.ascontiguousarray(rsbad, dtype=np.int32)
            rsp = _ip(rsbad)
        lib().orc_criteria(ctypes.byref(self.cfg), _dp(Us), _dp(Ustar), _ip(order), rsp,
                           bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint)), _ip(tr))
        return bits, tr

    def relax(self, Us):
        Us = self._arr(Us)
        out = np.empty((self.ny, self.nx, 5))
        lib().orc_relax(ctypes.byref(self.cfg), _dp(Us), _dp(out))
        return out

    def dt(self, U, cfl):
        return lib().orc_dt(ctypes.byref(self.cfg), _dp(self._arr(U)), float(cfl))

    def run(self, U, cfl=0.8, nsteps=1, fixed_dt=0.0):
        """nsteps SSP-RK3 steps.  Returns (U, dts, counts[nsteps,3,nlev], iters[nsteps,3])."""
        U = self._arr(U).copy()
        dts = np.zeros(nsteps)
        counts = np.zeros((nsteps, 3, len(self.cascade)), dtype=np.int64)
        iters = np.zeros((nsteps, 3), dtype=np.int32)
        lib().orc_run(ctypes.byref(self.cfg), _dp(U), float(cfl), float(fixed_dt), int(nsteps),
                      _dp(dts), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), _ip(iters))
        return U, dts, counts, iters

    def totals(self, U):
        t = np.zeros(4)
        lib().orc_totals(ctypes.byref(self.cfg), _dp(self._arr(U)), _dp(t))
        return t


def hllc(UL, UR, direction=0, gamma=1.4):
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    F = np.zeros(4)
    lib().orc_hllc(float(gamma), _dp(UL), _dp(UR), int(direction), _dp(F))
    return F


def hll(UL, UR, direction=0, gamma=1.4):
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    F = np.zeros(4)
    lib().orc_hll(float(gamma), _dp(UL), _dp(UR), int(direction), _dp(F))
    return F


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """OpenMP threads of the oracle's loops from now on (timing only)."""
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------------------- 3D
class _Cfg3(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("d", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3),
        ("gamma", ctypes.c_double),
        ("nlev", ctypes.c_int),
        ("rad", ctypes.c_int * 4),
        ("nst", ctypes.c_int * 4),
        ("off", ctypes.POINTER(ctypes.c_int) * 4),
        ("nq", ctypes.c_int * 4),
        ("qw", ctypes.POINTER(ctypes.c_double) * 4),
        ("z", ctypes.POINTER(ctypes.c_double) * 4),
        ("w2", ctypes.POINTER(ctypes.c_double)),
        ("off1", ctypes.POINTER(ctypes.c_int)),
        ("sigma_v", ctypes.c_double), ("sigma_p", ctypes.c_double),
        ("flags", ctypes.c_uint),
    ]


_lib3 = None


def lib3():
    global _lib3
    if _lib3 is None:
        _compile(_SRC3, _LIB3, False)
        L = ctypes.CDLL(_LIB3)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        cp = ctypes.POINTER(_Cfg3)
        L.orc3_stage.argtypes = [cp, ctypes.c_int, dp, dp, ctypes.c_double, dp, ip, ctypes.POINTER(ctypes.c_longlong)]
        L.orc3_stage.restype = ctypes.c_int
        L.orc3_dt.argtypes = [cp, dp, ctypes.c_double]
        L.orc3_dt.restype = ctypes.c_double
        L.orc3_run.argtypes = [cp, dp, ctypes.c_double, ctypes.c_int, dp, ip, ctypes.POINTER(ctypes.c_longlong)]
        L.orc3_hllc.argtypes = [ctypes.c_double, dp, dp, ctypes.c_int, dp]
        L.orc3_relax.argtypes = [cp, dp, dp]
        L.orc3_candidate.argtypes = [cp, dp, ctypes.c_double, ip, dp, ip]
        _lib3 = L
    return _lib3


class Oracle3D:
    """3D GP-MOOD oracle on [lo, hi] with n = (nx, ny, nz) cells, five variables
    (rho, rho u, rho v, rho w, E) in SoA (5, nz, ny, nx).  bc: per axis, 0 periodic /
    1 outflow.  cascade: radii (at most 2), strictly decreasing, ending in 0."""

    def __init__(self, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(1, 1, 1), cascade=(2, 1, 0),
                 ell=None, gamma=1.4, sigma_v=5.0, sigma_p=5.0, flags=ORC_ALL):
        from . import weights3d_mp as w3
        self.n = tuple(int(x) for x in n)
        self.d = tuple((hi[k] - lo[k]) / self.n[k] for k in range(3))
        if ell is None:
            ell = 12.0 * min(self.d)
        self.ell = ell
        self.cascade = tuple(cascade)
        a = [ell / self.d[k] for k in range(3)]
        self._keep = []
        c = _Cfg3()
        for k in range(3):
            c.n[k], c.d[k], c.bc[k] = self.n[k], self.d[k], int(bc[k])
        c.gamma = gamma
        c.nlev = len(cascade)
        for l, R in enumerate(cascade):
            st = np.array(w3.stencil3(R), dtype=np.int32).reshape(-1)
            z = np.array(w3.weights3(R, a[0], a[1], a[2]), dtype=np.float64).reshape(-1)
            qw = np.array(w3.node_weights3(R), dtype=np.float64)
            self._keep += [st, z, qw]
            c.rad[l] = R
            c.nst[l] = len(st) // 3
            c.off[l] = _ip(st)
            c.nq[l] = len(qw)
            c.qw[l] = _dp(qw)
            c.z[l] = _dp(z)
        w2 = np.array(w3.d2_weights3(a[0], a[1], a[2], ell), dtype=np.float64).reshape(-1)
        off1 = np.array(w3.stencil3(1), dtype=np.int32).reshape(-1)
        self._keep += [w2, off1]
        c.w2 = _dp(w2)
        c.off1 = _ip(off1)
        c.sigma_v, c.sigma_p, c.flags = sigma_v, sigma_p, flags
        self.cfg = c

    def _arr(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (5, self.n[2], self.n[1], self.n[0])
        return U

    def stage(self, s, Un, Us, dt):
        """One stage with the full MOOD loop.  Returns (Uout, order, counts, iters)."""
        Un, Us = self._arr(Un), self._arr(Us)
        out = np.empty_like(Us)
        order = np.empty((self.n[2], self.n[1], self.n[0]), dtype=np.int32)
        counts = np.zeros(len(self.cascade), dtype=np.int64)
        it = lib3().orc3_stage(ctypes.byref(self.cfg), int(s), _dp(Un), _dp(Us), float(dt), _dp(out),
                               _ip(order), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
        return out, order, counts, it

    def candidate(self, Us, dt, order):
        """U* = Us - dt F(Us) for the given per-cell radii, and the per-cell
        Riemann-state CAD flags."""
        Us = self._arr(Us)
        order = np.ascontiguousarray(order, dtype=np.int32)
        out = np.empty_like(Us)
        rs = np.empty(order.shape, dtype=np.int32)
        lib3().orc3_candidate(ctypes.byref(self.cfg), _dp(Us), float(dt), _ip(order), _dp(out), _ip(rs))
        return out, rs

    def relax(self, Us):
        """Per cell (nz, ny, nx, 5): rmin, rmax of the density over the cell and its six
        face neighbours, and the plateau, CSD and u2 verdicts (0/1)."""
        Us = self._arr(Us)
        out = np.empty((self.n[2], self.n[1], self.n[0], 5))
        lib3().orc3_relax(ctypes.byref(self.cfg), _dp(Us), _dp(out))
        return out

    def dt(self, U, cfl):
        return lib3().orc3_dt(ctypes.byref(self.cfg), _dp(self._arr(U)), float(cfl))

    def run(self, U, cfl=0.3, nsteps=1):
        """nsteps SSP-RK3 steps.  Returns (U, dts, iters[nsteps, 3], counts of the last stage)."""
        U = self._arr(U).copy()
        dts = np.zeros(nsteps)
        iters = np.zeros((nsteps, 3), dtype=np.int32)
        counts = np.zeros(len(self.cascade), dtype=np.int64)
        lib3().orc3_run(ctypes.byref(self.cfg), _dp(U), float(cfl), int(nsteps), _dp(dts), _ip(iters),
                        counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
        return U, dts, iters, counts


def hllc3(gamma, UL, UR, d):
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    F = np.zeros(5)
    lib3().orc3_hllc(float(gamma), _dp(UL), _dp(UR), int(d), _dp(F))
    return F
