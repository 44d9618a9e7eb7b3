"""Thin ctypes binding of libgpmood.so (include/gpmood.h), names as in the C ABI.

Argument marshalling only: every step of the stage runs in the HIP kernels of the
library.  PyTorch supplies device memory (uint8 tensors sized by
gpm_workspace_size) and the HIP stream.  If the library has not been built the
import fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpmood.so")

GPM_OK, GPM_EINVAL, GPM_ENOMEM, GPM_EHIP, GPM_ESTATE, GPM_ENOTCONV, GPM_EUNSUPPORTED = range(7)
GPM_F32, GPM_F64 = 0, 1
GPM_BC_PERIODIC, GPM_BC_OUTFLOW, GPM_BC_REFLECT = 0, 1, 2
GPM_CSD, GPM_PLATEAU, GPM_U2, GPM_RSCAD = 1, 2, 4, 8
GPM_FLAGS_ALL = 15

# every symbol include/gpmood.h declares
EXPORTS = ("gpm_create", "gpm_set_scheme", "gpm_workspace_size", "gpm_bind", "gpm_state_ptr",
           "gpm_init_state", "gpm_get_state", "gpm_compute_dt", "gpm_compute_dt_dev", "gpm_set_dt", "gpm_stage_dev",
           "gpm_stage_coef", "gpm_lincomb4",
           "gpm_step", "gpm_troubled_counts", "gpm_get_order_mask", "gpm_totals", "gpm_totals_dev",
           "gpm_totals_static",
           "gpm_set_tuning", "gpm_instrument", "gpm_instrument_read", "gpm_cascade_stats", "gpm_order_ptr", "gpm_adjoint_workspace_size",
           "gpm_bind_adjoint", "gpm_stage_vjp", "gpm_stage_vjp_acc",
           "gpm_batch_create",
           "gpm_batch_set_scheme", "gpm_batch_workspace_size", "gpm_batch_bind", "gpm_batch_set_tuning",
           "gpm_batch_set_tuning_per_problem", "gpm_batch_autotune", "gpm_batch_autotune_cascade",
           "gpm_batch_init_state", "gpm_batch_get_state", "gpm_batch_step", "gpm_batch_status",
           "gpm_batch_troubled_counts", "gpm_batch_get_order_mask", "gpm_batch_last_error",
           "gpm_batch_destroy", "gpm3_create", "gpm3_set_scheme", "gpm3_workspace_size", "gpm3_bind",
           "gpm3_init_state", "gpm3_get_state", "gpm3_compute_dt", "gpm3_step", "gpm3_troubled_counts",
           "gpm3_get_order_mask", "gpm3_totals", "gpm3_last_error", "gpm3_destroy",
           "gpm_strerror", "gpm_last_error", "gpm_destroy")


class gpm_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3), ("gamma", ctypes.c_double),
                ("slit", ctypes.c_int), ("slit_x", ctypes.c_double * 2), ("slit_prim", ctypes.c_double * 4),
                ("slit_prim_top", ctypes.c_double * 4)]


class gpm_scheme(ctypes.Structure):
    _fields_ = [("nlev", ctypes.c_int), ("radius", ctypes.c_int * 4), ("ell", ctypes.c_double),
                ("sigma_v", ctypes.c_double), ("sigma_p", ctypes.c_double), ("flags", ctypes.c_uint),
                ("stencil", ctypes.c_int), ("solver", ctypes.c_int)]


GPM_STENCILS = {"diamond": 0, "cross": 1, "poly3": 2}
GPM_SOLVERS = {"hllc": 0, "hll": 1}


class GpmError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libgpmood.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: the HIP library must be built (python -c "
                          "'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, st = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    ctxp = ctypes.c_void_p
    sig = {
        "gpm_create": ([ctypes.POINTER(gpm_grid), ctypes.c_int, vp, ctypes.POINTER(ctxp)], st),
        "gpm_set_scheme": ([ctxp, ctypes.POINTER(gpm_scheme)], st),
        "gpm_workspace_size": ([ctxp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], st),
        "gpm_bind": ([ctxp, vp, vp], st),
        "gpm_state_ptr": ([ctxp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int)], st),
        "gpm_init_state": ([ctxp, dp], st),
        "gpm_get_state": ([ctxp, dp], st),
        "gpm_compute_dt": ([ctxp, ctypes.c_double, dp], st),
        "gpm_compute_dt_dev": ([ctxp, vp, ctypes.c_double, dp], st),
        "gpm_set_dt": ([ctxp, ctypes.c_double], st),
        "gpm_stage_dev": ([ctxp, ctypes.c_int, vp, vp, vp], st),
        "gpm_stage_coef": ([ctxp, vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double], st),
        "gpm_lincomb4": ([ctxp, vp, vp, ctypes.c_double, vp, ctypes.c_double, vp, ctypes.c_double, vp,
                          ctypes.c_double], st),
        "gpm_step": ([ctxp, ctypes.c_double, ctypes.c_int], st),
        "gpm_troubled_counts": ([ctxp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)], st),
        "gpm_get_order_mask": ([ctxp, ctypes.POINTER(ctypes.c_ubyte)], st),
        "gpm_totals": ([ctxp, dp], st),
        "gpm_totals_dev": ([ctxp, vp, dp], st),
        "gpm_totals_static": ([ctxp, vp, dp], st),
        "gpm_set_tuning": ([ctxp, ctypes.c_int, ctypes.c_int, ctypes.c_int], st),
        "gpm_instrument": ([ctxp, ctypes.c_int], st),
        "gpm_instrument_read": ([ctxp, dp, ctypes.POINTER(ctypes.c_longlong), dp, ctypes.POINTER(ctypes.c_longlong),
                                 ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)], st),
        "gpm_cascade_stats": ([ctxp, ctypes.POINTER(ctypes.c_longlong)], st),
        "gpm_order_ptr": ([ctxp, ctypes.POINTER(vp)], st),
        "gpm_adjoint_workspace_size": ([ctxp, ctypes.POINTER(ctypes.c_size_t)], st),
        "gpm_bind_adjoint": ([ctxp, vp], st),
        "gpm_stage_vjp": ([ctxp, ctypes.c_int, vp, vp, vp, ctypes.c_double, vp, vp, vp, dp], st),
        "gpm_stage_vjp_acc": ([ctxp, ctypes.c_int, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp], st),
        "gpm_batch_create": ([ctypes.c_int, ctypes.POINTER(gpm_grid), ctypes.c_int, vp, ctypes.POINTER(ctxp)], st),
        "gpm_batch_set_scheme": ([ctxp, ctypes.POINTER(gpm_scheme)], st),
        "gpm_batch_workspace_size": ([ctxp, ctypes.POINTER(ctypes.c_size_t)], st),
        "gpm_batch_bind": ([ctxp, vp], st),
        "gpm_batch_set_tuning": ([ctxp, ctypes.c_int], st),
        "gpm_batch_set_tuning_per_problem": ([ctxp, ctypes.POINTER(ctypes.c_int)], st),
        "gpm_batch_autotune": ([ctxp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp], st),
        "gpm_batch_autotune_cascade": ([ctxp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp], st),
        "gpm_batch_init_state": ([ctxp, ctypes.c_int, dp], st),
        "gpm_batch_get_state": ([ctxp, ctypes.c_int, dp], st),
        "gpm_batch_step": ([ctxp, ctypes.c_double, ctypes.c_int, ctypes.c_int], st),
        "gpm_batch_status": ([ctxp, ctypes.POINTER(ctypes.c_int), dp], st),
        "gpm_batch_troubled_counts": ([ctxp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                       ctypes.POINTER(ctypes.c_int)], st),
        "gpm_batch_get_order_mask": ([ctxp, ctypes.c_int, ctypes.POINTER(ctypes.c_ubyte)], st),
        "gpm_batch_last_error": ([ctxp], ctypes.c_char_p),
        "gpm_batch_destroy": ([ctxp], None),
        "gpm3_create": ([ctypes.POINTER(gpm_grid), ctypes.c_int, vp, ctypes.POINTER(ctxp)], st),
        "gpm3_set_scheme": ([ctxp, ctypes.POINTER(gpm_scheme)], st),
        "gpm3_workspace_size": ([ctxp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], st),
        "gpm3_bind": ([ctxp, vp, vp], st),
        "gpm3_init_state": ([ctxp, dp], st),
        "gpm3_get_state": ([ctxp, dp], st),
        "gpm3_compute_dt": ([ctxp, ctypes.c_double, dp], st),
        "gpm3_step": ([ctxp, ctypes.c_double, ctypes.c_int], st),
        "gpm3_troubled_counts": ([ctxp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)], st),
        "gpm3_get_order_mask": ([ctxp, ctypes.POINTER(ctypes.c_ubyte)], st),
        "gpm3_totals": ([ctxp, dp], st),
        "gpm3_last_error": ([ctxp], ctypes.c_char_p),
        "gpm3_destroy": ([ctxp], None),
        "gpm_strerror": ([st], ctypes.c_char_p),
        "gpm_last_error": ([ctxp], ctypes.c_char_p),
        "gpm_destroy": ([ctxp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class GPMood:
    """One 2D problem on the GPU: owns torch device buffers and a library context.

    nx, ny, lo, hi, bc=(bcx, bcy) with 0 periodic / 1 outflow / 2 reflecting wall, prec 'f32' | 'f64',
    cascade = GP radii ending in 0, ell = physical length scale (None: 12 min(dx, dy)),
    stencil "diamond" / "cross" / "poly3", solver "hllc" / "hll", slit None or
    (sides, x0, x1, (rho, u, v, p)): an inflow slit on the y boundaries (bit 0
    bottom, bit 1 top) over the cells with centres in [x0, x1].
    """

    def __init__(self, nx, ny, lo=(0.0, 0.0), hi=(1.0, 1.0), bc=(0, 0), prec="f64",
                 cascade=(3, 2, 1, 0), ell=None, gamma=1.4, sigma_v=5.0, sigma_p=5.0,
                 flags=GPM_FLAGS_ALL, stream=None, device=None, stencil="diamond", solver="hllc", slit=None):
        import torch
        L = lib()
        self.torch = torch
        self.device = torch.device(device if device is not None else "cuda")
        self.nx, self.ny = int(nx), int(ny)
        # everything but the stream, for a twin context (vjp_twin)
        self._init_kw = dict(lo=lo, hi=hi, bc=bc, prec=prec, cascade=cascade, ell=ell, gamma=gamma,
                             sigma_v=sigma_v, sigma_p=sigma_p, flags=flags, device=device, stencil=stencil,
                             solver=solver, slit=slit)
        self._twin = None
        self.prec = prec
        self.dtype = torch.float64 if prec == "f64" else torch.float32
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        g = gpm_grid()
        g.dim = 2
        g.n[0], g.n[1], g.n[2] = self.nx, self.ny, 1
        g.lo[0], g.lo[1] = lo
        g.hi[0], g.hi[1] = hi
        g.bc[0], g.bc[1] = bc
        g.gamma = gamma
        if slit is not None:
            # (sides, x0, x1, (rho, u, v, p)): an inflow slit on the y boundaries
            g.slit, g.slit_x[0], g.slit_x[1] = int(slit[0]), float(slit[1]), float(slit[2])
            top = slit[4] if len(slit) > 4 else slit[3]
            for k in range(4):
                g.slit_prim[k] = float(slit[3][k])
                g.slit_prim_top[k] = float(top[k])
        ctx = ctypes.c_void_p()
        self._check(L.gpm_create(ctypes.byref(g), GPM_F64 if prec == "f64" else GPM_F32,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)), None)
        self.ctx = ctx
        s = gpm_scheme()
        s.nlev = len(cascade)
        for k, r in enumerate(cascade):
            s.radius[k] = r
        s.ell = 0.0 if ell is None else float(ell)
        s.sigma_v, s.sigma_p, s.flags = sigma_v, sigma_p, flags
        s.stencil = GPM_STENCILS[stencil]
        s.solver = GPM_SOLVERS[solver]
        self._check(L.gpm_set_scheme(self.ctx, ctypes.byref(s)))
        dx, dy = (hi[0] - lo[0]) / self.nx, (hi[1] - lo[1]) / self.ny
        self.ell = 12.0 * min(dx, dy) if ell is None else float(ell)
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(L.gpm_workspace_size(self.ctx, ctypes.byref(sb), ctypes.byref(wb)))
        self.state_buf = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
        self.work_buf = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        self._check(L.gpm_bind(self.ctx, ctypes.c_void_p(self.state_buf.data_ptr()),
                               ctypes.c_void_p(self.work_buf.data_ptr())))
        self.slot_elems = sb.value // 3 // (8 if prec == "f64" else 4)

    # -- plumbing
    def _check(self, st, ctx=0):
        if st != GPM_OK:
            L = lib()
            msg = L.gpm_strerror(st).decode()
            c = self.ctx if ctx == 0 else ctx
            if c is not None:
                msg += ": " + (L.gpm_last_error(c) or b"").decode()
            raise GpmError(f"status {st}: {msg}")

    def close(self):
        if getattr(self, "_twin", None) is not None:
            self._twin.close()
            self._twin = None
        if getattr(self, "ctx", None) is not None:
            lib().gpm_destroy(self.ctx)
            self.ctx = None

    def vjp_twin(self):
        """A second context with this one's grid and scheme (so the same weights, bit
        for bit) on a stream of its own, made on the first call and kept: the
        checkpointed backward runs the stage adjoints of one segment on it while
        this context recomputes the previous segment."""
        if self._twin is None:
            st = self.torch.cuda.Stream(device=self.device)
            self._twin = GPMood(self.nx, self.ny, stream=st, **self._init_kw)
        return self._twin

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def slot(self, k):
        """Torch view (4, ny, nx) of state slot k."""
        n = 4 * self.nx * self.ny
        esz = 8 if self.prec == "f64" else 4
        base = self.state_buf[k * self.slot_elems * esz:(k * self.slot_elems + n) * esz]
        return base.view(self.dtype).view(4, self.ny, self.nx)

    def current_slot(self):
        p, cur = ctypes.c_void_p(), ctypes.c_int()
        self._check(lib().gpm_state_ptr(self.ctx, 0, ctypes.byref(p), ctypes.byref(cur)))
        return cur.value

    # -- ABI calls
    def gpm_init_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (4, self.ny, self.nx)
        self._check(lib().gpm_init_state(self.ctx, _dp(U)))

    def gpm_get_state(self):
        U = np.empty((4, self.ny, self.nx))
        self._check(lib().gpm_get_state(self.ctx, _dp(U)))
        return U

    def gpm_compute_dt(self, cfl, sync=True):
        if sync:
            dt = ctypes.c_double()
            self._check(lib().gpm_compute_dt(self.ctx, float(cfl), ctypes.byref(dt)))
            return dt.value
        self._check(lib().gpm_compute_dt(self.ctx, float(cfl), None))
        return None

    def gpm_compute_dt_dev(self, U, cfl):
        """dt from a device state U (torch (4, ny, nx)); kept on the device for the next stages."""
        assert U.dtype == self.dtype and U.is_contiguous() and U.numel() == 4 * self.nx * self.ny
        dt = ctypes.c_double()
        self._check(lib().gpm_compute_dt_dev(self.ctx, ctypes.c_void_p(U.data_ptr()), float(cfl), ctypes.byref(dt)))
        return dt.value

    def gpm_set_dt(self, dt):
        self._check(lib().gpm_set_dt(self.ctx, float(dt)))

    def gpm_stage_dev(self, s, Un, Us, Uout):
        """Un, Us, Uout: torch tensors (4, ny, nx) of the context dtype on the device."""
        for t in (Un, Us, Uout):
            assert t.dtype == self.dtype and t.is_contiguous() and t.numel() == 4 * self.nx * self.ny
        self._check(lib().gpm_stage_dev(self.ctx, int(s), ctypes.c_void_p(Un.data_ptr()),
                                        ctypes.c_void_p(Us.data_ptr()), ctypes.c_void_p(Uout.data_ptr())))

    def gpm_stage_coef(self, B, Us, Uout, a, b, cf):
        """General SSP-RK stage Uout = a B + b (Us - cf dt F(Us)) with the MOOD loop
        (B may be None when a == 0); torch tensors (4, ny, nx) on the device."""
        for t in (Us, Uout) + ((B,) if B is not None else ()):
            assert t.dtype == self.dtype and t.is_contiguous() and t.numel() == 4 * self.nx * self.ny
        self._check(lib().gpm_stage_coef(self.ctx, ctypes.c_void_p(B.data_ptr() if B is not None else 0),
                                         ctypes.c_void_p(Us.data_ptr()), ctypes.c_void_p(Uout.data_ptr()),
                                         float(a), float(b), float(cf)))

    def gpm_lincomb4(self, out, X0, w0, X1, w1, X2, w2, X3, w3):
        """out = w0 X0 + w1 X1 + w2 X2 + w3 X3 (device tensors, left to right)."""
        for t in (out, X0, X1, X2, X3):
            assert t.dtype == self.dtype and t.is_contiguous() and t.numel() == 4 * self.nx * self.ny
        self._check(lib().gpm_lincomb4(self.ctx, ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(X0.data_ptr()), float(w0), ctypes.c_void_p(X1.data_ptr()),
                                       float(w1), ctypes.c_void_p(X2.data_ptr()), float(w2),
                                       ctypes.c_void_p(X3.data_ptr()), float(w3)))

    def gpm_step(self, cfl=0.8, nsteps=1):
        self._check(lib().gpm_step(self.ctx, float(cfl), int(nsteps)))

    def gpm_troubled_counts(self):
        c = (ctypes.c_longlong * 4)()
        it = ctypes.c_int()
        self._check(lib().gpm_troubled_counts(self.ctx, c, ctypes.byref(it)))
        return np.array(list(c), dtype=np.int64), it.value

    def gpm_get_order_mask(self):
        m = np.empty((self.ny, self.nx), dtype=np.uint8)
        self._check(lib().gpm_get_order_mask(self.ctx, m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))))
        return m

    def gpm_totals(self):
        t = np.zeros(4)
        self._check(lib().gpm_totals(self.ctx, _dp(t)))
        return t

    def gpm_totals_dev(self, U):
        t = np.zeros(4)
        self._check(lib().gpm_totals_dev(self.ctx, ctypes.c_void_p(U.data_ptr()), _dp(t)))
        return t

    def gpm_cascade_stats(self):
        """(multi-block passes, tail passes, hand-backs) of the last stage's cascade."""
        st = (ctypes.c_longlong * 3)()
        self._check(lib().gpm_cascade_stats(self.ctx, st))
        return tuple(int(x) for x in st)

    def gpm_totals_static(self, U):
        """gpm_totals_dev without the bound workspace (the library's static scratch)."""
        t = np.zeros(4)
        self._check(lib().gpm_totals_static(self.ctx, ctypes.c_void_p(U.data_ptr()), _dp(t)))
        return t

    def gpm_order_ptr(self):
        """Torch uint8 view (ny, nx) of the context's order array (device memory)."""
        p = ctypes.c_void_p()
        self._check(lib().gpm_order_ptr(self.ctx, ctypes.byref(p)))
        off = p.value - self.work_buf.data_ptr()
        return self.work_buf[off:off + self.nx * self.ny].view(self.ny, self.nx)

    def bind_adjoint(self):
        """Allocate and bind the adjoint workspace (once; torch device memory)."""
        if getattr(self, "adj_buf", None) is None:
            nb = ctypes.c_size_t()
            self._check(lib().gpm_adjoint_workspace_size(self.ctx, ctypes.byref(nb)))
            self.adj_buf = self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.device)
            self._check(lib().gpm_bind_adjoint(self.ctx, ctypes.c_void_p(self.adj_buf.data_ptr())))

    def gpm_stage_vjp(self, s, Un, Us, order, dt, lam_out, lam_Us, lam_Un=None, want_dell=True):
        """Stage adjoint; torch device tensors.  Returns this stage's dL/d(ell) (or None).
        Binds the adjoint workspace on first use."""
        self.bind_adjoint()
        for t in (Us, lam_out, lam_Us) + (() if s == 0 else (Un,)) + (() if lam_Un is None else (lam_Un,)):
            assert t.dtype == self.dtype and t.is_contiguous() and t.numel() == 4 * self.nx * self.ny
        assert order.dtype == self.torch.uint8 and order.numel() == self.nx * self.ny
        d = ctypes.c_double(0.0)
        vp = ctypes.c_void_p
        self._check(lib().gpm_stage_vjp(self.ctx, int(s), vp(Un.data_ptr() if Un is not None else 0),
                                        vp(Us.data_ptr()), vp(order.data_ptr()), float(dt),
                                        vp(lam_out.data_ptr()), vp(lam_Us.data_ptr()),
                                        vp(lam_Un.data_ptr() if lam_Un is not None else 0),
                                        ctypes.byref(d) if want_dell else None))
        return d.value if want_dell else None

    def gpm_stage_vjp_acc(self, s, Un, Us, order, dt, lam_out, lam_Us, lam_Un, dl_dev):
        """Stage adjoint adding dL/d(ell) into the float64 device tensor dl_dev (one
        element), in stream order, without synchronising."""
        self.bind_adjoint()
        for t in (Us, lam_out, lam_Us) + (() if s == 0 else (Un,)) + (() if lam_Un is None else (lam_Un,)):
            assert t.dtype == self.dtype and t.is_contiguous() and t.numel() == 4 * self.nx * self.ny
        assert order.dtype == self.torch.uint8 and order.numel() == self.nx * self.ny
        assert dl_dev.dtype == self.torch.float64 and dl_dev.numel() >= 1 and dl_dev.is_cuda
        vp = ctypes.c_void_p
        self._check(lib().gpm_stage_vjp_acc(self.ctx, int(s), vp(Un.data_ptr() if Un is not None else 0),
                                            vp(Us.data_ptr()), vp(order.data_ptr()), float(dt),
                                            vp(lam_out.data_ptr()), vp(lam_Us.data_ptr()),
                                            vp(lam_Un.data_ptr() if lam_Un is not None else 0),
                                            vp(dl_dev.data_ptr())))

    def gpm_set_tuning(self, passes_per_check=4, rows_per_wave=12, tail_threshold=32):
        self._check(lib().gpm_set_tuning(self.ctx, int(passes_per_check), int(rows_per_wave), int(tail_threshold)))

    def gpm_instrument(self, mode=1):
        """mode 0: off, 1: events and iteration counts, 3: also final-order counts (True means 1)."""
        self._check(lib().gpm_instrument(self.ctx, int(mode)))

    def gpm_instrument_read(self):
        fp, cm = ctypes.c_double(), ctypes.c_double()
        nfp, nst, it = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
        lev = (ctypes.c_longlong * 4)()
        self._check(lib().gpm_instrument_read(self.ctx, ctypes.byref(fp), ctypes.byref(nfp), ctypes.byref(cm),
                                              ctypes.byref(nst), lev, ctypes.byref(it)))
        return {"first_pass_ms": fp.value, "first_pass_launches": nfp.value, "cascade_ms": cm.value,
                "stages": nst.value, "level_cells": list(lev), "mood_iters": it.value}


class GPMoodBatch:
    """Many independent 2D problems advanced together (one launch per kernel kind).

    sizes: list of (nx, ny); lo, hi, bc, prec, cascade, ell as for GPMood (shared).
    """

    def __init__(self, sizes, lo=(0.0, 0.0), hi=(1.0, 1.0), bc=(0, 0), prec="f32", cascade=(3, 2, 1, 0),
                 ell=None, gamma=1.4, sigma_v=5.0, sigma_p=5.0, flags=GPM_FLAGS_ALL, stream=None, device=None,
                 solver="hllc"):
        import torch
        L = lib()
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        self.nprob = len(self.sizes)
        self.prec = prec
        self.top = int(cascade[0])
        self.torch = torch
        grids = (gpm_grid * len(self.sizes))()
        for k, (nx, ny) in enumerate(self.sizes):
            g = grids[k]
            g.dim = 2
            g.n[0], g.n[1], g.n[2] = nx, ny, 1
            g.lo[0], g.lo[1] = lo
            g.hi[0], g.hi[1] = hi
            g.bc[0], g.bc[1] = bc
            g.gamma = gamma
        b = ctypes.c_void_p()
        st = L.gpm_batch_create(len(self.sizes), grids, GPM_F64 if prec == "f64" else GPM_F32,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(b))
        if st != GPM_OK:
            raise GpmError(f"status {st}: {L.gpm_strerror(st).decode()}")
        self.b = b
        s = gpm_scheme()
        s.nlev = len(cascade)
        for k, r in enumerate(cascade):
            s.radius[k] = r
        s.ell = 0.0 if ell is None else float(ell)
        s.sigma_v, s.sigma_p, s.flags = sigma_v, sigma_p, flags
        s.solver = GPM_SOLVERS[solver]
        self._check(L.gpm_batch_set_scheme(self.b, ctypes.byref(s)))
        nb = ctypes.c_size_t()
        self._check(L.gpm_batch_workspace_size(self.b, ctypes.byref(nb)))
        self.buf = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self._check(L.gpm_batch_bind(self.b, ctypes.c_void_p(self.buf.data_ptr())))

    def _check(self, st):
        if st != GPM_OK:
            L = lib()
            raise GpmError(f"status {st}: {L.gpm_strerror(st).decode()}: "
                           f"{(L.gpm_batch_last_error(self.b) or b'').decode()}")

    def close(self):
        if getattr(self, "b", None) is not None:
            lib().gpm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gpm_batch_set_tuning(self, rows_per_wave=12):
        self._check(lib().gpm_batch_set_tuning(self.b, int(rows_per_wave)))

    def gpm_batch_set_tuning_per_problem(self, rows):
        arr = (ctypes.c_int * self.nprob)(*[int(r) for r in rows])
        self._check(lib().gpm_batch_set_tuning_per_problem(self.b, arr))

    def gpm_batch_autotune(self, cfl=0.8, reps=3):
        """Run the library's autotuner; returns (rows per problem, first-pass gain
        of the choice over the default march length)."""
        arr = (ctypes.c_int * self.nprob)()
        gain = ctypes.c_double()
        self._check(lib().gpm_batch_autotune(self.b, float(cfl), int(reps), arr, ctypes.byref(gain)))
        return [int(x) for x in arr], gain.value

    def gpm_batch_autotune_cascade(self, cfl=0.8, reps=3):
        """Choose the batch's cascade threshold on the device; returns (threshold, gain)."""
        t = ctypes.c_int()
        gain = ctypes.c_double()
        self._check(lib().gpm_batch_autotune_cascade(self.b, float(cfl), int(reps), ctypes.byref(t), ctypes.byref(gain)))
        return t.value, gain.value

    def autotune(self, cfl=0.8, reps=3, cache=None):
        """Autotuned march lengths with an on-disk cache (JSON file `cache`, keyed by
        device, precision, top radius and size class of problem): a batch whose
        classes are all cached takes the cached choice without timing anything.
        Returns (rows per problem, gain or None when taken from the cache)."""
        import json
        import os
        classes = [int(nx * ny).bit_length() - 1 for nx, ny in self.sizes]
        dev = self.torch.cuda.get_device_name(self.device)
        keys = [f"{dev}|{self.prec}|r{self.top}|c{k}" for k in classes]
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if all(k in table for k in keys):
            rows = [int(table[k]) for k in keys]
            self.gpm_batch_set_tuning_per_problem(rows)
            return rows, None
        rows, gain = self.gpm_batch_autotune(cfl, reps)
        if cache:
            for k, r in zip(keys, rows):
                table[k] = r
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return rows, gain

    def gpm_batch_init_state(self, p, U):
        nx, ny = self.sizes[p]
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (4, ny, nx)
        self._check(lib().gpm_batch_init_state(self.b, int(p), _dp(U)))

    def gpm_batch_get_state(self, p):
        nx, ny = self.sizes[p]
        U = np.empty((4, ny, nx))
        self._check(lib().gpm_batch_get_state(self.b, int(p), _dp(U)))
        return U

    def gpm_batch_step(self, cfl=0.8, nsteps=1, use_graph=True):
        self._check(lib().gpm_batch_step(self.b, float(cfl), int(nsteps), 1 if use_graph else 0))

    def gpm_batch_status(self):
        n = len(self.sizes)
        it = (ctypes.c_int * n)()
        dt = np.zeros(n)
        self._check(lib().gpm_batch_status(self.b, it, _dp(dt)))
        return np.array(list(it), dtype=np.int64), dt

    def gpm_batch_troubled_counts(self, p):
        c = (ctypes.c_longlong * 4)()
        it = ctypes.c_int()
        self._check(lib().gpm_batch_troubled_counts(self.b, int(p), c, ctypes.byref(it)))
        return np.array(list(c), dtype=np.int64), it.value

    def gpm_batch_get_order_mask(self, p):
        nx, ny = self.sizes[p]
        m = np.empty((ny, nx), dtype=np.uint8)
        self._check(lib().gpm_batch_get_order_mask(self.b, int(p), m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))))
        return m


class GPMood3D:
    """One 3D problem (GP-MOOD5 and lower) on the GPU: torch buffers and a gpm3 context.

    n = (nx, ny, nz); lo, hi, bc per axis (0 periodic / 1 outflow); state arrays are
    float64 host arrays (5, nz, ny, nx).
    """

    def __init__(self, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(1, 1, 1), prec="f32", cascade=(2, 1, 0),
                 ell=None, gamma=1.4, sigma_v=5.0, sigma_p=5.0, flags=GPM_FLAGS_ALL, stream=None, device=None):
        import torch
        L = lib()
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n = tuple(int(x) for x in n)
        self.prec = prec
        g = gpm_grid()
        g.dim = 3
        for a in range(3):
            g.n[a], g.lo[a], g.hi[a], g.bc[a] = self.n[a], lo[a], hi[a], bc[a]
        g.gamma = gamma
        ctx = ctypes.c_void_p()
        st = L.gpm3_create(ctypes.byref(g), GPM_F64 if prec == "f64" else GPM_F32,
                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if st != GPM_OK:
            raise GpmError(f"status {st}: {L.gpm_strerror(st).decode()}")
        self.ctx = ctx
        s = gpm_scheme()
        s.nlev = len(cascade)
        for k, r in enumerate(cascade):
            s.radius[k] = r
        s.ell = 0.0 if ell is None else float(ell)
        s.sigma_v, s.sigma_p, s.flags = sigma_v, sigma_p, flags
        self._check(L.gpm3_set_scheme(self.ctx, ctypes.byref(s)))
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(L.gpm3_workspace_size(self.ctx, ctypes.byref(sb), ctypes.byref(wb)))
        self.state_buf = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
        self.work_buf = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        self._check(L.gpm3_bind(self.ctx, ctypes.c_void_p(self.state_buf.data_ptr()),
                                ctypes.c_void_p(self.work_buf.data_ptr())))

    def _check(self, st):
        if st != GPM_OK:
            L = lib()
            raise GpmError(f"status {st}: {L.gpm_strerror(st).decode()}: "
                           f"{(L.gpm3_last_error(self.ctx) or b'').decode()}")

    def close(self):
        if getattr(self, "ctx", None) is not None:
            lib().gpm3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape(self):
        return (5, self.n[2], self.n[1], self.n[0])

    def gpm3_init_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == self._shape()
        self._check(lib().gpm3_init_state(self.ctx, _dp(U)))

    def gpm3_get_state(self):
        U = np.empty(self._shape())
        self._check(lib().gpm3_get_state(self.ctx, _dp(U)))
        return U

    def gpm3_compute_dt(self, cfl):
        dt = ctypes.c_double()
        self._check(lib().gpm3_compute_dt(self.ctx, float(cfl), ctypes.byref(dt)))
        return dt.value

    def gpm3_step(self, cfl=0.3, nsteps=1):
        self._check(lib().gpm3_step(self.ctx, float(cfl), int(nsteps)))

    def gpm3_troubled_counts(self):
        c = (ctypes.c_longlong * 3)()
        it = ctypes.c_int()
        self._check(lib().gpm3_troubled_counts(self.ctx, c, ctypes.byref(it)))
        return np.array(list(c), dtype=np.int64), it.value

    def gpm3_get_order_mask(self):
        m = np.empty(self._shape()[1:], dtype=np.uint8)
        self._check(lib().gpm3_get_order_mask(self.ctx, m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))))
        return m

    def gpm3_totals(self):
        t = np.zeros(5)
        self._check(lib().gpm3_totals(self.ctx, _dp(t)))
        return t
