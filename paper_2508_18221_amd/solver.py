"""Python face of the C-ABI: a Solver owns one context and the two device
buffers it borrows.  PyTorch provides the device memory and the stream; all
arithmetic happens in the HIP kernels of libgrmhd.so."""

import ctypes

import numpy as np

from . import _lib
from ._lib import Grid, Phys, Diag, check, NFIELDS


def make_grid(nr, nth, nph, r_in=1.8, r_out=20.0, th_min=0.05, th_max=np.pi - 0.05,
              filt_alpha=36.0, filt_order=16, filter_on=True):
    return Grid(nr, nth, nph, r_in, r_out, th_min, th_max, filt_alpha, filt_order, int(filter_on))


def make_phys(M=1.0, a=0.5, gamma_ad=4.0 / 3.0, cfl=0.25, eta=2.0, cowling=False, gauge_k0=True,
              r_c=8.0, rho_c=1e-8, beta_min=100.0, pert_amp=1e-6, seed=1, rho_floor=1e-20, p_floor=1e-24):
    return Phys(M, a, gamma_ad, cfl, eta, int(cowling), int(gauge_k0), r_c, rho_c, beta_min,
                pert_amp, seed, rho_floor, p_floor)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One evolution context on the current CUDA (HIP) device and stream."""

    def __init__(self, grid, phys, prec=_lib.GRMHD_FP64, stream=None):
        import torch
        self.torch = torch
        lib = _lib.load()
        self.lib = lib
        self.grid, self.phys = grid, phys
        self.shape = (grid.nph, grid.nth, grid.nr)
        self.P = grid.nr * grid.nth * grid.nph
        res, scr = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib.grmhd_query_bytes(ctypes.byref(grid), prec, ctypes.byref(res), ctypes.byref(scr)))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.resident = torch.empty(res.value, dtype=torch.uint8, device="cuda")
        self.scratch = torch.empty(scr.value, dtype=torch.uint8, device="cuda")
        ctx = ctypes.c_void_p()
        check(lib.grmhd_create(ctypes.byref(grid), ctypes.byref(phys), prec, _ptr(self.resident),
                               _ptr(self.scratch), ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.byref(ctx)))
        self.ctx = ctx
        dU, dK = ctypes.c_void_p(), ctypes.c_void_p()
        check(lib.grmhd_state_ptr(ctx, ctypes.byref(dU), ctypes.byref(dK)))
        off = dU.value - self.resident.data_ptr()
        n = NFIELDS * self.P
        self.U = self.resident[off:off + 8 * n].view(torch.float64).view((NFIELDS,) + self.shape)
        offk = dK.value - self.resident.data_ptr()
        self.K0 = self.resident[offk:offk + 8 * self.P].view(torch.float64).view(self.shape)

    def close(self):
        if self.ctx:
            check(self.lib.grmhd_destroy(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state -------------------------------------------------------------------
    def init_state(self):
        check(self.lib.grmhd_init_state(self.ctx))

    def set_state(self, U, K0=None, t=0.0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        if U.size != NFIELDS * self.P:
            raise ValueError("state must have 32 * P entries")
        k = None
        if K0 is not None:
            K0 = np.ascontiguousarray(K0, dtype=np.float64)
            k = K0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        check(self.lib.grmhd_set_state(self.ctx, U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       U.size, k, float(t)))

    def get_state(self, with_k0=False):
        U = np.empty((NFIELDS,) + self.shape)
        K0 = np.empty(self.shape) if with_k0 else None
        check(self.lib.grmhd_get_state(self.ctx, U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), U.size,
                                       K0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if with_k0 else None))
        return (U, K0) if with_k0 else U

    # ---- compute -------------------------------------------------------------------
    def rhs(self, U_dev, out_dev):
        check(self.lib.grmhd_rhs(self.ctx, _ptr(U_dev), _ptr(out_dev)))

    def step(self, n=1):
        check(self.lib.grmhd_step(self.ctx, int(n)))

    def diagnostics(self):
        d = Diag()
        check(self.lib.grmhd_diagnostics(self.ctx, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def apply_operator(self, axis, op, inp, out):
        nf = inp.numel() // self.P
        check(self.lib.grmhd_apply_operator(self.ctx, int(axis), int(op), _ptr(inp), _ptr(out), nf))

    def con2prim(self, U_dev, prim_out, flux_out=None):
        check(self.lib.grmhd_con2prim(self.ctx, _ptr(U_dev), _ptr(prim_out),
                                      _ptr(flux_out) if flux_out is not None else None))

    def profile_step(self, nsteps=1):
        """Advance nsteps RK4 steps, returning {launch kind: (avg ms, count)}
        measured with HIP events on the context stream."""
        n = len(_lib.KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        check(self.lib.grmhd_profile_step(self.ctx, int(nsteps), ms, n, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KERNEL_KINDS)}

    @property
    def dt(self):
        return self.lib.grmhd_dt(self.ctx)

    @property
    def time(self):
        return self.lib.grmhd_time(self.ctx)
