"""Python face of the C-ABI: a Solver owns one context and the two device
buffers it borrows.  PyTorch provides the device memory and the stream; all
arithmetic happens in the HIP kernels of libgrmhd.so."""

import ctypes

import numpy as np

from . import _lib
from ._lib import Grid, Phys, Diag, JobInfo, ServerStats, check, check_server, NFIELDS


def make_grid(nr, nth, nph, r_in=1.8, r_out=20.0, th_min=0.05, th_max=np.pi - 0.05,
              filt_alpha=36.0, filt_order=16, filter_on=True, dealias=False):
    return Grid(nr, nth, nph, r_in, r_out, th_min, th_max, filt_alpha, filt_order, int(filter_on), int(dealias))


def make_phys(M=1.0, a=0.5, gamma_ad=4.0 / 3.0, cfl=0.25, eta=2.0, cowling=False, gauge_k0=True,
              r_c=8.0, rho_c=1e-8, beta_min=100.0, pert_amp=1e-6, seed=1, rho_floor=1e-20, p_floor=1e-24,
              id_kind="michel", tor_r_in=6.0, tor_r_max=12.0, tor_rho_max=1e-8, tor_atm=1e-2,
              tor_loop_cut=0.2, glm=False, glm_ch=1.0, glm_tau=2.0, split=False, c2p="exact"):
    kind = {"michel": 0, "torus": 1}[id_kind]
    return Phys(M, a, gamma_ad, cfl, eta, int(cowling), int(gauge_k0), r_c, rho_c, beta_min,
                pert_amp, seed, rho_floor, p_floor, kind, tor_r_in, tor_r_max, tor_rho_max, tor_atm,
                tor_loop_cut, int(glm), glm_ch, glm_tau, int(split), {"exact": 0, "damped": 1}[c2p])


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One evolution context on the current CUDA (HIP) device and stream."""

    def __init__(self, grid, phys, prec=_lib.GRMHD_FP64, stream=None, scratch=True):
        """scratch=False: no scratch buffer (the context is stepped by
        step_noalloc only, its state set with set_state and an explicit K0)."""
        import torch
        self.torch = torch
        lib = _lib.load()
        self.lib = lib
        self.grid, self.phys = grid, phys
        self.shape = (grid.nph, grid.nth, grid.nr)
        self.P = grid.nr * grid.nth * grid.nph
        # fields of the state: 32, and psi with GLM constraint damping
        self.nfields = NFIELDS + 1 if phys.glm else NFIELDS
        res, scr = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib.grmhd_query_bytes(ctypes.byref(grid), prec, ctypes.byref(res), ctypes.byref(scr)))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        # one block: resident buffer, then scratch (contexts laid out alike can
        # be stepped together by step_batch)
        rb = (res.value + 255) // 256 * 256
        self.block = torch.empty(rb + (scr.value if scratch else 0), dtype=torch.uint8, device="cuda")
        self.resident = self.block[:rb]
        self.scratch = self.block[rb:] if scratch else None
        ctx = ctypes.c_void_p()
        check(lib.grmhd_create(ctypes.byref(grid), ctypes.byref(phys), prec, _ptr(self.resident),
                               _ptr(self.scratch) if scratch else None,
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx
        dU, dK = ctypes.c_void_p(), ctypes.c_void_p()
        check(lib.grmhd_state_ptr(ctx, ctypes.byref(dU), ctypes.byref(dK)))
        off = dU.value - self.resident.data_ptr()
        n = self.nfields * self.P
        self.U = self.resident[off:off + 8 * n].view(torch.float64).view((self.nfields,) + self.shape)
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
        if U.size not in (NFIELDS * self.P, self.nfields * self.P):
            raise ValueError("state must have 32 * P entries (33 * P with GLM)")
        k = None
        if K0 is not None:
            K0 = np.ascontiguousarray(K0, dtype=np.float64)
            k = K0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        check(self.lib.grmhd_set_state(self.ctx, U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       U.size, k, float(t)))

    def get_state(self, with_k0=False):
        U = np.empty((self.nfields,) + self.shape)
        K0 = np.empty(self.shape) if with_k0 else None
        check(self.lib.grmhd_get_state(self.ctx, U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), U.size,
                                       K0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if with_k0 else None))
        return (U, K0) if with_k0 else U

    # ---- compute -------------------------------------------------------------------
    def rhs(self, U_dev, out_dev):
        check(self.lib.grmhd_rhs(self.ctx, _ptr(U_dev), _ptr(out_dev)))

    def step(self, n=1):
        check(self.lib.grmhd_step(self.ctx, int(n)))

    def step_noalloc(self, n=1):
        """RK4 steps with the stage temporaries in the library's own device
        array (no scratch buffer of the context is used)."""
        check(self.lib.grmhd_step_noalloc(self.ctx, int(n)))

    def diagnostics(self):
        d = Diag()
        check(self.lib.grmhd_diagnostics(self.ctx, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def apply_operator(self, axis, op, inp, out):
        nf = inp.numel() // self.P
        check(self.lib.grmhd_apply_operator(self.ctx, int(axis), int(op), _ptr(inp), _ptr(out), nf))

    def con2prim(self, U_dev, prim_out, flux_out=None, fail_out=None):
        check(self.lib.grmhd_con2prim(self.ctx, _ptr(U_dev), _ptr(prim_out),
                                      _ptr(flux_out) if flux_out is not None else None,
                                      _ptr(fail_out) if fail_out is not None else None))

    def xcts_solve(self, E_dev, psi_dev, max_iter=200, tol=1e-11):
        """Conformal factor of the conformally flat, time-symmetric data:
        psi_dev holds the initial guess with the Dirichlet boundary values and
        receives the solution.  Returns (iterations, last relative change)."""
        it, ch = ctypes.c_int32(), ctypes.c_double()
        check(self.lib.grmhd_xcts_solve(self.ctx, _ptr(E_dev), _ptr(psi_dev), int(max_iter), float(tol),
                                        ctypes.byref(it), ctypes.byref(ch)))
        return it.value, ch.value

    def profile_step(self, nsteps=1):
        """Advance nsteps RK4 steps, returning {launch kind: (avg ms, count)}
        measured with HIP events on the context stream."""
        n = len(_lib.KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        check(self.lib.grmhd_profile_step(self.ctx, int(nsteps), ms, n, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KERNEL_KINDS)}

    def set_dt(self, dt):
        check(self.lib.grmhd_set_dt(self.ctx, float(dt)))

    @property
    def dt(self):
        return self.lib.grmhd_dt(self.ctx)

    @property
    def time(self):
        return self.lib.grmhd_time(self.ctx)


def step_batch(solvers, nsteps=1):
    """Advance same-class solvers together, one launch per kernel for all."""
    lib = _lib.load()
    arr = (ctypes.c_void_p * len(solvers))(*[s.ctx.value for s in solvers])
    check(lib.grmhd_step_batch(arr, len(solvers), int(nsteps)))


class Server:
    """Continuous-batching job server over a device arena of `budget` bytes
    (allocated here with PyTorch).  budget = 0 or dry=True: no device work."""

    def __init__(self, budget, max_batch=32, dry=False):
        lib = _lib.load()
        self.lib = lib
        self.arena = None
        ptr = None
        if not dry:
            import torch
            self.arena = torch.empty(int(budget), dtype=torch.uint8, device="cuda")
            ptr = ctypes.c_void_p(self.arena.data_ptr())
            stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        else:
            stream = None
        srv = ctypes.c_void_p()
        check_server(lib.grmhd_server_create(ptr, int(budget), int(max_batch), stream, ctypes.byref(srv)))
        self.srv = srv

    def close(self):
        if self.srv:
            self.lib.grmhd_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, grid, phys, t_end, prec=_lib.GRMHD_FP64, keep_state=False):
        jid = ctypes.c_int64()
        rc = self.lib.grmhd_server_submit(self.srv, ctypes.byref(grid), ctypes.byref(phys), int(prec),
                                          float(t_end), int(keep_state), ctypes.byref(jid))
        if rc == -5:   # over budget: the job is recorded as rejected
            return jid.value
        check_server(rc)
        return jid.value

    def tick(self):
        n = ctypes.c_int32()
        check_server(self.lib.grmhd_server_tick(self.srv, ctypes.byref(n)))
        return n.value

    def poll(self, job_id):
        info = JobInfo()
        check_server(self.lib.grmhd_server_poll(self.srv, int(job_id), ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in JobInfo._fields_}

    def cancel(self, job_id):
        """Cancel a queued or running job; its memory is released as soon as
        none of its steps is in flight."""
        check_server(self.lib.grmhd_server_cancel(self.srv, int(job_id)))

    def result(self, job_id, shape, nfields=NFIELDS):
        """Kept final state of a finished job (nfields 33 for a GLM job)."""
        U = np.empty((nfields,) + tuple(shape))
        check_server(self.lib.grmhd_server_result(self.srv, int(job_id),
                                                  U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), U.size))
        return U

    def stats(self):
        st = ServerStats()
        check_server(self.lib.grmhd_server_stats(self.srv, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def clock(self):
        return self.lib.grmhd_server_clock(self.srv)
