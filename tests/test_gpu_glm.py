"""GPU parity of the GLM constraint-damping form (psi field, Methods "GLM
Constraint Damping Source") against the oracle, through the C-ABI: one
right-hand side on two grids and 10 RK4 steps, from the oracle's Michel state
with a smooth psi and a radial field perturbation that carries divergence
(so every GLM term is active); the FP32 form with GLM; and the cleaning effect
(the divergence of a seeded field shrinks with GLM and not without)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from gpu_util import workload, oracle_problem, solver, field_errors, rhs_errors, log  # noqa: E402

GLM = dict(glm=True, glm_ch=0.8, glm_tau=1.5)


def glm_workload(**grid):
    w = workload("ks_michel_16x16x16", **grid)
    w["phys"].update(GLM)
    return w


def seeded(g, U):
    """psi = 1e-4 exp(-ln(r/5)^2) cos(theta) sin(phi); sqrt(gamma) B^r scaled
    by 1 + 0.05 exp(-ln(r/5)^2) sin(theta) sin(phi) (nonzero divergence)."""
    U = U.copy()
    one = np.ones(g.shape)
    bump = np.exp(-np.log(g.R / 5.0) ** 2)
    U[29] = U[29] * (1.0 + 0.05 * bump * np.sin(g.TH) * np.sin(g.PH) * one)
    if U.shape[0] > 32:
        U[32] = 1e-4 * bump * np.cos(g.TH) * np.sin(g.PH) * one
    return U


@pytest.mark.parametrize("size", [(16, 16, 16), (20, 18, 12)])
def test_glm_rhs_matches_oracle(size):
    log(f"[glm rhs] grid {size}")
    w = glm_workload(nr=size[0], nth=size[1], nph=size[2])
    g, pb, U, K0 = oracle_problem(w)
    assert U.shape[0] == 33
    U = seeded(g, U)
    s = solver(w)
    s.set_state(U, K0)
    dU = torch.tensor(U, device="cuda")
    out = torch.full_like(dU, np.nan)
    s.rhs(dU, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    s.close()
    ref = pb.rhs(U, K0)
    e = rhs_errors(got, ref, U)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    assert np.isfinite(got).all()
    assert np.abs(ref[32]).max() > 0  # the psi right-hand side is active
    assert e.max() < 1e-11


def test_glm_ten_steps_match_oracle():
    log("[glm evolve] 16^3, 10 RK4 steps")
    w = glm_workload()
    g, pb, U, K0 = oracle_problem(w)
    U = seeded(g, U)
    ref = pb.evolve(U, K0, pb.dt(), 10)
    s = solver(w)
    s.set_state(U, K0)
    s.step(10)
    got = s.get_state()
    d = s.diagnostics()
    s.close()
    assert got.shape[0] == 33 and np.isfinite(got).all()
    e = field_errors(got, ref)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    assert e.max() < 1e-11
    assert d["nonfinite"] == 0 and d["c2p_fail"] == 0


@pytest.mark.parametrize("form", [1, 3])
def test_glm_fp32_form_close_to_fp64(form):
    """The FP32 and FP32-storage forms with GLM (the psi derivatives and the
    divergence of the field ride in the FP32 flux-derivative arrays)."""
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    log(f"[glm mixed] prec {form}, 16^3, 10 RK4 steps vs the FP64 path")
    w = glm_workload()
    g, pb, U, K0 = oracle_problem(w)
    U = seeded(g, U)
    out = {}
    for prec in (0, form):
        s = Solver(make_grid(**w["grid"]), make_phys(**w["phys"]), prec=prec)
        s.set_state(U, K0)
        s.step(10)
        out[prec] = s.get_state()
        s.close()
    assert np.isfinite(out[form]).all()
    rel = np.abs(out[form][32] - out[0][32]).max() / np.abs(out[0][32]).max()
    log(f"  psi max rel difference vs FP64: {rel:.2e}")
    assert rel < (1e-4 if form == 1 else 1e-6)


def test_glm_damps_a_seeded_divergence():
    """With psi = 0 and the divergence-carrying field, 120 steps at 16^3: the
    L2 norm (interior nodes) of d_i(sqrt(gamma) B^i) decreases with GLM
    (c_h = 1, tau = 0.5) and does not without it."""
    log("[glm cleaning] 16^3, 120 RK4 steps with and without GLM")
    norms = {}
    for glm in (False, True):
        w = workload("ks_michel_16x16x16")
        w["phys"].update(dict(glm=glm, glm_ch=1.0, glm_tau=0.5))
        g, pb, U, K0 = oracle_problem(w)
        U = seeded(g, U)
        if glm:
            U[32] = 0.0
        s = solver(w)
        s.set_state(U, K0)
        got0 = s.get_state()
        s.step(120)
        got = s.get_state()
        s.close()

        def div_l2(V):
            d = sum(g.d1(V[29 + i], i) for i in range(3))
            inner = (slice(None), slice(1, -1), slice(1, None))
            return np.sqrt(np.mean(d[inner] ** 2))
        norms[glm] = (div_l2(got0), div_l2(got))
        log(f"  glm={glm}: |div| {norms[glm][0]:.3e} -> {norms[glm][1]:.3e}")
    assert norms[True][1] < 0.95 * norms[True][0]
    assert norms[False][1] > norms[False][0]
    assert norms[True][1] < norms[False][1]


def test_served_glm_job_beside_a_plain_job_equals_alone():
    """A GLM job and a plain job of the same grid are different job classes
    (their kernels differ); served together, the GLM job's final state (psi
    included) equals the same job stepped alone."""
    from paper_2508_18221_amd import Server, Solver, make_grid, make_phys
    log("[server] GLM job beside a plain job on 16^3")
    srv = Server(budget=4 << 30, max_batch=32)
    g = make_grid(16, 16, 16)
    p_glm = make_phys(a=0.5, seed=41, **GLM)
    ids = [srv.submit(g, make_phys(a=0.5, seed=40), 0.05), srv.submit(g, p_glm, 0.06, keep_state=True)]
    while srv.tick() > 0:
        pass
    assert srv.stats()["completed"] == 2
    info = srv.poll(ids[1])
    served = srv.result(ids[1], (16, 16, 16), nfields=33)
    srv.close()
    s = Solver(g, p_glm)
    s.init_state()
    s.set_dt(info["dt"])
    s.step(info["steps_total"])
    alone = s.get_state()
    s.close()
    assert alone.shape[0] == 33
    assert np.array_equal(served, alone)
