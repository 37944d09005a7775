"""Reduced-precision forms: derivative contractions in FP32 or split-BF16x3
on MFMA with FP32 accumulation, or FP64 MFMA contractions whose derivative
arrays are stored in FP32 (the FP32-storage form); everything else FP64.
Bounds: after the evolution the density differs from the FP64 reference by
at most 1e-6 in relative L2 (unweighted over the nodes) and the
Hamiltonian-constraint L2 norm is within a factor 2 of the FP64 run's.

The FP32-storage form meets them also on the magnetised torus at
128 x 96 x 192 over 200 steps, where the FP32 form does not: rounding the
contraction inputs to FP32 is amplified by the derivative operators (up to
N^2 for D1 and N^4 for D2 relative to the field's variation), while rounding
the derivatives themselves once costs only their own unit roundoff."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from gpu_util import workload, oracle_problem, rhs_errors, log  # noqa: E402

PRECS = {"fp32": 1, "bf16x3": 2, "store32": 3}


def solver_prec(w, prec):
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    return Solver(make_grid(**w["grid"]), make_phys(**w["phys"]), prec=prec)


@pytest.mark.parametrize("name", ["fp32", "bf16x3", "store32"])
@pytest.mark.parametrize("size", [(16, 16, 16), (20, 18, 12)])
def test_mixed_rhs_close_to_oracle(name, size):
    log(f"[mixed rhs] {name} grid {size}")
    w = workload("ks_michel_16x16x16", nr=size[0], nth=size[1], nph=size[2])
    g, pb, U, K0 = oracle_problem(w)
    s = solver_prec(w, PRECS[name])
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
    # A characterisation, not the form's accuracy bound (that is on the
    # evolution, below): the contraction inputs are rounded to the low
    # precision (unit roundoff eps_low, after the shift by the line's middle
    # value), and the second-derivative operator amplifies an input error by
    # up to ||D2||_inf ~ N^4 / 3 (the CGL second-derivative matrix) relative to
    # the field's variation; the group scale of the right-hand side is at
    # least that variation, so e_f <= eps_low N^4.  The FP32-storage form
    # rounds the FP64 derivatives once (eps_32 of each) and feeds the mixed
    # second derivatives FP32 first derivatives (an input error amplified by
    # ||D1|| ~ N^2): e_f <= eps_32 N^2.
    if name == "store32":
        assert e.max() < 2.0 ** -24 * max(size) ** 2
        return
    eps = {"fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16}[name]
    assert e.max() < eps * max(size) ** 4


def rho_of(pb, U):
    return pb.primitives(U)["rho"]


BF16_MISS = ("split-BF16x3 keeps about 16 significand bits of each operand (2^-17 relative per hi/lo pair "
             "product left out), which the second-derivative operators amplify by ~N^4: measured rho L2 "
             "7.0e-6 at 16^3 after 10 steps and 8.7e-5 (Hamiltonian-norm ratio 6.05) at 64x64x128 after "
             "100 steps, against the bounds 1e-6 and 2")


@pytest.mark.parametrize("name", ["fp32", "store32",
                                  pytest.param("bf16x3", marks=pytest.mark.xfail(strict=True, reason=BF16_MISS))])
def test_mixed_evolution_within_bounds(name):
    log(f"[mixed evolve] {name} 16^3, 10 RK4 steps")
    w = workload("ks_michel_16x16x16")
    g, pb, U, K0 = oracle_problem(w)
    ref = pb.evolve(U, K0, pb.dt(), 10)
    s64 = solver_prec(w, 0)
    s64.set_state(U, K0)
    s64.step(10)
    d64 = s64.diagnostics()
    s64.close()
    s = solver_prec(w, PRECS[name])
    s.set_state(U, K0)
    s.step(10)
    got = s.get_state()
    d = s.diagnostics()
    s.close()
    r_ref, r_got = rho_of(pb, ref), rho_of(pb, got)
    l2 = np.sqrt(np.sum((r_got - r_ref) ** 2) / np.sum(r_ref ** 2))
    log(f"  rho L2 rel {l2:.2e}; H L2 {d['ham_l2']:.4e} vs FP64 {d64['ham_l2']:.4e}")
    assert d["nonfinite"] == 0 and d["c2p_fail"] == 0
    # the form's bounds: density within 1e-6 (relative L2), Hamiltonian-
    # constraint norm within 2x of the FP64 run's
    assert l2 < 1e-6
    assert d["ham_l2"] < 2.0 * d64["ham_l2"]


def test_hamiltonian_diagnostic_matches_oracle():
    from oracle import diagnostics
    from oracle.spectral import clenshaw_curtis_weights  # noqa: F401
    w = workload("ks_michel_16x16x16", nr=20, nth=18, nph=12)
    g, pb, U, K0 = oracle_problem(w)
    s = solver_prec(w, 0)
    s.set_state(U, K0)
    d = s.diagnostics()
    s.close()
    H = diagnostics.hamiltonian_constraint(pb, U)
    wts = diagnostics.weights(g)
    l2 = np.sqrt(np.sum(H * H * wts) / np.sum(wts))
    log(f"[ham] GPU L2 {d['ham_l2']:.6e} oracle {l2:.6e}; Linf {d['ham_linf']:.6e} vs {np.abs(H).max():.6e}")
    assert abs(d["ham_l2"] / l2 - 1) < 1e-9
    assert abs(d["ham_linf"] / np.abs(H).max() - 1) < 1e-9


@pytest.mark.parametrize("name", ["fp32", "store32"])
def test_fp32_form_full_size_within_bounds(name):
    """The FP32 and FP32-storage forms at 64 x 64 x 128, where their
    contractions take the copy-ahead pipelined kernels (all three axes):
    after 10 RK4 steps from the same state the density stays within 1e-6
    (relative L2) of the FP64 path and the Hamiltonian-constraint norm within
    a factor 2 of the FP64 run's."""
    log(f"[mixed evolve] {name} 64x64x128, 10 RK4 steps vs the FP64 path")
    w = workload("ks_michel_64x64x128")
    s64 = solver_prec(w, 0)
    s64.init_state()
    U0, K0 = s64.get_state(with_k0=True)
    s64.step(10)
    ref = s64.get_state()
    d64 = s64.diagnostics()
    s64.close()
    s = solver_prec(w, PRECS[name])
    s.set_state(U0, K0)
    s.step(10)
    got = s.get_state()
    d = s.diagnostics()
    s.close()
    # rest-mass density through the oracle's recovery on both states
    from oracle import spectral, evolve
    import workloads
    ga, pk, _ = workloads.oracle_kwargs(w)
    pb = evolve.Problem(spectral.Grid(*ga), **pk)
    r_ref, r_got = rho_of(pb, ref), rho_of(pb, got)
    l2 = np.sqrt(np.sum((r_got - r_ref) ** 2) / np.sum(r_ref ** 2))
    log(f"  rho L2 rel {l2:.2e}; H L2 {d['ham_l2']:.4e} vs FP64 {d64['ham_l2']:.4e}")
    assert np.isfinite(got).all()
    assert l2 < 1e-6
    assert d["ham_l2"] < 2.0 * d64["ham_l2"]
    assert d["nonfinite"] == 0 and d["c2p_fail"] == 0


def test_fp32_storage_form_within_bounds_on_the_torus():
    """The FP32-storage form on the magnetised torus at 128 x 96 x 192 (the
    second measured configuration, atmosphere nodes included) over its 200
    RK4 steps from the library's initial data: density within 1e-6 (relative
    L2, unweighted) of the FP64 path, Hamiltonian-constraint norm within a
    factor 2, the same atmosphere count.  (The FP32 form misses both here:
    rho 1.1e-5, norm ratio 20.)"""
    import workloads
    w = workloads.WORKLOADS["ks_torus_128x96x192"]
    steps = w["steps"]
    log(f"[store32] torus 128x96x192, {steps} RK4 steps vs the FP64 path")
    out = {}
    for name, prec in (("fp64", 0), ("store32", 3)):
        s = solver_prec(w, prec)
        s.init_state()
        s.step(steps)
        d = s.diagnostics()
        prim = torch.empty((5,) + s.shape, dtype=torch.float64, device="cuda")
        s.con2prim(s.U, prim)
        out[name] = (prim[0].clone(), d)
        s.close()
    r64, d64 = out["fp64"]
    r32, d32 = out["store32"]
    l2 = float(torch.sqrt(torch.sum((r32 - r64) ** 2) / torch.sum(r64 ** 2)))
    log(f"  rho L2 rel {l2:.2e}; H L2 {d32['ham_l2']:.4e} vs FP64 {d64['ham_l2']:.4e}; "
        f"atmosphere {d32['c2p_fail']} vs {d64['c2p_fail']}")
    assert d32["nonfinite"] == 0
    assert l2 < 1e-6
    assert d32["ham_l2"] < 2.0 * d64["ham_l2"]
    assert abs(d32["c2p_fail"] - d64["c2p_fail"]) <= 1e-3 * d64["c2p_fail"]
