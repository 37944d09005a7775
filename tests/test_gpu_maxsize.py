"""The largest grids the library accepts: 256 nodes on one axis (the LDS
bound of the one-tile contraction kernels, where an even size takes the
folded kernel with 128-row halves) and 255 on a Chebyshev axis (the unfolded
kernel with a 256-row padded tile).  Every operator and one coupled
right-hand side against the oracle; the reduced-precision forms' kernels at
the same sizes give a finite right-hand side."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from gpu_util import log, oracle_problem, rhs_errors, solver, workload  # noqa: E402
import workloads  # noqa: E402
from oracle import spectral  # noqa: E402

MAX_SIZES = [(256, 8, 8), (8, 256, 8), (8, 8, 256), (255, 9, 8), (9, 255, 8)]


def oracle_op(g, f, axis, op, alpha=36.0, order=16):
    ax = (-1, -2, -3)[axis]
    if op == 1:
        return g.d1(f, axis)
    if op == 2:
        return g.d2(f, axis, axis)
    if axis < 2:
        return spectral.cheb_filter(f, ax, alpha, order)
    return spectral.fourier_filter(f, ax, alpha, order)


def big_axis(size):
    return int(np.argmax(size))


@pytest.mark.parametrize("size", MAX_SIZES)
def test_operators_at_the_maximum_size(size):
    nr, nth, nph = size
    log(f"[operators, maximum size] grid {size}")
    w = workload("ks_michel_16x16x16", nr=nr, nth=nth, nph=nph)
    s = solver(w)
    g = spectral.Grid(nr, nth, nph, 1.8, 20.0, 0.05, np.pi - 0.05)
    nf = 4
    smooth = workloads.smooth_fields(g.r, g.th, g.ph, nf, seed=15)
    noise = workloads.random_fields(g.shape, nf, seed=16)
    for name, data in (("smooth", smooth), ("noise", noise)):
        dev_in = torch.tensor(data, device="cuda")
        for axis in range(3):
            for op in (1, 2, 3):
                dev_out = torch.full_like(dev_in, np.nan)
                s.apply_operator(axis, op, dev_in, dev_out)
                torch.cuda.synchronize()
                got = dev_out.cpu().numpy()
                ref = np.array([oracle_op(g, data[i], axis, op) for i in range(nf)])
                err = np.abs(got - ref).max() / np.abs(ref).max()
                n = size[axis]
                # FP64 conditioning of the two routes: ~N^2 eps (first), ~N^4 eps
                # (second); the filter is a dense sum of N terms on the library's
                # side (modal on the oracle's): ~N eps, 2e-15 N = 9 N eps
                tol = {1: 1e-15 * n * n, 2: 4e-16 * n ** 4, 3: max(1e-13, 2e-15 * n)}[op]
                log(f"  {name} axis {axis} op {op}: rel err {err:.2e} (tol {tol:.1e})")
                assert np.isfinite(got).all()
                assert err < max(tol, 1e-14), (name, axis, op, err)
    s.close()


@pytest.mark.parametrize("size", MAX_SIZES)
def test_rhs_at_the_maximum_size(size):
    """All derivative passes (two-operator and mixed tasks included) and the
    pointwise kernels on the oracle's Michel state; the bar is the second
    derivatives' FP64 conditioning along the long axis, 4e-16 N^4."""
    log(f"[rhs, maximum size] grid {size}")
    w = workload("ks_michel_16x16x16", nr=size[0], nth=size[1], nph=size[2])
    g, pb, U, K0 = oracle_problem(w)
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
    n = size[big_axis(size)]
    bar = max(4e-16 * n ** 4, 1e-11)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e) + f"  (bar {bar:.1e})")
    assert np.isfinite(got).all()
    assert e.max() < bar


@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("size", [(256, 8, 8), (8, 256, 8), (8, 8, 256), (255, 9, 8)])
def test_reduced_precision_forms_run_at_the_maximum_size(size, prec):
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    log(f"[mixed form {prec}, maximum size] grid {size}: one RHS and one step")
    w = workload("ks_michel_16x16x16", nr=size[0], nth=size[1], nph=size[2])
    s = Solver(make_grid(**w["grid"]), make_phys(**w["phys"]), prec=prec)
    s.init_state()
    U = s.get_state()
    dU = torch.tensor(U, device="cuda")
    out = torch.full_like(dU, np.nan)
    s.rhs(dU, out)
    s.step(1)
    d = s.diagnostics()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    s.close()
    assert np.isfinite(got).all()
    assert d["nonfinite"] == 0
