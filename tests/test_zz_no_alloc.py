"""The allocation-free entry point (grmhd_step_noalloc) against grmhd_step,
through the C-ABI: contexts created without a scratch buffer, stepped with
the stage temporaries in the library's own device array, must end bitwise
equal to the same state stepped by grmhd_step with a scratch buffer of their
own -- on two calls in a row, the second on a smaller grid (the array keeps
the first call's contents), in the FP64 and FP32 forms and on a fixed
background (whose derivatives the array must not carry over between calls);
a grid too large for the array is refused with a clear error, and the
calls that need a scratch buffer refuse a context without one."""

import numpy as np
import pytest

from gpu_util import log, oracle_problem, workload

pytestmark = pytest.mark.gpu


def pair(w, prec=0):
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    g, p = make_grid(**w["grid"]), make_phys(**w["phys"])
    return Solver(g, p, prec=prec), Solver(g, p, prec=prec, scratch=False)


@pytest.mark.parametrize("prec,cowling", [(0, False), (1, False), (0, True)])
def test_noalloc_step_equals_step(prec, cowling):
    for over, nsteps in ((dict(nr=24, nth=20, nph=16), 3), (dict(nr=16, nth=16, nph=16), 2)):
        log(f"[noalloc] prec {prec} cowling {cowling} grid {over}, {nsteps} steps")
        w = workload("ks_michel_16x16x16", **over)
        w["phys"]["cowling"] = cowling
        g, pb, U, K0 = oracle_problem(w)
        ref, na = pair(w, prec)
        ref.set_state(U, K0)
        na.set_state(U, K0)
        ref.step(nsteps)
        na.step_noalloc(nsteps)
        a, b = ref.get_state(), na.get_state()
        ref.close()
        na.close()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b)


def test_noalloc_limits_and_refusals():
    from paper_2508_18221_amd._lib import GrmhdError
    log("[noalloc] 32x32x64 exceeds the array; scratch-less context refuses step, rhs, diagnostics, init")
    w = workload("ks_michel_16x16x16", nr=32, nth=32, nph=64)
    big_ref, big = pair(w)
    big_ref.init_state()
    U, K0 = big_ref.get_state(with_k0=True)
    big_ref.close()
    big.set_state(U, K0)
    with pytest.raises(GrmhdError, match="too large for grmhd_step_noalloc"):
        big.step_noalloc(1)
    big.close()
    w = workload("ks_michel_16x16x16")
    _, na = pair(w)
    with pytest.raises(GrmhdError, match="no scratch buffer"):
        na.init_state()
    g, pb, U, K0 = oracle_problem(w)
    with pytest.raises(GrmhdError, match="no scratch buffer"):
        na.set_state(U)                    # K0 from the state needs scratch
    na.set_state(U, K0)
    for call in (lambda: na.step(1), lambda: na.diagnostics()):
        with pytest.raises(GrmhdError, match="no scratch buffer"):
            call()
    na.step_noalloc(1)
    assert np.isfinite(na.get_state()).all()
    na.close()
