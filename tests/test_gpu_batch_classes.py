"""Served form: a job's arithmetic is the same alone and in a batch of any
size (each result the same alone and in the mix, bitwise), for the grid
classes of the served stream where the contraction kernels change with the
grid (the copy-ahead contractions run on some axes of 32x32x64, 48x48x96 and
64x64x128): jobs stepped by grmhd_step_batch in batches of 4, 8 and 32 (2 at
64x64x128) equal the same jobs stepped alone, in the FP64, FP32 and
FP32-storage forms."""

import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


def make_jobs(n, nr, nth, nph, prec):
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    jobs = []
    for j in range(n):
        a = 0.95 * j / max(n - 1, 1)
        jobs.append(Solver(make_grid(nr, nth, nph), make_phys(a=a, seed=100 + j, beta_min=10.0 + 30.0 * j),
                           prec=prec))
    return jobs


@pytest.mark.parametrize("shape,sizes,prec", [
    ((32, 32, 64), (4, 8, 32), 0),
    ((32, 32, 64), (4, 8), 1),
    ((48, 48, 96), (4, 8), 0),
    ((48, 48, 96), (4,), 1),
    ((64, 64, 128), (2,), 0),
    ((32, 32, 64), (4, 8), 3),
    ((64, 64, 128), (2,), 3),
])
def test_batched_equals_alone(shape, sizes, prec):
    from paper_2508_18221_amd.solver import step_batch
    nmax = max(sizes)
    log(f"[batch classes] {shape} prec {prec}: batches of {sizes}")
    jobs = make_jobs(nmax, *shape, prec)
    watch = sorted({0, 3, nmax - 1} & set(range(nmax)))
    alone = {}
    for j in watch:
        jobs[j].init_state()
        jobs[j].step(2)
        alone[j] = jobs[j].get_state()
    for n in sizes:
        for s in jobs[:n]:
            s.init_state()
        step_batch(jobs[:n], 2)
        for j in watch:
            if j < n:
                got = jobs[j].get_state()
                assert np.isfinite(got).all()
                assert np.array_equal(got, alone[j]), (shape, prec, n, j)
        log(f"  batch of {n}: bitwise equal to alone for jobs {[j for j in watch if j < n]}")
    for s in jobs:
        s.close()
