"""Served form on the GPU: jobs of one grid class stepped together (one launch
per kernel for all of them) give bitwise the same state as each job stepped
alone, and a job run through the continuous-batching server in a mix of jobs
of several classes ends bitwise where it ends when run alone."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from gpu_util import log  # noqa: E402


def r_in_for(a, M=1.0):
    """Inner radius scaled with the horizon so it stays inside it for every spin."""
    rh = lambda s: M + np.sqrt(M * M - s * s)  # noqa: E731
    return 1.8 * rh(a) / rh(0.5)


def job(a, beta, seed, size=(16, 16, 16)):
    from paper_2508_18221_amd import make_grid, make_phys
    return (make_grid(*size, r_in=r_in_for(a)), make_phys(a=a, beta_min=beta, seed=seed))


def test_step_batch_bitwise_equals_alone():
    from paper_2508_18221_amd import Solver, step_batch
    specs = [(0.1, 30.0, 11), (0.5, 100.0, 12), (0.9, 700.0, 13)]
    log("[batch] 3 jobs 16^3, 5 RK4 steps, batched vs alone")
    batch = []
    for a, b, sd in specs:
        g, p = job(a, b, sd)
        s = Solver(g, p)
        s.init_state()
        batch.append(s)
    step_batch(batch, 5)
    got = [s.get_state() for s in batch]
    for s in batch:
        s.close()
    for (a, b, sd), U in zip(specs, got):
        g, p = job(a, b, sd)
        s = Solver(g, p)
        s.init_state()
        s.step(5)
        ref = s.get_state()
        s.close()
        assert np.isfinite(U).all()
        assert np.array_equal(U, ref), f"job a={a}: max diff {np.abs(U - ref).max()}"


def test_server_result_equals_job_alone():
    from paper_2508_18221_amd import Server, Solver
    log("[server] 5 jobs in two grid classes; job 1 vs alone")
    srv = Server(budget=8 << 30, max_batch=32)
    specs = [((16, 16, 16), 0.2, 50.0, 21, 0.05), ((16, 16, 16), 0.7, 300.0, 22, 0.08),
             ((20, 18, 12), 0.4, 20.0, 23, 0.06), ((16, 16, 16), 0.95, 900.0, 24, 0.03),
             ((20, 18, 12), 0.0, 100.0, 25, 0.04)]
    ids = []
    for k, (size, a, beta, sd, T) in enumerate(specs):
        g, p = job(a, beta, sd, size)
        ids.append(srv.submit(g, p, T, keep_state=(k == 1)))
        srv.tick()                      # arrivals interleave with running work
    while srv.tick() > 0:
        pass
    st = srv.stats()
    log(f"  completed {st['completed']}, p50 {st['p50_latency']:.3f} s, p99 {st['p99_latency']:.3f} s")
    assert st["completed"] == len(specs)
    info = srv.poll(ids[1])
    size, a, beta, sd, T = specs[1]
    served = srv.result(ids[1], (size[2], size[1], size[0]))
    srv.close()
    g, p = job(a, beta, sd, size)
    s = Solver(g, p)
    s.init_state()
    s.set_dt(info["dt"])
    s.step(info["steps_total"])
    alone = s.get_state()
    s.close()
    assert abs(info["dt"] * info["steps_total"] - T) < 1e-15
    assert np.array_equal(served, alone)


def test_server_cancel_mid_run_frees_the_slot():
    """A budget for one 32x32x64 job: the running job is cancelled with steps
    still in flight; it takes no further step, its block is released once they
    complete, and the queued job is admitted into it and ends bitwise where it
    ends when run alone."""
    from paper_2508_18221_amd import Server, Solver
    from test_server_dry import footprint
    log("[server] cancel a running 32x32x64 job; the queued one takes its block")
    size = (32, 32, 64)
    g0, p0 = job(0.3, 60.0, 31, size)
    g1, p1 = job(0.6, 200.0, 32, size)
    fp = footprint(g0)
    srv = Server(budget=fp + 4096, max_batch=32)
    j0 = srv.submit(g0, p0, 0.2)
    j1 = srv.submit(g1, p1, 0.05, keep_state=True)
    for _ in range(3):
        srv.tick()                      # job 0 running, two steps in flight
    assert srv.poll(j0)["state"] == 1 and srv.poll(j1)["state"] == 0
    srv.cancel(j0)
    while srv.tick() > 0:
        pass
    i0, i1 = srv.poll(j0), srv.poll(j1)
    st = srv.stats()
    log(f"  job 0 cancelled after {i0['steps_done']} of {i0['steps_total']} steps; job 1 state {i1['state']}")
    assert i0["state"] == 4 and 0 < i0["steps_done"] < i0["steps_total"]
    assert i1["state"] == 2 and st["cancelled"] == 1 and st["completed"] == 1 and st["bytes_in_use"] == 0
    served = srv.result(j1, (size[2], size[1], size[0]))
    srv.close()
    s = Solver(g1, p1)
    s.init_state()
    s.set_dt(i1["dt"])
    s.step(i1["steps_total"])
    alone = s.get_state()
    s.close()
    assert np.array_equal(served, alone)
