"""Scheduling logic of the job server without a GPU (dry run: no device work,
each job step completes at once): FIFO admission against the memory budget,
continuous admission as memory frees up, rejection of oversize jobs, step
counts landing exactly on the end time, latency bookkeeping."""

import math

import pytest

from paper_2508_18221_amd import Server, make_grid, make_phys


def footprint(grid):
    import ctypes
    from paper_2508_18221_amd import _lib
    res, scr = ctypes.c_size_t(), ctypes.c_size_t()
    _lib.check(_lib.load().grmhd_query_bytes(ctypes.byref(grid), 0, ctypes.byref(res), ctypes.byref(scr)))
    return (res.value + 255) // 256 * 256 + (scr.value + 255) // 256 * 256


def dt_of(grid, cfl=0.25):
    import ctypes
    from paper_2508_18221_amd import _lib
    dt = ctypes.c_double()
    _lib.check(_lib.load().grmhd_time_step(ctypes.byref(grid), cfl, ctypes.byref(dt)))
    return dt.value


def test_budget_fifo_and_continuous_admission():
    g = make_grid(16, 16, 16)
    fp = footprint(g)
    srv = Server(budget=2 * fp + 100, dry=True)      # room for two jobs
    phys = make_phys()
    dt = dt_of(g)
    ends = [3 * dt, 5 * dt, 2 * dt, 1 * dt]
    ids = [srv.submit(g, phys, T) for T in ends]
    assert [srv.poll(i)["state"] for i in ids] == [0, 0, 0, 0]
    srv.tick()                                       # jobs 0, 1 admitted and stepped once
    st = [srv.poll(i) for i in ids]
    assert [s["state"] for s in st] == [1, 1, 0, 0]
    assert [s["steps_done"] for s in st] == [1, 1, 0, 0]
    assert [s["steps_total"] for s in st] == [3, 5, 2, 1]
    srv.tick()
    srv.tick()                                       # job 0 finishes at its third step
    assert srv.poll(0)["state"] == 2
    srv.tick()                                       # job 2 enters in the freed block
    assert srv.poll(2)["state"] == 1 and srv.poll(3)["state"] == 0
    while srv.tick() > 0:
        pass
    for i in ids:
        s = srv.poll(i)
        assert s["state"] == 2 and s["steps_done"] == s["steps_total"] and s["latency"] >= 0
    stats = srv.stats()
    assert stats["completed"] == 4 and stats["rejected"] == 0
    assert stats["bytes_in_use"] == 0 and stats["bytes_peak"] == 2 * fp
    assert stats["point_stage_updates"] == 4 * 16 ** 3 * (3 + 5 + 2 + 1)
    assert stats["p50_latency"] <= stats["p99_latency"]


def test_end_time_is_hit_exactly():
    g = make_grid(20, 18, 12)
    srv = Server(budget=footprint(g), dry=True)
    T = 0.0123
    j = srv.submit(g, make_phys(), T)
    info = srv.poll(j)
    dt = dt_of(g)
    assert info["steps_total"] == math.ceil(T / dt)
    assert abs(info["dt"] * info["steps_total"] - T) < 1e-15
    assert info["dt"] <= dt


def test_oversize_job_rejected_and_fifo_blocks_behind_large_job():
    small, big = make_grid(16, 16, 16), make_grid(32, 32, 64)
    fs, fb = footprint(small), footprint(big)
    srv = Server(budget=fb, dry=True)
    phys = make_phys()
    dt = dt_of(small)
    j_big = srv.submit(big, phys, 2 * dt_of(big))
    j_small = srv.submit(small, phys, dt)            # arrives behind the big job
    j_huge = srv.submit(make_grid(64, 64, 128), phys, 1.0)
    assert srv.poll(j_huge)["state"] == 3
    srv.tick()
    assert srv.poll(j_big)["state"] == 1
    # the small job waits (FIFO, the big job holds the whole budget)
    assert srv.poll(j_small)["state"] == 0
    while srv.tick() > 0:
        pass
    assert srv.poll(j_small)["state"] == 2
    assert srv.stats()["rejected"] == 1
    assert fs < fb


def test_invalid_submissions():
    srv = Server(budget=1 << 30, dry=True)
    with pytest.raises(Exception):
        srv.submit(make_grid(16, 16, 15), make_phys(), 1.0)
    with pytest.raises(Exception):
        srv.submit(make_grid(16, 16, 16), make_phys(), -1.0)


@pytest.mark.parametrize("bad", [
    dict(a=1.5),                                  # |a| > M
    dict(M=0.0, a=0.0),                           # no black hole: no initial data
    dict(gamma_ad=1.0),                           # Gamma <= 1
    dict(r_c=1.0),                                # inside the transonic Michel bound
    dict(beta_min=0.0),                           # no field normalisation
    dict(pert_amp=1.0),                           # perturbation outside [0, 1)
    dict(rho_c=0.0),
    dict(id_kind="torus", tor_r_in=12.0, tor_r_max=6.0),
    dict(glm=True, glm_tau=0.0),
    dict(split=True, cowling=True),
    dict(cfl=0.0),
])
def test_jobs_without_initial_data_are_refused_at_submission(bad):
    """A job whose parameters grmhd_create would refuse, or for which no
    initial data exist, is refused by submit (not queued), so it can never
    fail later inside a tick; the server keeps serving the valid jobs."""
    from paper_2508_18221_amd._lib import GrmhdError
    g = make_grid(16, 16, 16)
    srv = Server(budget=4 * footprint(g), dry=True)
    ok1 = srv.submit(g, make_phys(), 2 * dt_of(g))
    with pytest.raises(GrmhdError, match="rejected"):
        srv.submit(g, make_phys(**bad), 1.0)
    ok2 = srv.submit(g, make_phys(seed=3), dt_of(g))
    while srv.tick() > 0:
        pass
    assert srv.poll(ok1)["state"] == 2 and srv.poll(ok2)["state"] == 2
    st = srv.stats()
    assert st["submitted"] == 2 and st["completed"] == 2 and st["queued"] == 0


def test_cancel_frees_the_slot():
    """Cancelling a queued job takes it out of the queue; cancelling a running
    job releases its block, and the next queued job is admitted into it."""
    g = make_grid(16, 16, 16)
    fp = footprint(g)
    srv = Server(budget=fp + 100, dry=True)           # room for one job
    phys = make_phys()
    dt = dt_of(g)
    ids = [srv.submit(g, phys, 10 * dt) for _ in range(3)]
    srv.tick()                                       # job 0 admitted and stepped once
    assert [srv.poll(i)["state"] for i in ids] == [1, 0, 0]
    srv.cancel(ids[2])                               # queued: leaves the queue at once
    assert srv.poll(ids[2])["state"] == 4
    srv.cancel(ids[0])                               # running, no step in flight: released
    assert srv.poll(ids[0])["state"] == 4 and srv.poll(ids[0])["steps_done"] == 1
    assert srv.stats()["bytes_in_use"] == 0
    srv.tick()                                       # job 1 enters the freed block
    assert srv.poll(ids[1])["state"] == 1
    for i in (ids[0], ids[2]):
        with pytest.raises(RuntimeError, match="already done, rejected or cancelled"):
            srv.cancel(i)
    with pytest.raises(RuntimeError, match="unknown job"):
        srv.cancel(99)
    while srv.tick() > 0:
        pass
    st = srv.stats()
    assert srv.poll(ids[1])["state"] == 2 and st["completed"] == 1 and st["cancelled"] == 2
    assert st["bytes_in_use"] == 0 and st["point_stage_updates"] == 4 * 16 ** 3 * 10
