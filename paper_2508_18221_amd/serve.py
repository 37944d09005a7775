"""Served form: replay a job stream against the continuous-batching server.

    python -m paper_2508_18221_amd.serve [--jobs 256] [--rate 4] [--t-scale 0.001] [--prec 0]

Jobs arrive on the wall clock at their (seeded Poisson) arrival times and are
submitted the moment the replay loop sees them; the server admits them against
the memory budget, keeps each grid class's next RK4 steps queued on the device
(one batched launch sequence per class and step, classes independent of each
other) and retires finished ones.  Latency is measured from the nominal
arrival time to the moment a tick sees the job's last step completed."""

import argparse
import json
import math
import time

import numpy as np

from .solver import Server, make_grid, make_phys


def horizon(a, M=1.0):
    return M + math.sqrt(M * M - a * a)


def job_args(j):
    """Grid and physics of one served job: the inner radius scales with the
    horizon radius so that it stays inside the horizon for every spin."""
    nr, nth, nph = j["grid"]
    grid = make_grid(nr, nth, nph, r_in=1.8 * horizon(j["a"]) / horizon(0.5))
    phys = make_phys(a=j["a"], beta_min=j["beta"], seed=j["seed"], cowling=j.get("cowling", False))
    return grid, phys


def run_stream(jobs, prec=0, budget=200e9, max_batch=32, log=None):
    srv = Server(budget=int(budget), max_batch=max_batch)
    t0 = srv.clock()
    ids, nxt, pending, ticks = [], 0, 0, 0
    n = len(jobs)
    while nxt < n or pending > 0:
        now = srv.clock() - t0
        new = 0
        while nxt < n and jobs[nxt]["arrival"] <= now:
            g, p = job_args(jobs[nxt])
            ids.append(srv.submit(g, p, jobs[nxt]["T"], prec=prec))
            nxt += 1
            new += 1
        if pending == 0 and new == 0:      # idle: wait for the next arrival
            time.sleep(max(0.0, jobs[nxt]["arrival"] - now))
            continue
        pending = srv.tick()
        ticks += 1
        if log and ticks % 200 == 0:
            log(f"serve: t={now:.1f}s submitted {nxt}/{n} pending {pending}")
    infos = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.close()
    done = [(inf, j) for inf, j in zip(infos, jobs) if inf["state"] == 2]
    lat = np.array([inf["t_done"] - t0 - j["arrival"] for inf, j in done])
    work = sum(4.0 * inf["steps_total"] * inf["nr"] * inf["nth"] * inf["nph"] for inf, _ in done)
    last = max(inf["t_done"] for inf, _ in done) - t0 if done else 0.0
    span = last - min(j["arrival"] for j in jobs)

    def pct(q):
        if lat.size == 0:
            return None
        s = np.sort(lat)
        return float(s[min(max(int(math.ceil(q * s.size)), 1), s.size) - 1])

    by_grid = {}
    for inf, j in done:
        key = f"{inf['nr']}x{inf['nth']}x{inf['nph']}" + ("/fixed" if j.get("cowling") else "")
        by_grid.setdefault(key, []).append(inf["t_done"] - t0 - j["arrival"])

    def pct_of(v, q):
        s = np.sort(np.asarray(v))
        return float(s[min(max(int(math.ceil(q * s.size)), 1), s.size) - 1])
    return {
        "jobs": n, "completed": len(done), "rejected": int(st["rejected"]), "ticks": ticks,
        "p50_latency_s": pct(0.50), "p99_latency_s": pct(0.99),
        "mean_latency_s": float(lat.mean()) if lat.size else None,
        "aggregate_point_stage_updates_per_s": work / span if span > 0 else None,
        "point_stage_updates": work, "span_s": span, "busy_s": st["busy"],
        "peak_bytes": int(st["bytes_peak"]),
        "p50_latency_s_by_grid": {k: pct_of(v, 0.50) for k, v in sorted(by_grid.items())},
        "p99_latency_s_by_grid": {k: pct_of(v, 0.99) for k, v in sorted(by_grid.items())},
        "jobs_by_grid": {k: len(v) for k, v in sorted(by_grid.items())},
    }


def main():
    import workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=256)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--t-scale", type=float, default=1e-3)
    ap.add_argument("--prec", type=int, default=0)
    ap.add_argument("--budget", type=float, default=200e9)
    ap.add_argument("--cowling-frac", type=float, default=0.0,
                    help="fraction of jobs on the fixed Kerr-Schild background")
    args = ap.parse_args()
    jobs = workloads.served_stream(args.jobs, args.rate, t_scale=args.t_scale, cowling_frac=args.cowling_frac)
    out = run_stream(jobs, prec=args.prec, budget=args.budget, log=lambda m: print(m, flush=True))
    out.update(rate=args.rate, t_scale=args.t_scale, prec=args.prec)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
