"""Writes <workload>_<steps>steps.json: the oracle's state after `steps` RK4
steps (CFL 0.25, filter on) of a workload, at a fixed set of sampled grid
points, plus the whole-field L2 norms.

Calls only the oracle and the seeded workload definitions.  Run from the
repository root (tens of minutes of CPU at full size):

    python tests/golden/make_oracle_samples.py ks_michel_64x64x128 10
    python tests/golden/make_oracle_samples.py ks_torus_128x96x192 10

An optional third argument runs a paper-literal variant of the workload and
names the file <workload>_<variant>_<steps>steps.json: split (the
operator-split coupled step), dealias (2/3 truncation after every step) or
damped (the damped primitive recovery):

    python tests/golden/make_oracle_samples.py ks_michel_64x64x128 4 split
"""

VARIANTS = {"split": ({}, {"split": True}), "dealias": ({"dealias": True}, {}), "damped": ({}, {"c2p": "damped"})}

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import evolve, spectral  # noqa: E402


def sample_points(nph, nth, nr, seed=7, n_random=256):
    """(phi, theta, r) indices: seeded uniform interior points plus points on
    and next to every boundary (r_out j = 0, r_in j = nr - 1, theta ends)."""
    rng = np.random.default_rng(seed)
    pts = set()
    while len(pts) < n_random:
        pts.add((int(rng.integers(nph)), int(rng.integers(nth)), int(rng.integers(nr))))
    for j in (0, 1, nr // 2, nr - 2, nr - 1):
        for k in (0, 1, nth // 2, nth - 2, nth - 1):
            for l in (0, nph // 4, nph // 2 + 1):
                pts.add((l, k, j))
    return sorted(pts)


def main(name, steps, variant=None):
    tag = f"{name}_{variant}" if variant else name
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{tag}_{steps}steps.json")
    w = workloads.WORKLOADS[name]
    if variant:
        gk, pk_extra = VARIANTS[variant]
        w = dict(grid=dict(w["grid"], **gk), phys=dict(w["phys"], **pk_extra), steps=w["steps"])
    ga, pk, ik = workloads.oracle_kwargs(w)
    g = spectral.Grid(*ga)
    pb = evolve.Problem(g, **pk)
    U, K0, _ = evolve.initial_state(g, pb, **ik)
    dt = pb.dt()
    t0 = time.time()
    for n in range(steps):
        U = pb.step(U, K0, dt)
        print(f"step {n + 1}/{steps}  {time.time() - t0:.0f} s", flush=True)
    pts = sample_points(*U.shape[1:])
    idx = tuple(np.array(pts).T)
    vals = U[(slice(None),) + idx].T  # (npoints, 32)
    with open(out, "w") as f:
        json.dump({"workload": name, "variant": variant, "steps": steps, "dt": dt, "shape": list(U.shape),
                   "points": pts, "values": [[float.hex(float(v)) for v in row] for row in vals],
                   "field_norms_full": [float(np.sqrt(np.sum(U[q] ** 2))) for q in range(U.shape[0])]},
                  f, separators=(",", ":"))
    print(f"wrote {out}: {len(pts)} points")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), sys.argv[3] if len(sys.argv) > 3 else None)
