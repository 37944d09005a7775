"""Helpers for the GPU parity tests: build the library path and the oracle on
the same seeded workload, and compare them field by field.

Per-field error (relative, per tensor group):  e_f = max|f_gpu - f_oracle| /
max(max|f_oracle|, s_g), where s_g is the largest magnitude over the field's
tensor group (phi | gt | At | K | Gt and the driver Bd | alpha | beta |
D | S_j | tau | B^i) of the reference array."""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

GROUPS = [[0], list(range(1, 7)), list(range(7, 13)), [13], [14, 15, 16, 21, 22, 23], [17],
          [18, 19, 20], [24], [25, 26, 27], [28], [29, 30, 31]]


def groups_for(n):
    """Tensor groups of an n-field state (psi, field 32, alone)."""
    return GROUPS + [[32]] if n > 32 else GROUPS


def field_errors(gpu, ref):
    """e_f for each field (arrays shaped (32 or 33, ...))."""
    e = np.zeros(ref.shape[0])
    for grp in groups_for(ref.shape[0]):
        sg = max(np.abs(ref[f]).max() for f in grp)
        for f in grp:
            den = max(np.abs(ref[f]).max(), sg)
            d = np.abs(gpu[f] - ref[f]).max()
            e[f] = 0.0 if d == 0 else (d / den if den > 0 else np.inf)
    return e


def rhs_errors(gpu, ref, U):
    """Errors of one RHS evaluation: max|dU_gpu - dU_oracle| over a field,
    divided by the larger of the group's RHS magnitude and the group's state
    magnitude (time unit M = 1).  At t = 0 the RHS of a stationary field is
    pure truncation error (~0), so its own magnitude is no scale for
    round-off; the state magnitude is the rate that changes it by O(1) per
    unit time."""
    e = np.zeros(ref.shape[0])
    for grp in groups_for(ref.shape[0]):
        sg = max(max(np.abs(ref[f]).max(), np.abs(U[f]).max()) for f in grp)
        for f in grp:
            d = np.abs(gpu[f] - ref[f]).max()
            e[f] = 0.0 if d == 0 else d / sg
    return e


def workload(name, **grid_over):
    w = workloads.WORKLOADS[name]
    w = dict(grid=dict(w["grid"]), phys=dict(w["phys"]), steps=w["steps"])
    w["grid"].update(grid_over)
    return w


def oracle_problem(w):
    from oracle import spectral, evolve
    ga, pk, ik = workloads.oracle_kwargs(w)
    g = spectral.Grid(*ga)
    pb = evolve.Problem(g, **pk)
    U, K0, mat = evolve.initial_state(g, pb, **ik)
    return g, pb, U, K0


def solver(w):
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    return Solver(make_grid(**w["grid"]), make_phys(**w["phys"]))


def log(msg):
    print(msg, flush=True)
