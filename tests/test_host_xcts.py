"""The library's XCTS solver (csrc/xcts.hip, with csrc/operators.cpp for its
grid) built with g++ against a host stand-in for the HIP runtime
(tests/host/hip_shim: blocks one after another, the threads of a block on a
pool of host threads that meet at __syncthreads) and run on the CPU under
AddressSanitizer and UndefinedBehaviorSanitizer.  The same kernel source, the
same host operators and the same iteration as on the GPU, compared with the
oracle's direct collocation solve (oracle/xcts.py) on the cases of the GPU
parity test, with the exact Plummer-like conformal factor, and on a
non-finite source.  This checks the algorithm and every memory access of
the kernels on the host; it is not GPU parity (the device entry point is
switched off in the library)."""

import os
import subprocess

import numpy as np
import pytest

from xcts_case import boundary_guess, manufactured

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2508_18221_amd", "csrc")

R_IN, R_OUT = 1.8, 20.0


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("xcts")
    exe = str(d / "xcts_harness")
    cmd = ["g++", "-O1", "-g", "-std=c++20", "-pthread", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-w",
           "-I", os.path.join(HERE, "host", "hip_shim"), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-x", "c++", os.path.join(CSRC, "xcts.hip"), "-x", "c++", os.path.join(CSRC, "operators.cpp"),
           "-x", "c++", os.path.join(HERE, "host", "xcts_harness.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    return exe, d


def host_solve(harness, shape, th0, E, guess, max_iter=200):
    exe, d = harness
    src, out = d / "in.bin", d / "out.bin"
    src.write_bytes(np.ascontiguousarray(E, dtype=np.float64).tobytes() +
                    np.ascontiguousarray(guess, dtype=np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, *map(str, shape), str(R_IN), str(R_OUT), str(th0), str(np.pi - th0), str(max_iter),
                        str(src), str(out)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    b = out.read_bytes()
    rc, it = np.frombuffer(b[:8], np.int32)
    ch = np.frombuffer(b[8:16], np.float64)[0]
    psi = np.frombuffer(b[16:], np.float64).reshape(E.shape)
    return int(rc), int(it), float(ch), psi


@pytest.mark.parametrize("shape,case", [((12, 10, 4), {}), ((16, 14, 8), dict(c=(2.0, 0.0, 0.0), w=4.0)),
                                        ((20, 18, 12), dict(c=(2.0, 0.0, 0.0), w=4.0)),
                                        ((15, 13, 6), dict(c=(0.0, 1.0, 3.0), w=3.0))])
def test_host_build_matches_oracle(harness, shape, case):
    from oracle import spectral, xcts
    g = spectral.Grid(*shape, R_IN, R_OUT, 0.05, np.pi - 0.05)
    psi_x, E = manufactured(g.R, g.TH, g.PH, **case)
    guess = boundary_guess(psi_x)
    ref, it_ref, _ = xcts.solve(g, E, guess)
    rc, it, ch, got = host_solve(harness, shape, 0.05, E, guess)
    assert rc == 0 and np.isfinite(got).all() and ch <= 1e-11
    assert abs(it - it_ref) <= 1
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    # Dirichlet data kept on the r ends and the theta ends
    assert np.array_equal(got[:, :, 0], guess[:, :, 0]) and np.array_equal(got[:, :, -1], guess[:, :, -1])
    assert np.array_equal(got[:, 0, :], guess[:, 0, :]) and np.array_equal(got[:, -1, :], guess[:, -1, :])


def test_host_build_recovers_the_exact_solution(harness):
    """32 x 28 x 4, the mass on the axis: the exact conformal factor to
    spectral accuracy (3e-10 here; 4e-12 at 40 x 36)."""
    from oracle import spectral
    shape = (32, 28, 4)
    g = spectral.Grid(*shape, R_IN, R_OUT, 0.05, np.pi - 0.05)
    psi_x, E = manufactured(g.R, g.TH, g.PH)
    rc, it, ch, got = host_solve(harness, shape, 0.05, E, boundary_guess(psi_x))
    assert rc == 0 and ch <= 1e-11
    assert np.abs(got - psi_x).max() < 1e-8


def test_host_build_stops_on_a_nonfinite_source(harness):
    shape = (12, 10, 4)
    E = np.zeros(shape[::-1])
    E[1, 4, 5] = np.nan
    rc, it, ch, got = host_solve(harness, shape, 0.05, E, np.ones(shape[::-1]), max_iter=20)
    assert rc == 0 and np.isnan(ch) and it == 1
