"""The XCTS solver's host eigen-decomposition (csrc/eig.h: Householder
Hessenberg reduction, shifted QR, back substitution), built with g++ into a
small harness and checked on the CPU:

  * on the collocation operators it decomposes -- the radial operator of
    r^2 times the flat Laplacian on the log-mapped Chebyshev grid and, per
    Fourier mode m, the polar one, both on the interior nodes -- and on random
    matrices with a known real spectrum: A V = V diag(lam), V V^-1 = I, and
    the eigenvalues equal LAPACK's (numpy.linalg.eigvals);
  * a matrix with a complex eigenvalue pair is refused."""

import os
import subprocess

import numpy as np
import pytest

from oracle import spectral

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2508_18221_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("eig")
    exe = str(d / "eig_harness")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "host", "eig_harness.cpp"),
                           "-o", exe])
    return exe, d


def decompose(harness, A):
    exe, d = harness
    n = A.shape[0]
    src, out = d / "A.bin", d / "out.bin"
    src.write_bytes(np.int32(n).tobytes() + np.ascontiguousarray(A, dtype=np.float64).tobytes())
    subprocess.check_call([exe, str(src), str(out)], stderr=subprocess.DEVNULL)
    b = out.read_bytes()
    if np.frombuffer(b[:4], np.int32)[0] != 1:
        return None
    v = np.frombuffer(b[4:], np.float64)
    return v[:n], v[n:n + n * n].reshape(n, n), v[n + n * n:].reshape(n, n)


def check(A, res):
    lam, V, Vi = res
    n = A.shape[0]
    scale = np.abs(A).max()
    assert np.abs(A @ V - V * lam).max() < 1e-10 * scale
    assert np.abs(V @ Vi - np.eye(n)).max() < 1e-10
    ref = np.sort(np.linalg.eigvals(A).real)
    assert np.abs(np.sort(lam) - ref).max() < 1e-10 * np.abs(ref).max()


def dmat(n, m):
    I = np.eye(n)
    return np.array([spectral.cheb_deriv(I[:, k][None, :], -1, m)[0] for k in range(n)]).T


@pytest.mark.parametrize("n", [5, 12, 40, 96])
def test_collocation_operators(harness, n):
    Lh, Th = 0.5 * np.log(20.0 / 1.8), 0.5 * (np.pi - 0.1)
    D1, D2 = dmat(n, 1), dmat(n, 2)
    A = ((D2 + Lh * D1) / Lh ** 2)[1:-1, 1:-1]
    check(A, decompose(harness, A))
    th = 0.5 * np.pi + Th * spectral.cgl_nodes(n)
    for m in sorted({0, 1, 3, n // 2}):
        B = (D2 / Th ** 2 + np.diag(1 / np.tan(th)) @ D1 / Th - np.diag(m * m / np.sin(th) ** 2))[1:-1, 1:-1]
        res = decompose(harness, B)
        check(B, res)
        assert (res[0] < 0).all()          # Dirichlet Laplacian pieces are negative definite here


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (30, 3)])
def test_known_real_spectrum(harness, n, seed):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(-10.0, 5.0, n))
    S = rng.standard_normal((n, n)) + n * np.eye(n)
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    res = decompose(harness, A)
    check(A, res)
    assert np.abs(np.sort(res[0]) - lam).max() < 1e-10 * np.abs(lam).max()


def test_complex_pair_is_refused(harness):
    A = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 2.0]])
    assert decompose(harness, A) is None
