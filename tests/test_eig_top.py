"""Host eigensolver of the Slepian window generator (csrc/eig_top.h), on the CPU.

The solver (Lanczos with complete reorthogonalisation, Sturm bisection, inverse
iteration) is built with g++ under the address and undefined-behaviour sanitizers and
run on matrices whose top eigenpair numpy's LAPACK routine fixes: random symmetric
matrices, concentration-like spectra clustered near 0 and 1, low-rank matrices (the
Krylov space turns invariant early and the process restarts), diagonal and
negative-definite matrices, a doubly degenerate top eigenvalue, and the real form of the
oracle's concentration matrix for the paper's region R_(pi/6, pi/6 + pi/240) at L_h = 18.
Non-finite input must be reported as failure."""
import math
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


@pytest.fixture(scope="module")
def solver(tmp_path_factory):
    exe = tmp_path_factory.mktemp("eig") / "eig_top_cli"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-Wall", "-Wextra", "-Werror",
                    os.path.join(HERE, "native", "eig_top_cli.cpp"), "-o", str(exe)], check=True)

    def run(A):
        A = np.ascontiguousarray(A, dtype=np.float64)
        n = A.shape[0]
        out = subprocess.run([str(exe)], input=struct.pack("<i", n) + A.tobytes(),
                             capture_output=True, timeout=120)
        if out.returncode == 3:
            return None
        assert out.returncode == 0, out.stderr.decode()
        v = np.frombuffer(out.stdout, dtype=np.float64)
        assert v.size == n + 1
        return float(v[0]), v[1:].copy()
    return run


def _check(A, res, gap_tol=1e-9):
    ev, V = np.linalg.eigh(A)
    lam, x = res
    scale = max(1.0, np.abs(ev).max())
    assert abs(lam - ev[-1]) <= 1e-12 * scale, (lam, ev[-1])
    assert abs(np.linalg.norm(x) - 1.0) <= 1e-13
    assert np.linalg.norm(A @ x - lam * x) <= 1e-11 * scale
    if len(ev) > 1 and ev[-1] - ev[-2] > 1e-3 * scale:
        v = V[:, -1]
        assert min(np.abs(x - v).max(), np.abs(x + v).max()) <= gap_tol


def _with_spectrum(rng, ev):
    Q, _ = np.linalg.qr(rng.standard_normal((len(ev), len(ev))))
    return (Q * ev) @ Q.T


@pytest.mark.parametrize("n", [1, 2, 3, 7, 40, 150])
def test_random_symmetric(solver, n):
    rng = np.random.default_rng(100 + n)
    B = rng.standard_normal((n, n))
    A = 0.5 * (B + B.T)
    _check(A, solver(A))


def test_concentration_like_spectrum(solver):
    """Eigenvalues clustered at 1 (a few) and at 0 (most), as for a Slepian block."""
    rng = np.random.default_rng(7)
    ev = np.concatenate([1.0 - 10.0 ** -rng.uniform(1, 6, 4), 0.5 * rng.uniform(size=5),
                         10.0 ** -rng.uniform(8, 16, 191)])
    A = _with_spectrum(rng, ev)
    _check(A, solver(A))


def test_low_rank_restarts(solver):
    """Rank 5 of 120: the Krylov space is invariant after 6 directions and the process
    restarts with fresh directions (zero off-diagonals in T)."""
    rng = np.random.default_rng(8)
    U = rng.standard_normal((120, 5))
    A = U @ np.diag([3.0, 2.0, 1.5, 1.0, 0.5]) @ U.T
    _check(A, solver(A))


def test_diagonal_and_negative_definite(solver):
    A = np.diag(np.arange(1.0, 31.0)[::-1])
    lam, x = solver(A)
    assert lam == pytest.approx(30.0, abs=1e-13) and abs(abs(x[0]) - 1.0) < 1e-13
    rng = np.random.default_rng(9)
    A = _with_spectrum(rng, -rng.uniform(1.0, 2.0, 25))
    _check(A, solver(A))


def test_zero_matrix_and_degenerate_top(solver):
    lam, x = solver(np.zeros((4, 4)))
    assert lam == 0.0 and np.linalg.norm(x) == pytest.approx(1.0)
    rng = np.random.default_rng(10)
    A = _with_spectrum(rng, np.array([2.0, 2.0, 1.0, 0.5, 0.25, 0.0]))
    lam, x = solver(A)
    assert lam == pytest.approx(2.0, abs=1e-13)
    assert np.linalg.norm(A @ x - lam * x) <= 1e-12


def test_non_finite_input_fails(solver):
    A = np.eye(5)
    A[2, 3] = A[3, 2] = math.nan
    assert solver(A) is None
    A[2, 3] = A[3, 2] = math.inf
    assert solver(A) is None


@pytest.mark.slow
def test_real_form_of_the_paper_region_matrix(solver):
    """The oracle's complex concentration matrix D for R_(pi/6, pi/6 + pi/240), L_h = 18,
    as the real symmetric [[Re D, -Im D], [Im D, Re D]]: every eigenvalue of D appears
    twice, so the top one is degenerate; its value is the window's concentration."""
    from oracle.slepian import concentration_matrix
    D = concentration_matrix(18, math.pi / 6, math.pi / 6 + math.pi / 240)
    R = np.block([[D.real, -D.imag], [D.imag, D.real]])
    R = 0.5 * (R + R.T)
    lam, x = solver(R)
    top = np.linalg.eigvalsh(D)[-1]
    assert abs(lam - top) <= 1e-13
    assert np.linalg.norm(R @ x - lam * x) <= 1e-12
