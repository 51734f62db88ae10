"""Host-side linear algebra of the driver (csrc/hostla.cpp), built with g++
for the CPU and checked against LAPACK (numpy) on random and structured
band matrices: the band-to-tridiagonal reduction preserves the spectrum,
bisection returns the requested eigenvalue, and inverse iteration returns an
eigenvector with a small residual."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2605_24840_amd", "csrc", "hostla.cpp")

SHIM = r"""
#include "hostla.h"
extern "C" {
void t_band_tridiag(int n, int bw, const double* Lb, double* d, double* e) { refl::band_tridiag(n, bw, Lb, d, e); }
double t_eigval(int n, const double* d, const double* e, int m) { return refl::tridiag_eigval(n, d, e, m); }
int t_count(int n, const double* d, const double* e, double x) { return refl::tridiag_count_below(n, d, e, x); }
double t_invit(int n, int bw, const double* Lb, double s, int it, double* y) { return refl::band_inverse_iteration(n, bw, Lb, s, it, y); }
int t_eig(int n, const double* A, double* w, double* Q) { return refl::sym_eig_small(n, A, w, Q); }
int t_bcount(int n, int bw, const double* Lb, double x, double* work) { return refl::band_count_below(n, bw, Lb, x, work); }
void t_ritz(int j, int b, int k, const double* TA, const double* TB, int extremes, double* out, const double* prev) {
  refl::RitzCheck rc, pv;
  if (prev) { pv.th_k = prev[0]; pv.th_k1 = prev[1]; pv.res_k = prev[2]; pv.res_k1 = prev[3]; }
  refl::ritz_check(j, b, k, TA, TB, extremes != 0, rc, prev ? &pv : nullptr);
  out[0] = rc.th_k; out[1] = rc.th_k1; out[2] = rc.res_k; out[3] = rc.res_k1; out[4] = rc.th_min; out[5] = rc.th_max;
}
int t_ritzvec(int j, int b, const double* TA, const double* TB, int nvec, double* Y) { return refl::ritz_vectors(j, b, TA, TB, nvec, Y); }
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("hostla")
    shim = d / "shim.cpp"
    shim.write_text(SHIM)
    so = d / "libhostla_test.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", os.path.dirname(SRC),
                    SRC, str(shim), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    L.t_band_tridiag.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
    L.t_eigval.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
    L.t_eigval.restype = ctypes.c_double
    L.t_count.argtypes = [ctypes.c_int, P, P, ctypes.c_double]
    L.t_invit.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_double, ctypes.c_int, P]
    L.t_invit.restype = ctypes.c_double
    L.t_eig.argtypes = [ctypes.c_int, P, P, P]
    L.t_ritz.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int, P, P]
    L.t_ritzvec.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int, P]
    return L


def band_matrix(n, bw, rng, upper_tri_blocks=False):
    A = rng.standard_normal((n, n))
    A = 0.5 * (A + A.T)
    i, j = np.indices((n, n))
    A[np.abs(i - j) > bw] = 0.0
    return A


def lower_band(A, bw):
    n = A.shape[0]
    Lb = np.zeros((n, bw + 1))
    for i in range(n):
        for t in range(min(bw, i) + 1):
            Lb[i, t] = A[i, i - t]
    return np.ascontiguousarray(Lb)


def ptr(a):
    return a.ctypes.data


@pytest.mark.parametrize("n,bw", [(1, 0), (2, 1), (5, 1), (12, 3), (40, 9), (97, 16), (130, 32)])
def test_band_tridiag_preserves_spectrum(lib, n, bw):
    rng = np.random.default_rng(n * 100 + bw)
    A = band_matrix(n, bw, rng)
    Lb = lower_band(A, bw)
    dg, e = np.zeros(n), np.zeros(max(n - 1, 1))
    lib.t_band_tridiag(n, bw, ptr(Lb), ptr(dg), ptr(e))
    T = np.diag(dg) + np.diag(e[:n - 1], -1) + np.diag(e[:n - 1], 1)
    w = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(np.linalg.eigvalsh(T), w, atol=1e-12 * max(1, np.abs(w).max()))
    for m in sorted({0, n // 2, n - 1}):
        assert abs(lib.t_eigval(n, ptr(dg), ptr(e), m) - w[m]) <= 1e-12 * max(1, np.abs(w).max())
    x = 0.5 * (w[0] + w[-1]) if n > 1 else w[0] + 1.0
    assert lib.t_count(n, ptr(dg), ptr(e), x) == int(np.sum(w < x))


def test_block_tridiagonal_with_upper_triangular_coupling(lib):
    # The shape the Lanczos run produces: symmetric diagonal blocks, upper
    # triangular sub-diagonal blocks, half-bandwidth b.
    rng = np.random.default_rng(7)
    b, J = 6, 9
    n = b * J
    T = np.zeros((n, n))
    for i in range(J):
        A = rng.standard_normal((b, b))
        T[i * b:(i + 1) * b, i * b:(i + 1) * b] = A + A.T
        if i + 1 < J:
            B = np.triu(rng.standard_normal((b, b)))
            T[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = B
            T[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = B.T
    Lb = lower_band(T, b)
    dg, e = np.zeros(n), np.zeros(n - 1)
    lib.t_band_tridiag(n, b, ptr(Lb), ptr(dg), ptr(e))
    w = np.linalg.eigvalsh(T)
    for m in range(n):
        assert abs(lib.t_eigval(n, ptr(dg), ptr(e), m) - w[m]) <= 1e-11 * np.abs(w).max()


@pytest.mark.parametrize("m", [0, 3, 20])
def test_inverse_iteration_eigenvector(lib, m):
    rng = np.random.default_rng(11)
    n, bw = 60, 5
    A = band_matrix(n, bw, rng)
    w, Q = np.linalg.eigh(A)
    Lb = lower_band(A, bw)
    y = np.zeros(n)
    res = lib.t_invit(n, bw, ptr(Lb), w[m], 3, ptr(y))
    assert abs(np.linalg.norm(y) - 1.0) < 1e-12
    assert res < 1e-10 * np.abs(w).max()
    np.testing.assert_allclose(abs(y @ Q[:, m]), 1.0, atol=1e-9)
    np.testing.assert_allclose(res, np.linalg.norm(A @ y - w[m] * y), rtol=1e-6, atol=1e-14)


def test_sym_eig_small_matches_lapack(lib):
    rng = np.random.default_rng(2)
    n = 20
    A = rng.standard_normal((n, n))
    A = np.ascontiguousarray(A + A.T)
    w, Q = np.zeros(n), np.zeros((n, n))
    assert lib.t_eig(n, ptr(A), ptr(w), ptr(Q)) == 0
    np.testing.assert_allclose(w, np.linalg.eigvalsh(A), atol=1e-12)
    np.testing.assert_allclose(Q.T @ A @ Q, np.diag(w), atol=1e-11)


def test_band_inertia_count(lib):
    lib.t_bcount.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    rng = np.random.default_rng(4)
    ok = tot = 0
    for n, bw in ((30, 3), (90, 9), (64, 16)):
        A = band_matrix(n, bw, rng)
        w = np.linalg.eigvalsh(A)
        Lb = lower_band(A, bw)
        work = np.zeros(n * (bw + 1))
        for x in list(0.5 * (w[1:] + w[:-1])) + [w[0] - 1.0, w[-1] + 1.0]:
            c = lib.t_bcount(n, bw, ptr(Lb), x, ptr(work))
            assert c == -1 or c == int(np.sum(w < x))
            ok += c >= 0
            tot += 1
    assert ok >= 0.9 * tot     # growth (a declined count) is rare on random band matrices


def _lanczos_blocks(b, J, seed):
    """Blocks of a block tridiagonal T: A_i symmetric, B_i upper triangular
    with a positive diagonal (column-major b x b, as the Lanczos run stores
    them), from a diagonal matrix with a cluster and a gap so that the Ritz
    values near the gap converge within J steps."""
    rng = np.random.default_rng(seed)
    TA = np.zeros((J, b, b))
    TB = np.zeros((J, b, b))
    for i in range(J):
        A = 0.05 * rng.standard_normal((b, b))
        TA[i] = A + A.T + np.diag(np.sin(0.7 * i + np.arange(b)) * 4.0)
        B = np.triu(0.02 * rng.standard_normal((b, b)))
        B[np.diag_indices(b)] = 0.05 + 0.01 * rng.random(b)
        TB[i] = B
    # Column-major storage: element (r, c) at r + c b.
    return (np.ascontiguousarray(TA.transpose(0, 2, 1)), np.ascontiguousarray(TB.transpose(0, 2, 1)))


def _dense_T(TA, TB, j, b):
    n = j * b
    T = np.zeros((n, n))
    for i in range(j):
        T[i * b:(i + 1) * b, i * b:(i + 1) * b] = TA[i].T
        if i > 0:
            B = TB[i - 1].T          # B_{i-1}[r, c], r <= c
            T[i * b:(i + 1) * b, (i - 1) * b:i * b] = B
            T[(i - 1) * b:i * b, i * b:(i + 1) * b] = B.T
    return T


def test_ritz_check_against_lapack(lib):
    """Ritz values of T_j against LAPACK, and the residual radius: for the
    unit Ritz vector y of T_j, ||H x - theta x|| = ||B_j y_last|| (the coupling
    to the next block) -- computed here from the dense T_{j+1}."""
    b, J, k = 4, 14, 3
    TA, TB = _lanczos_blocks(b, J + 1, 3)
    out = np.zeros(6)
    for j in (1, 2, 5, 9, 14):
        lib.t_ritz(j, b, k, ptr(TA), ptr(TB), 1, ptr(out), None)
        T = _dense_T(TA, TB, j, b)
        w, Y = np.linalg.eigh(T)
        scale = np.abs(w).max()
        assert abs(out[0] - w[k - 1]) <= 1e-9 * scale and abs(out[1] - w[k]) <= 1e-9 * scale
        assert abs(out[4] - w[0]) <= 1e-9 * scale and abs(out[5] - w[-1]) <= 1e-9 * scale
        Bj = TB[j - 1].T
        for col, r in ((k - 1, out[2]), (k, out[3])):
            want = np.linalg.norm(Bj @ Y[-b:, col])
            # ||(T_j - theta) y|| adds rounding of order 1e-15 scale to the radius.
            assert abs(r - want) <= 1e-7 * want + 1e-13 * scale, (j, col, r, want)


def test_ritz_check_warm_start_matches_cold(lib):
    """Chained checks that start from the previous check's values give the
    same Ritz values as checks from the Gershgorin bounds, also when the
    guess is wrong (a deliberately displaced previous value)."""
    b, J, k = 5, 30, 4
    TA, TB = _lanczos_blocks(b, J + 1, 8)
    cold, warm = np.zeros(6), np.zeros(6)
    prev = None
    for j in range(1, J + 1, 3):
        lib.t_ritz(j, b, k, ptr(TA), ptr(TB), 0, ptr(cold), None)
        lib.t_ritz(j, b, k, ptr(TA), ptr(TB), 0, ptr(warm), None if prev is None else ptr(prev))
        scale = np.abs(np.linalg.eigvalsh(_dense_T(TA, TB, j, b))).max()
        assert abs(cold[0] - warm[0]) <= 1e-9 * scale and abs(cold[1] - warm[1]) <= 1e-9 * scale
        # Residual radii: a warm start near convergence takes shifted inverse
        # iteration from the previous value instead of a bisection; both give
        # the radius of the same Ritz pair.
        assert np.all(np.abs(cold[2:4] - warm[2:4]) <= 1e-6 * cold[2:4] + 1e-10 * scale), (j, cold, warm)
        prev = np.array(warm[:4])
    bad = np.array([warm[0] + 3.0, warm[1] - 2.0, 1e-14, 1e-14])
    lib.t_ritz(J, b, k, ptr(TA), ptr(TB), 0, ptr(warm), ptr(bad))
    lib.t_ritz(J, b, k, ptr(TA), ptr(TB), 0, ptr(cold), None)
    assert abs(cold[0] - warm[0]) <= 1e-9 * scale and abs(cold[1] - warm[1]) <= 1e-9 * scale


@pytest.mark.parametrize("j,b,nvec", [(1, 4, 4), (6, 5, 9), (20, 9, 9)])
def test_ritz_vectors_against_lapack(lib, j, b, nvec):
    """The nvec lowest Ritz pairs of T_j: orthonormal vectors, T y = theta y,
    and the values of LAPACK."""
    TA, TB = _lanczos_blocks(b, j + 1, 20 + j)
    n = j * b
    Y = np.zeros((nvec, n))                       # column-major n x nvec
    assert lib.t_ritzvec(j, b, ptr(TA), ptr(TB), nvec, ptr(Y)) == 0
    Y = Y.T
    T = _dense_T(TA, TB, j, b)
    w = np.linalg.eigvalsh(T)
    scale = np.abs(w).max()
    np.testing.assert_allclose(Y.T @ Y, np.eye(nvec), atol=1e-10)
    th = np.einsum("ij,ij->j", Y, T @ Y)
    np.testing.assert_allclose(th, w[:nvec], atol=1e-9 * scale)
    assert np.linalg.norm(T @ Y - Y * th) <= 1e-8 * scale


def test_ritz_vectors_repeated_eigenvalue(lib):
    """Uncoupled identical blocks give eigenvalues of multiplicity j: the
    vectors still come out orthonormal and span the lowest eigenspace."""
    b, j = 3, 4
    A = np.array([[2.0, 0.5, 0.0], [0.5, 1.0, 0.2], [0.0, 0.2, 3.0]])
    TA = np.ascontiguousarray(np.repeat(A.T[None], j + 1, axis=0))
    TB = np.zeros((j + 1, b, b))
    n = j * b
    nvec = j                                     # exactly the lowest eigenspace
    Y = np.zeros((nvec, n))
    assert lib.t_ritzvec(j, b, ptr(TA), ptr(TB), nvec, ptr(Y)) == 0
    Y = Y.T
    T = _dense_T(TA, TB, j, b)
    w, V = np.linalg.eigh(T)
    np.testing.assert_allclose(Y.T @ Y, np.eye(nvec), atol=1e-10)
    P = V[:, :nvec] @ V[:, :nvec].T
    assert np.linalg.norm(P @ Y - Y) <= 1e-8
