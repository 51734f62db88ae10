"""Seeded input generators: exact planted gaps, Haar Q, Allen-Cahn operator."""
import numpy as np
import pytest

from paper_2605_24840_amd import inputs


@pytest.mark.parametrize("d,k,gap", [(64, 4, 0.1), (1024, 8, 0.02), (1024, 8, 0.002), (10, 1, 0.3),
                                     (10, 9, 0.3), (3, 1, 0.5)])
def test_planted_eigenvalues(d, k, gap):
    lam = inputs.planted_eigenvalues(d, k, gap, np.random.default_rng(0))
    assert lam.shape == (d,)
    assert np.all(np.diff(lam) >= 0)
    assert lam[k] - lam[k - 1] == pytest.approx(gap, abs=1e-15)
    assert lam[0] == -1.0 and lam[-1] == 1.0
    # Equal density on both sides of the gap.
    lo = -1.0 + (2.0 - gap) * (k - 1) / (d - 2)
    assert lam[k - 1] == pytest.approx(lo, abs=1e-15)


def test_haar_orthogonal_and_seeded():
    rng = np.random.default_rng(3)
    Q = inputs.haar_orthogonal(50, rng)
    assert np.abs(Q.T @ Q - np.eye(50)).max() < 1e-13
    Q2 = inputs.haar_orthogonal(50, np.random.default_rng(3))
    np.testing.assert_array_equal(Q, Q2)
    H1, _, _ = inputs.planted_hessian(40, 3, 0.1, 5)
    H2, _, _ = inputs.planted_hessian(40, 3, 0.1, 5)
    np.testing.assert_array_equal(H1, H2)
    np.testing.assert_array_equal(H1, H1.T)


def test_allen_cahn_2d_structure():
    n, eps = 16, 0.05
    H, u = inputs.allen_cahn_2d(n, eps, seed=1)
    d = n * n
    h = 1.0 / n
    c = eps * eps / (h * h)
    np.testing.assert_array_equal(H, H.T)
    assert np.max(np.abs(u)) == pytest.approx(1.0)
    np.testing.assert_allclose(np.diag(H), 4 * c + 3 * u.ravel() ** 2 - 1.0, rtol=0, atol=1e-14)
    off = H - np.diag(np.diag(H))
    assert np.all(np.sum(off != 0, axis=1) == 4)
    assert np.allclose(off[off != 0], -c)
    # ||-eps^2 Lap_h||_inf = 8 eps^2/h^2.
    Lap = H - np.diag(3 * u.ravel() ** 2 - 1.0)
    assert np.max(np.sum(np.abs(Lap), axis=1)) == pytest.approx(8 * c)
    # Periodic neighbours of grid point (0, 0).
    nb = set(np.nonzero(off[0])[0].tolist())
    assert nb == {1, n - 1, n, (n - 1) * n}
    # Same seed, same field.
    H2, u2 = inputs.allen_cahn_2d(n, eps, seed=1)
    np.testing.assert_array_equal(u, u2)


@pytest.mark.parametrize("d,k", [(300, 7), (50, 1), (97, 96)])
def test_planted_hessian_reflected(d, k):
    """The O(d^2) planted generator: H symmetric, its spectrum the planted
    one, and its lowest-k eigenspace spanned by the returned orthonormal Qk
    (LAPACK on the result)."""
    H, lam, Qk = inputs.planted_hessian_reflected(d, k, 0.1, 3)
    assert np.array_equal(H, H.T)
    w, V = np.linalg.eigh(H)
    np.testing.assert_allclose(w, lam, atol=1e-13)
    np.testing.assert_allclose(Qk.T @ Qk, np.eye(k), atol=1e-13)
    assert np.linalg.norm(V[:, :k] @ V[:, :k].T - Qk @ Qk.T) < 1e-12
