"""Seeded synthetic inputs: planted-spectrum and Allen-Cahn Hessians.

This module only draws random numbers and assembles test matrices.  It holds
none of the reflector method's arithmetic and imports nothing else from this
package, so both the HIP path and the CPU oracle can take their inputs from it.

Readings of the paper that fix the recipes (the paper itself states no sizes
for these workloads):

* Planted spectrum with an absolute gap g between lambda_k and lambda_{k+1}
  inside [-1, 1]: with l = -1 + (2 - g)(k - 1)/(d - 2), set lambda_1 = -1,
  lambda_k = l, lambda_{k+1} = l + g, lambda_d = 1, the other lower values
  i.i.d. U(-1, l) and the other upper values i.i.d. U(l + g, 1).  The relative
  gap (lambda_{k+1} - lambda_k)/(lambda_d - lambda_1) is g/2.
* Haar orthogonal Q: QR of an N(0,1) matrix, columns sign-fixed so that the
  R factor has a positive diagonal.
* Allen-Cahn Hessian H = eps^2 (-Lap_h) + diag(3u^2 - 1) (section 5.4).  The
  2-D variant uses the 5-point periodic Laplacian on an n x n grid of the unit
  square (h = 1/n), grid point (i, j) -> index i*n + j, and a smooth field u
  made of 16 low-frequency sine modes normalised to max |u| = 1.  The domain
  length 1 is the one for which the paper's 1-D example (eps = 0.4, n = 41,
  ghost-point Neumann Laplacian) has an index-one zero state.
"""
import math

import numpy as np

__all__ = [
    "haar_orthogonal", "planted_eigenvalues", "planted_hessian",
    "allen_cahn_field", "allen_cahn_2d", "allen_cahn_1d_neumann",
    "symmetric_normal", "diag_hessian", "batch_specs", "batch_problem",
    "RotatedQuartic", "AllenCahn1D",
]


def haar_orthogonal(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal d x d matrix from a seeded generator."""
    Z = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(Z)
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn


def planted_eigenvalues(d: int, k: int, gap: float, rng: np.random.Generator) -> np.ndarray:
    """Ascending spectrum in [-1, 1] with lambda_{k+1} - lambda_k = gap exactly
    (for 2 <= k <= d-2 the extremes are exactly -1 and 1)."""
    if d < 3 or not (1 <= k <= d - 1):
        raise ValueError("need d >= 3 and 1 <= k <= d-1")
    if not (0.0 < gap < 2.0):
        raise ValueError("gap must lie in (0, 2)")
    lo = -1.0 + (2.0 - gap) * (k - 1) / (d - 2)
    hi = lo + gap
    lam = np.empty(d, dtype=np.float64)
    n_lo = k - 2 if k >= 2 else 0      # values strictly between -1 and lambda_k
    n_hi = (d - k) - 2 if k <= d - 2 else 0
    lower = np.sort(rng.uniform(-1.0, lo, size=n_lo))
    upper = np.sort(rng.uniform(hi, 1.0, size=n_hi))
    if k >= 2:
        lam[:k] = np.concatenate([[-1.0], lower, [lo]])
    else:
        lam[0] = lo                      # k = 1: lambda_1 = l = -1
    if k <= d - 2:
        lam[k:] = np.concatenate([[hi], upper, [1.0]])
    else:
        lam[k] = hi                      # k = d-1: lambda_d = l + g = 1
    return lam


def planted_hessian_reflected(d: int, k: int, gap: float, seed: int, nrefl: int = 3):
    """H = Q diag(lambda) Q^T with Q a product of nrefl Householder
    reflectors of seeded random unit vectors: a dense symmetric matrix with
    the planted spectrum of planted_eigenvalues, built in O(nrefl d^2) (for
    large orders, where a Haar Q costs O(d^3)).  Returns ``(H, lam, Qk)``
    with Qk the first k columns of Q."""
    rng = np.random.default_rng(seed)
    lam = planted_eigenvalues(d, k, gap, rng)
    us = []
    for _ in range(nrefl):
        u = rng.standard_normal(d)
        us.append(u / np.linalg.norm(u))
    # Q = P_1 ... P_n with P_i = I - 2 u_i u_i^T; H = Q diag(lam) Q^T is
    # formed inside out, one two-sided reflection at a time:
    # P A P = A - 2 u w^T - 2 w u^T + 4 (u.w) u u^T with w = A u.
    H = np.diag(lam)
    for u in reversed(us):
        w = H @ u
        c = 4.0 * float(u @ w)
        H -= np.outer(u, 2.0 * w - c * u)
        H -= np.outer(2.0 * w, u)
    H = 0.5 * (H + H.T)
    Qk = np.eye(d, k)
    for u in reversed(us):
        Qk -= 2.0 * np.outer(u, u @ Qk)
    return np.ascontiguousarray(H), lam, Qk


def planted_hessian(d: int, k: int, gap: float, seed: int):
    """H = Q diag(lambda) Q^T with Haar Q and a planted gap.

    Returns ``(H, lam, Q)``; H is symmetrised exactly ((M + M^T)/2), so its
    eigenvalues equal ``lam`` up to FP64 rounding of the product.
    """
    rng = np.random.default_rng(seed)
    lam = planted_eigenvalues(d, k, gap, rng)
    Q = haar_orthogonal(d, rng)
    M = (Q * lam) @ Q.T
    H = 0.5 * (M + M.T)
    return np.ascontiguousarray(H), lam, Q


def allen_cahn_field(n: int, seed: int, modes: int = 16, fmax: int = 4, L: float = 1.0) -> np.ndarray:
    """Smooth periodic field on the n x n grid x_i = i L/n:
    u = sum_j a_j sin(2 pi (m_j x + q_j y)/L + phi_j), normalised to max|u| = 1,
    with integer (m_j, q_j) uniform in [-fmax, fmax]^2 minus (0, 0),
    a_j ~ N(0, 1), phi_j ~ U[0, 2 pi).  Draw order per mode: m, q (redrawn
    together until nonzero), a, phi.  Uses math.sin so the field does not
    depend on numpy's vectorised libm."""
    rng = np.random.default_rng(seed)
    u = np.zeros((n, n), dtype=np.float64)
    for _ in range(modes):
        while True:
            m, q = (int(v) for v in rng.integers(-fmax, fmax + 1, size=2))
            if (m, q) != (0, 0):
                break
        a = float(rng.standard_normal())
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
        for i in range(n):
            x = i * L / n
            for j in range(n):
                y = j * L / n
                u[i, j] += a * math.sin(2.0 * math.pi * (m * x + q * y) / L + phi)
    return u / np.max(np.abs(u))


def allen_cahn_2d(n: int = 64, eps: float = 0.05, seed: int = 0, L: float = 1.0):
    """Dense Hessian of the 2-D periodic semidiscrete Allen-Cahn energy at the
    seeded field u: H = eps^2 (-Lap_h) + diag(3u^2 - 1), d = n^2.

    Returns ``(H, u)``.  Entries: diagonal 4 eps^2/h^2 + 3u_p^2 - 1, and
    -eps^2/h^2 for each of the four periodic neighbours.
    """
    if n < 3:
        raise ValueError("n must be >= 3")
    h = L / n
    u = allen_cahn_field(n, seed, L=L)
    d = n * n
    c = eps * eps / (h * h)
    H = np.zeros((d, d), dtype=np.float64)
    for i in range(n):
        for j in range(n):
            p = i * n + j
            H[p, p] = 4.0 * c + 3.0 * u[i, j] ** 2 - 1.0
            for (ii, jj) in (((i + 1) % n, j), ((i - 1) % n, j), (i, (j + 1) % n), (i, (j - 1) % n)):
                H[p, ii * n + jj] -= c
    return H, u


def allen_cahn_1d_neumann(n: int = 41, eps: float = 0.4, L: float = 1.0, u=None):
    """Hessian of the paper's 1-D Allen-Cahn energy (section 5.4) with the
    ghost-point Neumann Laplacian on n nodes, h = L/(n-1):
    H = eps^2 (-Lap_h) + diag(3u^2 - 1).  The ghost-point rows at both ends
    read (2u_0 - 2u_1)/h^2 for -Lap_h, which is made symmetric by the usual
    half-weight at the boundary nodes; here the symmetric form
    D^{-1/2} (-Lap_h) D^{1/2} with D = diag(1/2, 1, ..., 1, 1/2) is used, which
    has the same eigenvalues.  ``u`` defaults to the zero state."""
    h = L / (n - 1)
    u = np.zeros(n) if u is None else np.asarray(u, dtype=np.float64)
    K = np.zeros((n, n))
    for i in range(n):
        K[i, i] = 2.0
        if i > 0:
            K[i, i - 1] = -1.0
        if i < n - 1:
            K[i, i + 1] = -1.0
    K[0, 1] = -2.0
    K[n - 1, n - 2] = -2.0
    K /= h * h
    # Similarity transform to a symmetric matrix with the same spectrum.
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    S = np.sqrt(w)
    Ks = (S[:, None] * K) / S[None, :]
    Ks = 0.5 * (Ks + Ks.T)
    return eps * eps * Ks + np.diag(3.0 * u * u - 1.0)


def symmetric_normal(d: int, seed: int) -> np.ndarray:
    """G = (Z + Z^T)/2 with Z i.i.d. N(0,1), seeded."""
    Z = np.random.default_rng(seed).standard_normal((d, d))
    return 0.5 * (Z + Z.T)


def diag_hessian(d: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Diagonal H with distinct i.i.d. U(lo, hi) entries in random order."""
    rng = np.random.default_rng(seed)
    return np.diag(rng.uniform(lo, hi, size=d))


def batch_specs(n: int = 256, seed: int = 0, sizes=(128, 256, 512, 1024), kmax: int = 16,
                grel_range=(1e-3, 1e-1)):
    """Shapes of a batch of planted problems: a list of ``(d, k, grel, pseed)``
    with d uniform over ``sizes``, k uniform in 1..kmax, the relative gap grel
    log-uniform over ``grel_range`` (absolute gap 2 grel), and pseed the seed
    of problem p's matrix (seed * 65536 + p)."""
    rng = np.random.default_rng(seed)
    ds = rng.choice(np.asarray(sizes), size=n)
    ks = rng.integers(1, kmax + 1, size=n)
    lo, hi = math.log(grel_range[0]), math.log(grel_range[1])
    gs = np.exp(rng.uniform(lo, hi, size=n))
    return [(int(ds[p]), int(ks[p]), float(gs[p]), seed * 65536 + p) for p in range(n)]


def batch_problem(spec):
    """``planted_hessian`` of one ``batch_specs`` entry: ``(H, lam, Q)``."""
    d, k, grel, pseed = spec
    return planted_hessian(d, k, 2.0 * grel, pseed)


class RotatedQuartic:
    """The rotated quartic family of the target-index scan (section 5.3):
    E(x) = 1/4 sum y_i^4 + 1/2 sum c_i y_i^2 with y = Q^T x, Q Haar (seeded),
    c_i < 0 for i <= k and c_i > 0 otherwise, so the origin is an index-k
    saddle.  The paper does not state c; here c_i = -(1 + (i-1)/d) for i <= k
    and c_i = 1 + (i-1)/d for i > k (distinct curvatures)."""

    def __init__(self, d: int = 64, k: int = 4, seed: int = 0):
        rng = np.random.default_rng(seed)
        self.Q = haar_orthogonal(d, rng)
        i = np.arange(d)
        self.c = np.where(i < k, -(1.0 + i / d), 1.0 + i / d)
        self.d, self.k = d, k

    def energy(self, x):
        y = self.Q.T @ x
        return 0.25 * np.sum(y ** 4) + 0.5 * np.sum(self.c * y * y)

    def grad(self, x):
        y = self.Q.T @ x
        return self.Q @ (y ** 3 + self.c * y)

    def hess(self, x):
        y = self.Q.T @ x
        M = (self.Q * (3.0 * y * y + self.c)) @ self.Q.T
        return 0.5 * (M + M.T)

    def start(self, seed: int, scale: float = 0.3):
        """A seeded random start near the saddle."""
        return scale * np.random.default_rng(seed).standard_normal(self.d)


class AllenCahn1D:
    """The 1-D semidiscrete Allen-Cahn energy of section 5.4 on n nodes with
    the ghost-point Neumann Laplacian K (h = L/(n-1)):
    grad E = eps^2 K u + u^3 - u,  Hessian eps^2 K + diag(3u^2 - 1).
    K is not symmetric; with S = diag(sqrt(w)), w = (1/2, 1, ..., 1, 1/2),
    S K S^-1 is, and ``hess_sym`` returns S H S^-1 (same eigenvalues), so that
    sgn(H) = S^-1 sgn(S H S^-1) S."""

    def __init__(self, n: int = 41, eps: float = 0.4, L: float = 1.0):
        h = L / (n - 1)
        K = np.zeros((n, n))
        for i in range(n):
            K[i, i] = 2.0
            if i > 0:
                K[i, i - 1] = -1.0
            if i < n - 1:
                K[i, i + 1] = -1.0
        K[0, 1] = -2.0
        K[n - 1, n - 2] = -2.0
        self.K = K / (h * h)
        w = np.ones(n)
        w[0] = w[-1] = 0.5
        self.S = np.sqrt(w)
        self.n, self.eps = n, eps

    def grad(self, u):
        return self.eps ** 2 * (self.K @ u) + u ** 3 - u

    def hess_sym(self, u):
        Ks = (self.S[:, None] * self.K) / self.S[None, :]
        Ks = 0.5 * (Ks + Ks.T)
        return self.eps ** 2 * Ks + np.diag(3.0 * u * u - 1.0)

    def start(self, seed: int, scale: float = 0.05):
        return scale * np.random.default_rng(seed).standard_normal(self.n)
