"""Oracle functions (TEST INFRASTRUCTURE ONLY; see the package docstring).

Everything is FP64 numpy or the plain C Jacobi solver in ``jacobi.c``.  Each
function names the passage of the paper it writes out.  A numpy matmul, sort
or ``eigvalsh`` on a tiny matrix serves as a library step where noted; there
is no blocking, fusion or reordering beyond the stated definitions.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_jacobi.so")
_lib = None

__all__ = [
    "jacobi_eigh", "oracle_threads", "reflector_from_eig", "reflector",
    "shifted_sign_from_eig", "midpoint", "ns_poly", "ns_scalar_error",
    "ns_error_recurrence", "ns_iterate", "ns_iterates", "ns_closed_form",
    "ns_depth_scalar", "inf_norm_shifted", "admissible", "certificates",
    "spectral_norm_sym",
]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_jacobi_eig.restype = ctypes.c_int
        lib.oracle_jacobi_eig.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def oracle_threads() -> int:
    """OpenMP threads the Jacobi solver uses (honours OMP_NUM_THREADS)."""
    return int(_load().oracle_num_threads())


def jacobi_eigh(H, max_sweeps: int = 60):
    """Full eigendecomposition H = V diag(w) V^T by cyclic Jacobi (jacobi.c).

    Returns ``(w, V, sweeps)`` with ``w`` ascending (the paper's ordering
    lambda_1 <= ... <= lambda_d, section 2.1) and V's columns the matching
    orthonormal eigenvectors.  H must be symmetric; it is not modified.
    """
    H = np.asarray(H, dtype=np.float64)
    d = H.shape[0]
    if H.shape != (d, d):
        raise ValueError("H must be square")
    A = np.ascontiguousarray(H.copy())
    w = np.empty(d, dtype=np.float64)
    V = np.empty((d, d), dtype=np.float64)
    sweeps = _load().oracle_jacobi_eig(d, A.ctypes.data, w.ctypes.data, V.ctypes.data, max_sweeps)
    if sweeps < 0:
        raise MemoryError("oracle_jacobi_eig failed")
    return w, V, int(sweeps)


def reflector_from_eig(V, k: int):
    """R_k = I - 2 P_k with P_k = Q_k Q_k^T (eq. Rk_intro, eq. Pk).

    Q_k is the first k columns of V (eigenvectors of the k smallest
    eigenvalues); k must lie in {1, ..., d-1} (section 2.1).
    """
    d = V.shape[0]
    if not (1 <= k <= d - 1):
        raise ValueError("k must lie in 1..d-1")
    Qk = V[:, :k]
    return np.eye(d) - 2.0 * (Qk @ Qk.T)


def reflector(H, k: int):
    """Exact prescribed-index reflector of H from the Jacobi eigensolver.

    Returns ``(R_k, w, V)``.
    """
    w, V, _ = jacobi_eigh(H)
    return reflector_from_eig(V, k), w, V


def shifted_sign_from_eig(w, V, s: float):
    """sgn(H - sI) by the spectral functional calculus (proof of Prop. 2.1).

    Returns ``(S, j)`` where j is the number of eigenvalues below s.  Raises
    if s equals an eigenvalue (the sign is undefined there).
    """
    a = np.asarray(w) - s
    if np.any(a == 0.0):
        raise ValueError("s is an eigenvalue: sgn(H - sI) undefined")
    sg = np.sign(a)
    return (V * sg) @ V.T, int(np.sum(a < 0))


def midpoint(w, k: int) -> float:
    """Midpoint shift s* = (lambda_k + lambda_{k+1})/2 (Prop. 4.1, eq. midpoint)."""
    return 0.5 * (float(w[k - 1]) + float(w[k]))


def ns_poly(t, m: int):
    """Scalar Newton-Schulz polynomial p_m(t) (eq. pm): p_0 = t,
    p_{m+1} = p_m (3 - p_m^2) / 2."""
    p = np.asarray(t, dtype=np.float64)
    for _ in range(m):
        p = 0.5 * p * (3.0 - p * p)
    return p


def ns_scalar_error(gamma, m: int):
    """eps_m(gamma) = 1 - p_m(gamma) (Prop. 3.6)."""
    return 1.0 - ns_poly(gamma, m)


def ns_error_recurrence(eps0, m: int):
    """eps_{m+1} = eps_m^2 (3 - eps_m) / 2 (eq. ns_scalar_recurrence)."""
    e = np.asarray(eps0, dtype=np.float64)
    for _ in range(m):
        e = 0.5 * e * e * (3.0 - e)
    return e


def ns_iterate(X):
    """One Newton-Schulz step X <- X (3I - X^2) / 2 (eq. NS), FP64."""
    d = X.shape[0]
    return 0.5 * (X @ (3.0 * np.eye(d) - X @ X))


def ns_iterates(H, s: float, alpha_norm: float, m: int):
    """X_0, ..., X_m of eq. NS with X_0 = (H - sI)/alpha_norm, FP64.

    The paper writes X_0 = alpha A with alpha = 1/norm; ``alpha_norm`` is the
    norm itself.
    """
    d = H.shape[0]
    X = (np.asarray(H, dtype=np.float64) - s * np.eye(d)) / alpha_norm
    out = [X]
    for _ in range(m):
        X = ns_iterate(X)
        out.append(X)
    return out


def ns_closed_form(w, V, s: float, alpha_norm: float, m: int):
    """X_m = Q diag(p_m((lambda_i - s)/alpha_norm)) Q^T: the iterate of eq. NS
    written through the spectral calculus (proof of Prop. 3.2)."""
    p = ns_poly((np.asarray(w) - s) / alpha_norm, m)
    return (V * p) @ V.T


def ns_depth_scalar(mu, tol: float, max_steps: int = 500) -> int:
    """Smallest m with ||p_m(A)^2 - I||_F < tol for a symmetric A whose
    eigenvalues are ``mu`` (already scaled): sqrt(sum (p_m(mu)^2 - 1)^2)."""
    t = np.asarray(mu, dtype=np.float64)
    for m in range(max_steps + 1):
        if np.sqrt(np.sum((t * t - 1.0) ** 2)) < tol:
            return m
        t = 0.5 * t * (3.0 - t * t)
    return max_steps + 1


def inf_norm_shifted(H, s: float) -> float:
    """||H - sI||_inf: the maximum absolute row sum (section 4.3, the cheap
    scaling surrogate)."""
    A = np.asarray(H, dtype=np.float64) - s * np.eye(H.shape[0])
    return float(np.max(np.sum(np.abs(A), axis=1)))


def admissible(lam_k_hat: float, lam_k1_hat: float, eps: float, s: float):
    """Prop. 4.2: with |lam_hat - lam| <= eps at both gap endpoints, the shift
    s is admissible if m_hat = min(s - lam_k_hat, lam_k1_hat - s) > eps.

    Returns ``(ok, m_hat, certified_margin)`` with margin m_hat - eps.
    """
    m_hat = min(s - lam_k_hat, lam_k1_hat - s)
    return bool(m_hat > eps), m_hat, m_hat - eps


def spectral_norm_sym(A) -> float:
    """||A||_2 of a symmetric matrix: the largest |eigenvalue| (proof of
    Prop. 3.2).  Library step: LAPACK eigvalsh."""
    return float(np.max(np.abs(np.linalg.eigvalsh(0.5 * (A + A.T)))))


def certificates(H, X, s: float):
    """Reference values of the quantities the library certifies, FP64:
    trace(X), ||X^2 - I||_F, and the commutator ||H X - X H||_F."""
    d = H.shape[0]
    T = X @ X
    C = H @ X - X @ H
    return {
        "trace": float(np.trace(X)),
        "resid_fro": float(np.linalg.norm(T - np.eye(d))),
        "commutator_fro": float(np.linalg.norm(C)),
    }
