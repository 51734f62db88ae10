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
    "jacobi_eigh", "oracle_threads", "set_oracle_threads", "reflector_from_eig", "reflector",
    "shifted_sign_from_eig", "midpoint", "ns_poly", "ns_scalar_error",
    "ns_error_recurrence", "ns_iterate", "ns_iterates", "ns_closed_form",
    "ns_depth_scalar", "bf16_round", "split_words", "word_product", "ns_step_words", "ns_iterates_words",
    "inf_norm_shifted", "fro_norm_shifted", "admissible", "certificates",
    "spectral_norm_sym", "splitmix64", "start_block", "lanczos_block_size",
    "lanczos_check_steps", "block_lanczos", "ns_step_derivative", "ns_adjoint", "ns_tangent",
    "ns_poly_derivative", "ns_frechet_dk", "sign_frechet_dk", "policy_step", "outer_descent",
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
        lib.oracle_set_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def oracle_threads() -> int:
    """OpenMP threads the Jacobi solver uses (honours OMP_NUM_THREADS)."""
    return int(_load().oracle_num_threads())


def set_oracle_threads(n: int) -> int:
    """Threads of the following Jacobi solves; returns the number in force."""
    return int(_load().oracle_set_threads(int(n)))


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



# ------------------------------------------- split-BF16 bulk arithmetic model
def bf16_round(x):
    """Round FP32 values to the nearest BF16 value, ties to the even
    significand (8 significant bits: 1 implicit + 7 stored), returned as
    FP32.  Written from the definition: x = f 2^e with f in [0.5, 1), keep
    f 2^8 rounded half-to-even (numpy rint), scale back."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    f, e = np.frexp(x)
    return np.ldexp(np.rint(f * 256.0) / 256.0, e).astype(np.float32)


def split_words(x, words: int):
    """The BF16 words of FP32 values (design reading of the bulk storage):
    w_0 = bf16(x), w_i = bf16(x - w_0 - ... - w_{i-1}); every remainder is
    exact in FP32.  Returns a list of FP32 arrays."""
    r = np.asarray(x, dtype=np.float32)
    out = []
    for _ in range(words):
        w = bf16_round(r)
        out.append(w)
        r = (r - w).astype(np.float32)
    return out


def word_product(Aw, Bw, mirror: bool = False):
    """The split-word product: the sum of the word products A_a B_b whose
    weight 2^-8(a + b) is at least 2^-8(W - 1) (W = 2: three products,
    "bf16x3"; W = 3: six, "bf16x6"; Henry, Tang and Heinecke, ARITH 2019),
    formed in FP64 and rounded once to FP32 (the model of an FP32
    accumulation without its intermediate roundings).  With ``mirror`` the
    product of two commuting symmetric matrices is taken from its upper
    triangle (i <= j) and mirrored, as the library stores it (reading R3)."""
    W = len(Aw)
    acc = np.zeros((Aw[0].shape[0], Bw[0].shape[1]))
    for a in range(W):
        for b in range(W - a):
            acc += Aw[a].astype(np.float64) @ Bw[b].astype(np.float64)
    if mirror:
        acc = np.triu(acc) + np.triu(acc, 1).T
    return acc.astype(np.float32)


def _word_total(ws):
    t = ws[0].copy()
    for w in ws[1:]:
        t = (t + w).astype(np.float32)
    return t


def ns_step_words(X, words: int):
    """One step of eq. NS in the split-BF16 bulk arithmetic from the iterate
    X (values exactly representable in FP32, e.g. a word sum): Xw = the words
    of fl32(X); T = word_product(Xw, Xw), N = words of fl32(I - T),
    P = word_product(Xw, N), X_new = words of fl32(fl32(sum of Xw) + P/2).
    Both products keep their upper triangle, mirrored (reading R3).  Only the
    order of the FP32 accumulation inside a product is not modelled.
    Returns the word sum of X_new as FP64."""
    X32 = np.asarray(X, dtype=np.float64).astype(np.float32)
    d = X32.shape[0]
    Xw = split_words(X32, words)
    T = word_product(Xw, Xw, mirror=True)
    Nw = split_words((np.eye(d, dtype=np.float32) - T).astype(np.float32), words)
    P = word_product(Xw, Nw, mirror=True)
    Xn = (_word_total(Xw) + (np.float32(0.5) * P).astype(np.float32)).astype(np.float32)
    return _word_total(split_words(Xn, words)).astype(np.float64)


def ns_iterates_words(H, s: float, alpha_norm: float, m: int, words: int):
    """X_0, ..., X_m of eq. NS in the split-BF16 bulk arithmetic (FP64
    arrays of the word sums): X_0 = the word sum of fl32((H - sI)/alpha),
    then ``ns_step_words`` m times."""
    d = H.shape[0]
    A = ((np.asarray(H, dtype=np.float64) - s * np.eye(d)) / alpha_norm).astype(np.float32)
    X = _word_total(split_words(A, words)).astype(np.float64)
    out = [X]
    for _ in range(m):
        X = ns_step_words(X, words)
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


# ------------------------------------------------------------ derivatives
# Differentiation of the finite-step reflector X_m(H) = p_m((H - sI)/alpha)
# with s and alpha held fixed (the shift and scale are chosen from spectral
# estimates, not differentiated through).  Three independent formulations:
# reverse accumulation over the steps of eq. NS, forward tangents, and the
# Daleckii-Krein divided-difference form of the derivative of a matrix
# function.


def ns_step_derivative(X, E):
    """Derivative of f(X) = X (3I - X^2)/2 (eq. NS) at X in direction E, by
    the product rule: (3E - (E X^2 + X E X + X^2 E))/2.  For symmetric X this
    linear map is self-adjoint in the Frobenius inner product."""
    X = np.asarray(X, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    X2 = X @ X
    return 0.5 * (3.0 * E - (E @ X2 + X @ E @ X + X2 @ E))


def ns_adjoint(H, s: float, alpha_norm: float, m: int, G):
    """Gradient of L(H) = <G, X_m(H)> over symmetric perturbations of H:
    Gbar_m = (G + G^T)/2, Gbar_j = Df(X_j)*[Gbar_{j+1}] = Df(X_j)[Gbar_{j+1}],
    gradient = Gbar_0 / alpha_norm (X_0 = (H - sI)/alpha_norm)."""
    Xs = ns_iterates(H, s, alpha_norm, m)
    G = np.asarray(G, dtype=np.float64)
    Gb = 0.5 * (G + G.T)
    for j in range(m - 1, -1, -1):
        Gb = ns_step_derivative(Xs[j], Gb)
    return Gb / alpha_norm


def ns_tangent(H, s: float, alpha_norm: float, m: int, E):
    """Directional derivative D X_m(H)[E] by forward tangents:
    Xdot_0 = E/alpha_norm, Xdot_{j+1} = Df(X_j)[Xdot_j]."""
    Xs = ns_iterates(H, s, alpha_norm, m)
    T = np.asarray(E, dtype=np.float64) / alpha_norm
    for j in range(m):
        T = ns_step_derivative(Xs[j], T)
    return T


def ns_poly_derivative(t, m: int):
    """p_m'(t) by the chain rule on eq. pm: p_0' = 1,
    p_{j+1}' = p_j' (3 - 3 p_j^2)/2."""
    p = np.asarray(t, dtype=np.float64)
    dp = np.ones_like(p)
    for _ in range(m):
        dp = dp * 1.5 * (1.0 - p * p)
        p = 0.5 * p * (3.0 - p * p)
    return dp


def _dk(w, V, phi, dphi, E):
    """Daleckii-Krein: D phi(A)[E] = V (F o (V^T E V)) V^T for A = V diag(w) V^T,
    F_ij = (phi_i - phi_j)/(w_i - w_j) (phi'_i where w_i = w_j)."""
    dw = w[:, None] - w[None, :]
    same = np.abs(dw) <= 1e-13 * max(1.0, float(np.max(np.abs(w))))
    F = np.where(same, 0.5 * (dphi[:, None] + dphi[None, :]),
                 (phi[:, None] - phi[None, :]) / np.where(same, 1.0, dw))
    B = V.T @ np.asarray(E, dtype=np.float64) @ V
    return V @ (F * B) @ V.T


def ns_frechet_dk(H, s: float, alpha_norm: float, m: int, E):
    """D X_m(H)[E] in Daleckii-Krein form with phi(x) = p_m((x - s)/alpha_norm)
    on the eigenvalues of H (eigendecomposition by LAPACK)."""
    Hs = np.asarray(H, dtype=np.float64)
    w, V = np.linalg.eigh(0.5 * (Hs + Hs.T))
    t = (w - s) / alpha_norm
    return _dk(w, V, ns_poly(t, m), ns_poly_derivative(t, m) / alpha_norm, E)


def sign_frechet_dk(H, s: float, E):
    """The limit m -> infinity: D sgn(H - sI)[E] with F_ij = 2/|a_i - a_j| when
    a_i = lambda_i - s and a_j have opposite signs, else 0."""
    Hs = np.asarray(H, dtype=np.float64)
    w, V = np.linalg.eigh(0.5 * (Hs + Hs.T))
    a = w - s
    opp = np.sign(a)[:, None] != np.sign(a)[None, :]
    F = np.where(opp, 2.0 / np.where(opp, np.abs(a[:, None] - a[None, :]), 1.0), 0.0)
    B = V.T @ np.asarray(E, dtype=np.float64) @ V
    return V @ (F * B) @ V.T


# ---------------------------------------------------------- shift policies
def policy_step(mode: str, state, estimate, drift=None, beta: float = 0.5, clip: float = 0.25,
                tau: float = 0.5):
    """One call of a shift policy of Alg. 4.3 (step 4) over a sequence of
    Hessians, with the certificates of Prop. 4.2.

    ``state`` is None or a dict with the shift in force ``s`` and the
    estimates of the last refresh ``lam_k``, ``lam_k1``, ``eps``.
    ``estimate()`` returns (lam_k_hat, lam_k1_hat, eps) for the current H and
    is called only when the policy refreshes.  ``drift`` is a bound on
    ||H - H_ref||_2 (H_ref the Hessian of the last refresh), used by 'reuse'.

    * 'midpoint': refresh every call, s = (lam_k_hat + lam_k1_hat)/2 (Prop. 4.1).
    * 'damped': refresh every call, s = (1 - beta) s_prev + beta * midpoint,
      clipped into [lam_k_hat + eps + clip w, lam_k1_hat - eps - clip w] with
      w = (lam_k1_hat - lam_k_hat)/2 - eps (midpoint on the first call).
    * 'reuse': keep s while min(s - lam_k, lam_k1 - s) - eps - drift exceeds
      tau (lam_k1 - lam_k)/2 (Prop. 4.2, second statement, with Weyl's bound),
      else refresh to the midpoint.

    Returns dict(s, margin, refreshed, state); margin is the certified lower
    bound on the distance from s to the true gap endpoints, and state is None
    when the shift is not certified (margin <= 0)."""
    if mode == "reuse" and state is not None:
        margin = min(state["s"] - state["lam_k"], state["lam_k1"] - state["s"]) - state["eps"] - drift
        if margin > tau * 0.5 * (state["lam_k1"] - state["lam_k"]):
            return {"s": state["s"], "margin": margin, "refreshed": False, "state": dict(state)}
    lk, lk1, eps = estimate()
    s = 0.5 * (lk + lk1)
    w = 0.5 * (lk1 - lk) - eps
    if mode == "damped" and state is not None and w > 0.0:
        raw = (1.0 - beta) * state["s"] + beta * s
        s = min(max(raw, lk + eps + clip * w), lk1 - eps - clip * w)
    margin = min(s - lk, lk1 - s) - eps
    new = {"s": s, "lam_k": lk, "lam_k1": lk1, "eps": eps} if margin > 0.0 else None
    return {"s": s, "margin": margin, "refreshed": True, "state": new}


def outer_descent(grad, hess, x0, k: int, eta: float, steps: int, shifts=None, m: int = 0,
                  gtol: float = 1e-10, similarity=None):
    """Alg. 4.3 with an exact engine: x_{n+1} = x_n - eta R_n g_n
    (eq. discrete_step).  R_n is the exact reflector R_k of H_n (m = 0) or the
    finite filter p_m((H_n - s_n I)/||H_n - s_n I||_inf) (eq. pm, section 4.3
    scaling), with s_n = shifts[n] when given, else the exact midpoint of
    H_n's eigenvalues (Prop. 4.1).  ``similarity`` as in the library driver:
    hess returns S H S^-1 and the direction is S^-1 R(S H S^-1) S g.
    Returns dict(x, steps, gnorm, shifts, xs)."""
    x = np.array(x0, dtype=np.float64)
    gn_hist, s_hist, xs = [], [], [x.copy()]
    n = 0
    for n in range(steps):
        g = grad(x)
        gn_hist.append(float(np.linalg.norm(g)))
        if gn_hist[-1] < gtol:
            break
        H = hess(x)
        w, V = np.linalg.eigh(H)
        s = shifts[n] if shifts is not None else midpoint(w, k)
        s_hist.append(s)
        if m == 0:
            R, _ = shifted_sign_from_eig(w, V, s)
        else:
            R = ns_iterates(H, s, inf_norm_shifted(H, s), m)[m]
        v = g if similarity is None else similarity * g
        dvec = R @ v
        if similarity is not None:
            dvec = dvec / similarity
        x = x - eta * dvec
        xs.append(x.copy())
    else:
        gn_hist.append(float(np.linalg.norm(grad(x))))
    return {"x": x, "steps": len(s_hist), "gnorm": gn_hist, "shifts": s_hist, "xs": xs}


def fro_norm_shifted(H, s: float) -> float:
    """||H - sI||_F, another cheap upper bound on the spectral radius of
    H - sI (an alternative to the section 4.3 surrogates)."""
    A = np.asarray(H, dtype=np.float64) - s * np.eye(H.shape[0])
    return float(np.sqrt(np.sum(A * A)))


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


# ---------------------------------------------------------------------------
# Shift estimation: block Lanczos for the gap endpoints (section 4.3)
# ---------------------------------------------------------------------------
_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(x):
    """SplitMix64 output from state x (Steele, Lea and Flood, "Fast splittable
    pseudorandom number generators", OOPSLA 2014): z = x + 0x9E3779B97F4A7C15,
    then the two xor-shift-multiply rounds and a final xor-shift.  uint64
    arithmetic wraps modulo 2^64."""
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _SM_GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def start_block(d: int, nb: int, seed: int):
    """The seeded start block of the Lanczos run: entry (row, c) is
    splitmix64(seed * 0x100000001B3 + c * d + row) mapped to (-1, 1) through
    its top 53 bits (u = top53 * 2^-53, value 2u - 1)."""
    rows = np.arange(d, dtype=np.uint64)[:, None]
    cols = np.arange(nb, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        ctr = np.uint64(seed) * np.uint64(0x100000001B3) + cols * np.uint64(d) + rows
    u = (splitmix64(ctr) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return 2.0 * u - 1.0


def lanczos_block_size(d: int, k: int) -> int:
    """Block width b = min(k + 4, 32, d) (a few guard vectors beyond the k + 1
    wanted Ritz values; the paper leaves the partial eigensolver open)."""
    return int(min(k + 4, 32, d))


def lanczos_check_steps(d: int, k: int, b: int, max_steps: int = 0):
    """Steps after which the convergence test runs: j0 = ceil((k+1)/b), then
    every ceil(64/b) steps, and always at the cap J (max_steps, or floor(d/b)
    when 0 or larger than that)."""
    cap = d // b
    J = cap if max_steps <= 0 else min(max_steps, cap)
    j0 = max(1, -(-(k + 1) // b))
    ci = max(1, -(-64 // b))
    out = list(range(j0, J + 1, ci))
    if not out or out[-1] != J:
        out.append(J)
    return [j for j in out if j <= J]


def block_lanczos(H, k: int, max_steps: int = 0, seed: int = 0):
    """Estimates of lambda_k, lambda_{k+1}, the error radius eps, the midpoint
    shift and the spectral radius of H - sI by block Lanczos with full
    reorthogonalisation (the partial-eigensolver route of section 4.3; the
    estimates feed Prop. 4.1 and the admissibility test of Prop. 4.2).

    Steps, in order: Q_1 = orthonormal basis of the start block (library QR);
    for j = 1, 2, ...: W = H Q_j, A_j = Q_j^T W, W <- W - V (V^T W) twice
    with V = [Q_1 .. Q_j], Q_{j+1} B_j = W (library QR; B_j = 0 once the
    basis spans the whole space).  At the steps of ``lanczos_check_steps``
    the block tridiagonal T_j (diagonal blocks A_i, sub-diagonal blocks B_i)
    is diagonalised (library eigh): Ritz values theta, and residual norms
    ||H x_i - theta_i x_i|| = ||B_j y_i(last block)||, each a radius that
    holds an eigenvalue of H.  Converged when eps = max(res_k, res_{k+1}) <
    (theta_{k+1} - theta_k)/4.  Returns a dict with the estimates, the step
    of the last test, and whether it converged.
    """
    H = np.asarray(H, dtype=np.float64)
    d = H.shape[0]
    if not (1 <= k <= d - 1):
        raise ValueError("k must lie in 1..d-1")
    b = lanczos_block_size(d, k)
    checks = set(lanczos_check_steps(d, k, b, max_steps))
    J = max(checks)
    Q, _ = np.linalg.qr(start_block(d, b, seed))
    blocks = [Q]
    A_list, B_list = [], []
    res = None
    for j in range(1, J + 1):
        Qj = blocks[-1]
        W = H @ Qj
        A_list.append(0.5 * (Qj.T @ W + (Qj.T @ W).T))
        V = np.hstack(blocks)
        for _ in range(2):
            W = W - V @ (V.T @ W)
        if j * b >= d:
            Bj = np.zeros((b, b))
            Qn = np.zeros((d, b))
        else:
            Qn, Bj = np.linalg.qr(W)
        B_list.append(Bj)
        blocks.append(Qn)
        if j in checks:
            n = j * b
            T = np.zeros((n, n))
            for i in range(j):
                T[i * b:(i + 1) * b, i * b:(i + 1) * b] = A_list[i]
                if i + 1 < j:
                    T[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = B_list[i]
                    T[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = B_list[i].T
            theta, Y = np.linalg.eigh(T)
            res = np.linalg.norm(B_list[-1] @ Y[-b:, :], axis=0)
            lk, lk1 = float(theta[k - 1]), float(theta[k])
            eps = float(max(res[k - 1], res[k]))
            converged = eps < 0.25 * (lk1 - lk)
            if converged or j == J:
                s = 0.5 * (lk + lk1)
                rho = float(max(theta[-1] - s, s - theta[0]))
                return {"lam_k": lk, "lam_k1": lk1, "eps": eps, "s": s, "rho": rho,
                        "steps": j, "b": b, "converged": bool(converged),
                        "theta": theta, "res": res, "basis": np.hstack(blocks[:-1])}
    raise AssertionError("unreachable: the cap is always a check step")
