"""GPU parity of the block-Lanczos shift estimate (section 4.3 partial
eigensolver; Prop. 4.1 midpoint; Prop. 4.2 margin) through the C-ABI.

The library and the oracle build the same block Krylov space from the same
SplitMix64 start block (each side implements the generator) and stop by the
same rule at the same test steps.  They differ only in rounding: the QR of
each block (shifted Cholesky QR against Householder), the order of the
Gram-Schmidt sums, and how the Ritz values of the block tridiagonal matrix
are found (inertia bisection and inverse iteration against a dense
eigensolver).  Ritz values are well conditioned (a perturbation of size
delta of the basis moves them by O(delta ||H||)), so they are compared to
1e-9 ||H||; residual radii to 1e-6 relative plus 1e-12 ||H||.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2605_24840_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def R():
    from paper_2605_24840_amd import refl
    refl.load()
    return refl


@pytest.fixture(scope="module")
def handle(R):
    h = R.Handle(torch.device("cuda", 0))
    yield h
    h.close()


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _compare(dev, ora, hnorm):
    s, lk, lk1, eps, rho = dev
    assert abs(lk - ora["lam_k"]) <= 1e-9 * hnorm
    assert abs(lk1 - ora["lam_k1"]) <= 1e-9 * hnorm
    assert abs(s - ora["s"]) <= 1e-9 * hnorm
    assert abs(rho - ora["rho"]) <= 1e-9 * hnorm
    assert abs(eps - ora["eps"]) <= 1e-6 * ora["eps"] + 1e-12 * hnorm


@pytest.mark.parametrize("steps", [1, 2, 5, 0])
def test_lanczos_planted_ragged_matches_oracle(R, handle, steps):
    # d = 300 (not a multiple of any tile or block), k = 4, b = 8.
    d, k, seed = 300, 4, 3
    _say(f"lanczos planted d={d} k={k} steps={steps}")
    H, lam, _ = inputs.planted_hessian(d, k, 0.1, seed)
    hn = float(np.abs(H).sum(axis=1).max())
    ora = oracle.block_lanczos(H, k, max_steps=steps, seed=seed)
    *vals, st = R.estimate_shift(_gpu(H), k, steps=steps, seed=seed, handle=handle, check=False)
    _say(f"  status {R.STATUS[st]} lam_k {vals[1]:.12f} / {ora['lam_k']:.12f} eps {vals[3]:.3e} / {ora['eps']:.3e}")
    _compare(vals, ora, hn)
    ok, _, _ = oracle.admissible(ora["lam_k"], ora["lam_k1"], ora["eps"], ora["s"])
    assert st == (0 if ok else R.REFL_ERR_NOT_ADMISSIBLE)
    if steps == 0:
        assert ora["converged"]
        assert abs(vals[1] - lam[k - 1]) <= vals[3] and abs(vals[2] - lam[k]) <= vals[3]
        assert lam[k - 1] < vals[0] < lam[k]


@pytest.mark.parametrize("k", [14, 28])
def test_lanczos_wide_blocks_match_oracle(R, handle, k):
    # b = k + 4 = 18 and 32 (the cap): the block kernels' widest
    # instantiation (32 columns) in the projections and the Cholesky QR
    # rounds; d = 400 is ragged against the 256-row slabs.
    d, seed, steps = 400, 6, 3
    _say(f"lanczos wide blocks d={d} k={k} b={min(k + 4, 32)} steps={steps}")
    H, lam, _ = inputs.planted_hessian(d, k, 0.1, seed)
    hn = float(np.abs(H).sum(axis=1).max())
    ora = oracle.block_lanczos(H, k, max_steps=steps, seed=seed)
    *vals, st = R.estimate_shift(_gpu(H), k, steps=steps, seed=seed, handle=handle, check=False)
    _say(f"  status {R.STATUS[st]} lam_k {vals[1]:.12f} / {ora['lam_k']:.12f} eps {vals[3]:.3e} / {ora['eps']:.3e}")
    _compare(vals, ora, hn)


def test_lanczos_full_space_is_exact(R, handle):
    # d = 56, k = 3: b = 7, 8 steps span R^56; the Ritz values are the
    # eigenvalues and the residual radius is 0.
    d, k = 56, 3
    _say(f"lanczos full space d={d} k={k}")
    rng = np.random.default_rng(8)
    G = rng.standard_normal((d, d))
    H = 0.5 * (G + G.T)
    w, _, _ = oracle.jacobi_eigh(H)
    s, lk, lk1, eps, rho, st = R.estimate_shift(_gpu(H), k, seed=5, handle=handle)
    assert st == 0
    hn = float(np.abs(H).sum(axis=1).max())
    assert abs(lk - w[k - 1]) <= 1e-12 * hn and abs(lk1 - w[k]) <= 1e-12 * hn
    assert eps <= 1e-12 * hn
    assert abs(rho - max(w[-1] - s, s - w[0])) <= 1e-12 * hn


def test_lanczos_sign_steps_and_reflector(R, handle):
    # refl_sign with the estimated shift and the Lanczos scale (FP64): the
    # step count equals the oracle's, alpha = 1.05 rho_hat, R = R_k.
    d, k, seed = 300, 4, 3
    _say(f"lanczos + fp64 sign d={d} k={k} scale=lanczos")
    H, lam, Q = inputs.planted_hessian(d, k, 0.1, seed)
    ora = oracle.block_lanczos(H, k, seed=seed)
    Rg, info, st = R.sign(_gpu(H), k, None, handle=handle, precision="fp64", tol=1e-12, seed=seed,
                          scale="lanczos")
    assert st == 0
    assert info["lanczos_steps"] == ora["steps"]
    assert info["alpha"] == pytest.approx(1.05 * ora["rho"], rel=1e-9)
    assert info["margin"] > 0 and info["index_j"] == k
    Rk = np.eye(d) - 2.0 * Q[:, :k] @ Q[:, :k].T
    err = np.linalg.norm(Rg.cpu().numpy() - Rk)
    _say(f"  ||R - R_k||_F = {err:.2e}, steps {info['ns_steps']}")
    assert err < 1e-11


def test_lanczos_allen_cahn_d4096(R, handle):
    # The d = 4096 Allen-Cahn Hessian (k = 5): the device estimate equals the
    # oracle's, brackets the true endpoints within eps, and the mixed path run
    # with it meets ||R - R_k||_F <= 1e-8 sqrt(d).
    g = np.load(os.path.join(GOLDEN, "allen_cahn_n64_seed0.npz"))
    H, u = inputs.allen_cahn_2d(64, float(g["eps"]), 0)
    d, k = H.shape[0], 5
    _say(f"lanczos allen-cahn d={d} k={k}")
    w = g["w"]
    hn = float(np.abs(H).sum(axis=1).max())
    ora = oracle.block_lanczos(H, k, seed=0)
    Hg = _gpu(H)
    s, lk, lk1, eps, rho, st = R.estimate_shift(Hg, k, seed=0, handle=handle)
    _say(f"  lam_k {lk:.12f} / {ora['lam_k']:.12f}  lam_k1 {lk1:.12f} / {ora['lam_k1']:.12f}  "
         f"eps {eps:.3e} / {ora['eps']:.3e}")
    assert st == 0
    _compare((s, lk, lk1, eps, rho), ora, hn)
    assert abs(lk - w[k - 1]) <= eps and abs(lk1 - w[k]) <= eps and w[k - 1] < s < w[k]
    target = 1e-8 * np.sqrt(d)
    Rg, info, st = R.sign(Hg, k, None, handle=handle, precision="mixed", words=2, tol=target, seed=0)
    assert st == 0 and info["lanczos_steps"] == ora["steps"]
    Vk = g["V"][:, :k]
    E = Rg.cpu().numpy()
    E -= np.eye(d)
    E += 2.0 * Vk @ Vk.T
    err = float(np.linalg.norm(E))
    _say(f"  mixed with estimated shift: ||R - R_k||_F = {err:.2e} (target {target:.1e}), "
         f"setup {info['ms_setup']:.1f} ms")
    assert err <= target


def test_lanczos_error_paths(R, handle):
    _say("lanczos error paths")
    d = 40
    w = np.linspace(-1.0, 1.0, d)
    w[4] = w[3]                      # lambda_4 == lambda_5: no gap at k = 4
    *_, st = R.estimate_shift(_gpu(np.diag(w)), 4, seed=1, handle=handle, check=False)
    assert st == R.REFL_ERR_NO_GAP
    H = _gpu(np.diag(np.linspace(-1.0, 1.0, d)))
    for k in (0, d):
        *_, st = R.estimate_shift(H, k, handle=handle, check=False)
        assert st == R.REFL_ERR_INVALID_ARG
    p = R.make_params(3, 0.1, scale="lanczos")    # Lanczos scale needs the Lanczos shift
    size = R.refl_workspace_size
    with pytest.raises(R.ReflError):
        size(handle.h, d, p)
