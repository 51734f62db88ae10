"""The controlled-spectra grid (d = 1024, k = 8; relative gaps 1e-1, 1e-2,
1e-3, i.e. absolute gaps 2e-1, 2e-2, 2e-3; shifts at theta = 0.1, 0.5, 0.9 of
the gap, section 5.1) through the C-ABI, in FP64 and FP32.

FP64: converged to ||X^2 - I||_F < 1e-10; the error against the exact R_k
(from the generator's Q) is at rounding level, and the depth equals the one
the scalar model of Prop. 3.6 predicts from the exact eigenvalues
(eigenwise, ||X_m^2 - I||_F = sqrt(sum_i (p_m(t_i)^2 - 1)^2)), within one
step where rounding meets the threshold.

FP32: the iterate stops at its rounding floor.  Products in FP32 perturb the
scaled matrix by about u32 sqrt(d) per step (u32 = 2^-24, norms of the scaled
iterates about 1), and a perturbation E of the scaled matrix moves the
reflector by at most 2 sqrt(2) ||E||_F / gamma with gamma the scaled half-gap
(Davis-Kahan), so err <= C u32 sqrt(d) / gamma with a constant C for the
number of products and their growth.  The measured ratios on this grid are
at most 0.32 (theta = 0.1 at the widest gap); C = 4 keeps a 12x margin.  The
index certificate must hold.
"""
import numpy as np
import pytest

import oracle
from paper_2605_24840_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


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


@pytest.fixture(scope="module")
def planted():
    cache = {}

    def get(grel, seed=0):
        key = (grel, seed)
        if key not in cache:
            cache[key] = inputs.planted_hessian(1024, 8, 2 * grel, seed)
        return cache[key]
    return get


GRID = [(g, t) for g in (1e-1, 1e-2, 1e-3) for t in (0.1, 0.5, 0.9)]


@pytest.mark.parametrize("grel,theta", GRID)
def test_c1_fp64(R, handle, planted, grel, theta):
    d, k, tol = 1024, 8, 1e-10
    H, lam, Q = planted(grel)
    s = lam[k - 1] + theta * (lam[k] - lam[k - 1])
    _say(f"fp64 d={d} k={k} grel={grel} theta={theta}")
    Hg = torch.from_numpy(H).to("cuda:0")
    Rg, info, st = R.sign(Hg, k, s, handle=handle, precision="fp64", tol=tol, check=False)
    Rk = np.eye(d) - 2.0 * Q[:, :k] @ Q[:, :k].T
    err = float(np.linalg.norm(Rg.cpu().numpy() - Rk))
    alpha = oracle.inf_norm_shifted(H, s)
    m_pred = oracle.ns_depth_scalar((lam - s) / alpha, tol)
    _say(f"  status={R.STATUS[st]} steps={info['ns_steps']} predicted={m_pred} ||R-R_k||_F={err:.2e}")
    assert st == 0 and info["index_j"] == k
    assert abs(info["ns_steps"] - m_pred) <= 1
    assert err < 1e-9


@pytest.mark.parametrize("grel,theta", GRID)
def test_c1_fp32(R, handle, planted, grel, theta):
    d, k = 1024, 8
    H, lam, Q = planted(grel)
    s = lam[k - 1] + theta * (lam[k] - lam[k - 1])
    _say(f"fp32 d={d} k={k} grel={grel} theta={theta}")
    Hg = torch.from_numpy(H).to("cuda:0")
    Rg, info, st = R.sign(Hg, k, s, handle=handle, precision="fp32", tol=1e-3, check=False)
    Rk = np.eye(d) - 2.0 * Q[:, :k] @ Q[:, :k].T
    err = float(np.linalg.norm(Rg.cpu().numpy() - Rk))
    alpha = oracle.inf_norm_shifted(H, s)
    gamma = min(s - lam[k - 1], lam[k] - s) / alpha
    bound = U32 * np.sqrt(d) / gamma
    _say(f"  status={R.STATUS[st]} steps={info['ns_steps']} ||R-R_k||_F={err:.2e} err/(u32 sqrt(d)/gamma)={err / bound:.2f}")
    assert info["index_j"] == k
    assert err <= 4 * bound


def test_e1_radius_grown_at_fixed_gap(R, handle):
    """Section 5.1 (ii): the spectral radius grows (r = 1, 4, 16) at a fixed
    absolute gap 0.02 (d = 512, k = 8, midpoint shift).  The scaled half-gap
    shrinks like 1/r, so the FP64 depth grows by about log_1.5(4) per
    factor 4; it equals the scalar model's depth on the exact eigenvalues
    (within one step), and the reflector stays exact to rounding."""
    d, k, g, tol = 512, 8, 0.02, 1e-10
    rng = np.random.default_rng(90)
    Q = inputs.haar_orthogonal(d, rng)
    depths = []
    for r in (1.0, 4.0, 16.0):
        lam = r * inputs.planted_eigenvalues(d, k, g / r, np.random.default_rng(91))
        H = (Q * lam) @ Q.T
        H = 0.5 * (H + H.T)
        s = 0.5 * (lam[k - 1] + lam[k])
        Rg, info, st = R.sign(torch.from_numpy(H).to("cuda:0"), k, s, handle=handle, precision="fp64",
                              tol=tol, check=False)
        err = float(np.linalg.norm(Rg.cpu().numpy() - (np.eye(d) - 2.0 * Q[:, :k] @ Q[:, :k].T)))
        m_pred = oracle.ns_depth_scalar((lam - s) / oracle.inf_norm_shifted(H, s), tol)
        _say(f"radius {r:g}: steps={info['ns_steps']} predicted={m_pred} alpha={info['alpha']:.3f} "
             f"||R-R_k||_F={err:.2e}")
        assert st == 0 and info["index_j"] == k
        assert abs(info["ns_steps"] - m_pred) <= 1 and err < 1e-9
        depths.append(info["ns_steps"])
    assert depths[0] < depths[1] < depths[2]
    assert all(2 <= b - a <= 5 for a, b in zip(depths, depths[1:]))
