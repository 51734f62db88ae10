"""Derivatives through the C-ABI (refl_sign_grad): the gradient of
L(H) = <G, R_m(H)> for the m-step reflector, s and alpha fixed.

Against the oracle (reverse accumulation, forward tangents and the
Daleckii-Krein form, pinned in the CPU suite):

* FP64, small and ragged d: the same recurrence in FP64 with other summation
  orders; the gradient agrees to 1e-11 relative (Frobenius), the loss and R
  to rounding.
* Checkpoint intervals recompute bit-identical iterates, so the gradient is
  the same bit for bit for every interval; forward tangents agree with the
  reverse sweep to rounding (self-adjointness).
* The differentiation workload (d = 2048, k = 10, gap 0.05, G symmetric
  N(0, 1), seed 0), FP64 to ||X^2 - I||_F < 1e-10: against the
  Daleckii-Krein gradient to 1e-9 relative, and the directional derivative
  against central differences of L along a unit symmetric direction E
  (t = 1e-4; the CPU sweep of t at d = 256 gives 7e-10) to 1e-6 relative.
* FP32: the derivative of the FP32 iteration.  Rounding of the products
  (u32 = 2^-24 per entry per step) perturbs the iterates by about u32 and the
  divided differences across the gap by about u32/gamma relative (gamma the
  scaled half-gap, min |lambda_i - s|/alpha); the test asserts
  err <= u32/gamma (measured: 0.1 u32/gamma).
"""
import numpy as np
import pytest

import oracle
from paper_2605_24840_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("d,k,m", [(100, 3, 8), (64, 4, 1), (200, 7, 12)])
def test_grad_fp64_matches_oracle(R, handle, d, k, m):
    _say(f"grad fp64 d={d} k={k} m={m}")
    H, lam, Q = inputs.planted_hessian(d, k, 0.1, d)
    s = 0.5 * (lam[k - 1] + lam[k])
    Gn = np.random.default_rng(d).standard_normal((d, d))   # not symmetric: only sym(G) counts
    alpha = oracle.inf_norm_shifted(H, s)
    want = oracle.ns_adjoint(H, s, alpha, m, Gn)
    Xm = oracle.ns_iterates(H, s, alpha, m)[m]
    for mode in ("reverse", "tangent"):
        g, loss, Rm, info, st = R.sign_grad(_gpu(H), _gpu(Gn), k, s, handle=handle, fixed_steps=m,
                                            grad_mode=mode, with_R=True)
        err = _rel(g.cpu().numpy(), want)
        lerr = abs(loss - np.sum(Gn * Xm)) / abs(np.sum(Gn * Xm))
        _say(f"  {mode}: status={R.STATUS[st]} steps={info['ns_steps']} grad rel={err:.2e} loss rel={lerr:.2e}")
        assert st == 0 and info["ns_steps"] == m
        assert err < 1e-11 and lerr < 1e-12
        assert np.max(np.abs(Rm.cpu().numpy() - Xm)) < 1e-13
        gn = g.cpu().numpy()
        assert np.array_equal(gn, gn.T)


def test_grad_checkpoint_intervals_bitwise(R, handle):
    d, k, m = 256, 5, 11
    H, lam, Q = inputs.planted_hessian(d, k, 0.05, 3)
    s = 0.5 * (lam[k - 1] + lam[k])
    G = _gpu(inputs.symmetric_normal(d, 4))
    Hg = _gpu(H)
    ref, _, _, _, _ = R.sign_grad(Hg, G, k, s, handle=handle, fixed_steps=m, ckpt_every=1)
    for c in (2, 3, 5, 11, 0):
        g, _, _, info, st = R.sign_grad(Hg, G, k, s, handle=handle, fixed_steps=m, ckpt_every=c)
        _say(f"  ckpt_every={c}: equal={torch.equal(g, ref)}")
        assert st == 0 and torch.equal(g, ref)
    t, _, _, _, _ = R.sign_grad(Hg, G, k, s, handle=handle, fixed_steps=m, grad_mode="tangent")
    err = float(torch.linalg.norm(t - ref) / torch.linalg.norm(ref))
    _say(f"  tangent vs reverse: {err:.2e}")
    assert err < 1e-12


def test_grad_tile_edges_bitwise(R, handle, monkeypatch):
    """The derivative products (-X Gbar over all tiles, the three-pair
    adjoint step over the upper tiles) give the same gradient bit for bit
    whichever FP64 tile edge runs: each entry is the same sum in the same
    order."""
    d, k, m = 200, 4, 7
    H, lam, Q = inputs.planted_hessian(d, k, 0.05, 5)
    s = 0.5 * (lam[k - 1] + lam[k])
    G = _gpu(inputs.symmetric_normal(d, 6))
    Hg = _gpu(H)
    out = {}
    for ts in (32, 64, 128):
        monkeypatch.setenv("REFL_F_TILE", str(ts))
        g, loss, _, info, st = R.sign_grad(Hg, G, k, s, handle=handle, fixed_steps=m)
        assert st == 0
        out[ts] = (g.clone(), loss)
    monkeypatch.delenv("REFL_F_TILE")
    _say(f"  grad tile edges 32/64/128 equal: {[torch.equal(out[32][0], out[t][0]) for t in (64, 128)]}")
    for ts in (64, 128):
        assert torch.equal(out[32][0], out[ts][0])


@pytest.fixture(scope="module")
def c4():
    d, k = 2048, 10
    H, lam, Q = inputs.planted_hessian(d, k, 0.05, 0)
    G = inputs.symmetric_normal(d, 0)
    s = 0.5 * (lam[k - 1] + lam[k])
    return H, lam, Q, G, s, k


def test_grad_differentiation_workload_fp64(R, handle, c4):
    H, lam, Q, G, s, k = c4
    d = H.shape[0]
    Hg, Gg = _gpu(H), _gpu(G)
    _say(f"grad fp64 d={d} k={k} converged")
    g, loss, _, info, st = R.sign_grad(Hg, Gg, k, s, handle=handle, tol=1e-10)
    m, alpha = info["ns_steps"], info["alpha"]
    _say(f"  status={R.STATUS[st]} steps={m} alpha={alpha:.6f} j={info['index_j']} ms={info['ms_total']:.1f}")
    assert st == 0 and info["index_j"] == k
    gn = g.cpu().numpy()
    dk = oracle.ns_frechet_dk(H, s, alpha, m, G)
    err = _rel(gn, dk)
    _say(f"  vs Daleckii-Krein (m={m}): {err:.2e}")
    assert err < 1e-9
    # Central differences along a unit symmetric direction, alpha and m fixed.
    E = inputs.symmetric_normal(d, 1)
    E /= np.linalg.norm(E)
    Eg = _gpu(E)
    t = 1e-4

    def L(Hx):
        Rx, inf2, st2 = R.sign(Hx, k, s, handle=handle, alpha=alpha, fixed_steps=m)
        assert st2 == 0
        return float((Gg * Rx).sum())
    fd = (L(Hg + t * Eg) - L(Hg - t * Eg)) / (2 * t)
    dd = float(np.sum(gn * E))
    _say(f"  directional derivative {dd:.12e}, central difference {fd:.12e}, rel {abs(dd - fd) / abs(fd):.2e}")
    assert abs(dd - fd) <= 1e-6 * abs(fd)


def test_grad_differentiation_workload_fp32(R, handle, c4):
    H, lam, Q, G, s, k = c4
    g, loss, _, info, st = R.sign_grad(_gpu(H), _gpu(G), k, s, handle=handle, precision="fp32",
                                       tol=1e-3)
    m, alpha = info["ns_steps"], info["alpha"]
    dk = oracle.ns_frechet_dk(H, s, alpha, m, G)
    err = _rel(g.cpu().numpy(), dk)
    gamma = min(s - lam[k - 1], lam[k] - s) / alpha
    bound = 2.0 ** -24 / gamma
    _say(f"grad fp32 d=2048: status={R.STATUS[st]} steps={m} vs Daleckii-Krein {err:.2e} "
         f"(u32/gamma = {bound:.2e})")
    assert info["index_j"] == k and err <= bound


def test_reflsign_autograd(R, handle):
    d, k = 96, 4
    H, lam, Q = inputs.planted_hessian(d, k, 0.2, 21)
    s = 0.5 * (lam[k - 1] + lam[k])
    Hg = _gpu(H).requires_grad_(True)
    G = _gpu(inputs.symmetric_normal(d, 22))
    Rk = R.ReflSign.apply(Hg, k, s, {"handle": handle, "fixed_steps": 9})
    (Rk * G).sum().backward()
    g, _, _, _, _ = R.sign_grad(Hg.detach(), G, k, s, handle=handle, fixed_steps=9)
    _say(f"autograd vs refl_sign_grad equal={torch.equal(Hg.grad, g)}")
    assert torch.equal(Hg.grad, g)


def test_grad_errors(R, handle):
    H, lam, Q = inputs.planted_hessian(64, 4, 0.1, 0)
    s = 0.5 * (lam[3] + lam[4])
    Hg, G = _gpu(H), _gpu(inputs.symmetric_normal(64, 0))
    for kw, want in ((dict(precision="mixed", fixed_steps=4), "REFL_ERR_UNSUPPORTED"),
                     (dict(ckpt_every=-1), "REFL_ERR_INVALID_ARG")):
        _, _, _, _, st = R.sign_grad(Hg, G, 4, s, handle=handle, check=False, **kw)
        assert R.STATUS[st] == want, kw
    _, _, _, _, st = R.sign_grad(Hg, G, 4, None, handle=handle, check=False)
    assert R.STATUS[st] == "REFL_ERR_UNSUPPORTED"


# --------------------------------------------- MIXED: gradient of the limit
def _limit_loss(H, G, k):
    """<G, R_k(H)> with R_k = I - 2 V_k V_k^T from LAPACK's eigenvectors (the
    definition, eq. Pk), as a reference for central differences."""
    w, V = np.linalg.eigh(H)
    Vk = V[:, :k]
    return float(np.trace(G) - 2.0 * np.sum(Vk * (G @ Vk)))


def test_grad_mixed_differentiation_workload(R, handle, c4):
    """MIXED forward (split-BF16 bulk, FP64 correction), then the gradient of
    the limit <G, sgn(H - sI)> from the certified eigenspace by projected
    FP64 solves.  Against the Daleckii-Krein form of D sgn (oracle) and central
    differences of <G, R_k(H + tE)> (R_k from LAPACK eigenvectors, t = 1e-4);
    target 1e-6 relative."""
    H, lam, Q, G, s, k = c4
    d = H.shape[0]
    Hg, Gg = _gpu(H), _gpu(G)
    g, loss, Rm, info, st = R.sign_grad(Hg, Gg, k, s, handle=handle, precision="mixed",
                                        tol=1e-8 * np.sqrt(d), with_R=True)
    _say(f"grad mixed d={d} k={k}: status={R.STATUS[st]} words={info['bulk_words']} steps={info['ns_steps']} "
         f"cg={info['cg_iters']} ms={info['ms_total']:.1f}")
    assert st == 0 and info["index_j"] == k
    gn = g.cpu().numpy()
    assert np.array_equal(gn, gn.T)
    dk = oracle.sign_frechet_dk(H, s, G)
    err = _rel(gn, dk)
    _say(f"  vs Daleckii-Krein of sgn: {err:.2e}")
    assert err < 1e-6
    Rk = np.eye(d) - 2.0 * Q[:, :k] @ Q[:, :k].T
    lexact = float(np.sum(G * Rk))
    _say(f"  loss {loss:.12e} exact {lexact:.12e}")
    assert abs(loss - lexact) <= 1e-9 * abs(lexact) + 1e-9
    assert np.linalg.norm(Rm.cpu().numpy() - Rk) <= 1e-8 * np.sqrt(d)
    E = inputs.symmetric_normal(d, 1)
    E /= np.linalg.norm(E)
    t = 1e-4
    fd = (_limit_loss(H + t * E, G, k) - _limit_loss(H - t * E, G, k)) / (2 * t)
    dd = float(np.sum(gn * E))
    _say(f"  directional derivative {dd:.12e}, central difference {fd:.12e}, rel {abs(dd - fd) / abs(fd):.2e}")
    assert abs(dd - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("d,k,lanczos", [(300, 5, False), (257, 3, True), (1000, 1, False)])
def test_grad_mixed_small(R, handle, d, k, lanczos):
    H, lam, Q = inputs.planted_hessian(d, k, 0.05, 100 + d)
    s = 0.5 * (lam[k - 1] + lam[k])
    Gn = np.random.default_rng(d).standard_normal((d, d))   # only sym(G) counts
    g, loss, _, info, st = R.sign_grad(_gpu(H), _gpu(Gn), k, None if lanczos else s, handle=handle,
                                       precision="mixed", tol=1e-8 * np.sqrt(d), seed=2)
    dk = oracle.sign_frechet_dk(H, s, 0.5 * (Gn + Gn.T))
    err = _rel(g.cpu().numpy(), dk)
    Rk = np.eye(d) - 2.0 * Q[:, :k] @ Q[:, :k].T
    lerr = abs(loss - np.sum(Gn * Rk)) / abs(np.sum(Gn * Rk))
    _say(f"grad mixed d={d} k={k} lanczos={lanczos}: status={R.STATUS[st]} cg={info['cg_iters']} "
         f"vs DK {err:.2e} loss rel {lerr:.2e}")
    assert st == 0 and err < 1e-7 and lerr < 1e-9
