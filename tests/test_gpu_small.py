"""The LDS-resident iteration of small problems (FP32 d <= 128, FP64 d <= 96):
one work-group runs every Newton-Schulz step of eq. NS with X and N held in
LDS and the stopping rule on the device.  refl_sign and refl_sign_batched both
route such problems there; REFL_SMALL=0 sends them through the tiled products
instead, which the tests use as a second GPU path.

Pins, all against the oracle (FP64, plain dense recurrences):

* Fixed depth m: X_m equals the oracle's iterate X_m of eq. NS from the same
  X_0 = (H - sI)/alpha with alpha = ||H - sI||_inf.  FP64: each step is an
  O(d u64) perturbation that later steps propagate with gain below 3 on the
  spectrum in [-1, 1], so 1e-12 over m <= 6 covers it.  FP32: the FP32 error
  of the same chain, m d u32 scaled.
* Converged: the reflector of the exact eigenvectors to 1e-9 (FP64, to
  ||X^2 - I||_F < 1e-11), or the FP32 bound resid + 4 u32 sqrt(d)/gamma of
  the batched tests.
* The two GPU paths (small, tiled) agree to the same levels and take the same
  number of steps on these well-separated problems.
* A step cap below the needed depth gives REFL_ERR_NOT_CONVERGED with X_cap.
* A batch of small problems only (no grouped steps at all) and a mixed batch
  (small problems on a side stream beside the grouped steps) both return, bit
  for bit, what refl_sign returns.
"""
import numpy as np
import pytest

import oracle
from paper_2605_24840_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def R():
    from paper_2605_24840_amd import refl
    refl.load()
    return refl


@pytest.fixture(scope="module")
def handle(R):
    h = R.Handle(torch.device("cuda:0"))
    yield h
    h.close()


def _problem(d, k, grel, seed):
    H, lam, Q = inputs.planted_hessian(d, k, 2 * grel, seed)
    s = 0.5 * (lam[k - 1] + lam[k])
    return H, lam, Q, s


ORDERS = [(3, 1), (7, 3), (16, 5), (33, 8), (64, 4), (96, 12), (128, 16)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k", ORDERS)
def test_small_fixed_depth_matches_oracle_iterates(R, handle, prec, d, k):
    if prec == "fp64" and d > 96:
        pytest.skip("FP64 small path holds d <= 96")
    H, lam, Q, s = _problem(d, k, 5e-2, 100 + d)
    Hd = torch.from_numpy(H).to("cuda:0")
    alpha = oracle.inf_norm_shifted(H, s)
    Xs = oracle.ns_iterates(H, s, alpha, 6)
    for m in (1, 2, 3, 6):
        _say(f"small fixed depth {prec} d={d} k={k} m={m}")
        Rm, info, st = R.sign(Hd, k, s, handle=handle, precision=prec, fixed_steps=m, check=False)
        assert st == 0 and info["ns_steps"] == m
        err = float(np.abs(Rm.cpu().numpy() - Xs[m]).max())
        bound = 1e-12 if prec == "fp64" else 4.0 * m * d * U32
        assert err <= bound, (m, err, bound)
        assert abs(info["alpha"] - alpha) <= 1e-14 * alpha
        # The reported trace is that of the returned iterate (R holds it exactly).
        assert abs(info["trace"] - float(torch.trace(Rm))) <= 1e-12 * d
        assert abs(info["trace"] - np.trace(Xs[m])) <= (1e-11 if prec == "fp64" else d * bound)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k", ORDERS)
def test_small_converged_matches_tiled_and_exact(R, handle, monkeypatch, prec, d, k):
    if prec == "fp64" and d > 96:
        pytest.skip("FP64 small path holds d <= 96")
    H, lam, Q, s = _problem(d, k, 2e-2, 200 + d)
    Hd = torch.from_numpy(H).to("cuda:0")
    tol = 1e-11 if prec == "fp64" else 1e-3
    _say(f"small converged {prec} d={d} k={k}")
    Rs, i_s, st_s = R.sign(Hd, k, s, handle=handle, precision=prec, tol=tol, check=False)
    Rs = Rs.clone()
    monkeypatch.setenv("REFL_SMALL", "0")
    Rt, i_t, st_t = R.sign(Hd, k, s, handle=handle, precision=prec, tol=tol, check=False)
    monkeypatch.delenv("REFL_SMALL")
    assert st_s == 0 and st_t == 0
    assert i_s["index_j"] == k and i_t["index_j"] == k
    assert i_s["ns_steps"] == i_t["ns_steps"], (i_s["ns_steps"], i_t["ns_steps"])
    exact = oracle.reflector_from_eig(Q, k)
    e_s = float(np.linalg.norm(Rs.cpu().numpy() - exact))
    e_t = float(np.linalg.norm(Rt.cpu().numpy() - exact))
    diff = float(np.linalg.norm((Rs - Rt).cpu().numpy()))
    if prec == "fp64":
        assert e_s < 1e-9 and e_t < 1e-9 and diff < 1e-9, (e_s, e_t, diff)
    else:
        alpha = oracle.inf_norm_shifted(H, s)
        gamma = min(s - lam[k - 1], lam[k] - s) / alpha
        dk = 4 * U32 * np.sqrt(d) / gamma
        assert e_s <= i_s["resid_fro"] + dk, (e_s, i_s["resid_fro"], dk)
        assert diff <= i_s["resid_fro"] + i_t["resid_fro"] + 2 * dk
    _say(f"  steps={i_s['ns_steps']} err small={e_s:.2e} tiled={e_t:.2e} diff={diff:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_step_cap_not_converged(R, handle, prec):
    d, k = 48, 6
    H, lam, Q, s = _problem(d, k, 1e-3, 301)
    Hd = torch.from_numpy(H).to("cuda:0")
    alpha = oracle.inf_norm_shifted(H, s)
    Xs = oracle.ns_iterates(H, s, alpha, 4)
    _say(f"small step cap {prec}")
    Rm, info, st = R.sign(Hd, k, s, handle=handle, precision=prec, tol=1e-12, max_iter=4, check=False)
    assert R.STATUS[st] == "REFL_ERR_NOT_CONVERGED", R.STATUS[st]
    assert info["ns_steps"] == 4
    err = float(np.abs(Rm.cpu().numpy() - Xs[4]).max())
    assert err <= (1e-12 if prec == "fp64" else 16.0 * d * U32), err
    ref = float(np.linalg.norm(Xs[4] @ Xs[4] - np.eye(d)))
    assert abs(info["resid_fro"] - ref) <= (1e-10 if prec == "fp64" else 1e-3 * ref), (info["resid_fro"], ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_small_only_and_mixed_equal_single(R, handle, prec):
    small = [(16, 2, 5e-2, 401), (64, 7, 1e-2, 402), (96, 3, 2e-2, 403), (40, 1, 1e-1, 404)]
    if prec == "fp32":
        small.append((128, 9, 1e-2, 405))
    large = [(160, 4, 2e-2, 406), (256, 11, 1e-2, 407)]
    tol = 1e-10 if prec == "fp64" else 1e-3
    for specs in (small, small + large):
        probs = [_problem(d, k, g, sd) for d, k, g, sd in specs]
        Hs = [torch.from_numpy(p[0]).to("cuda:0") for p in probs]
        ks = [sp[1] for sp in specs]
        ss = [p[3] for p in probs]
        _say(f"batched {prec}: d={[sp[0] for sp in specs]}")
        Rs, infos, sts, st = R.sign_batched(Hs, ks, ss, handle=handle, precision=prec, tol=tol,
                                            check=False)
        assert st == 0 and all(x == 0 for x in sts)
        for p in range(len(specs)):
            R1, i1, st1 = R.sign(Hs[p], ks[p], ss[p], handle=handle, precision=prec, tol=tol,
                                 check=False)
            assert st1 == 0
            assert torch.equal(Rs[p], R1), p
            assert infos[p]["ns_steps"] == i1["ns_steps"] and infos[p]["trace"] == i1["trace"]
            assert infos[p]["index_j"] == ks[p]
            exact = oracle.reflector_from_eig(probs[p][2], ks[p])
            err = float(np.linalg.norm(Rs[p].cpu().numpy() - exact))
            if prec == "fp64":
                assert err < 1e-9, (p, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_order_limit(R, handle, prec):
    """refl.SMALL_MAX names the largest order of the one-launch path: with
    timing events, an order at the limit runs one timed launch, one above it
    the tiled products (m + 1 residual and m update products)."""
    dmax = R.SMALL_MAX[prec]
    for d, small in ((dmax, True), (dmax + 1, False)):
        H, lam, Q, s = _problem(d, 5, 5e-2, 500 + d)
        Hd = torch.from_numpy(H).to("cuda:0")
        _say(f"small limit {prec} d={d}")
        _, info, st = R.sign(Hd, 5, s, handle=handle, precision=prec, fixed_steps=3, timing=True,
                             check=False)
        assert st == 0 and info["ns_steps"] == 3
        assert info["gemm_launches"] == (1 if small else 7), info["gemm_launches"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_sign_apply_matches_sign(R, handle, prec):
    """R V without forming R takes the same one-launch iteration: it equals
    the formed R times V up to the rounding of the thin product."""
    d, k = 80, 7
    H, lam, Q, s = _problem(d, k, 2e-2, 601)
    Hd = torch.from_numpy(H).to("cuda:0")
    rng = np.random.default_rng(1)
    Vn = rng.standard_normal((d, 4))
    tol = 1e-11 if prec == "fp64" else 1e-3
    _say(f"small sign_apply {prec}")
    Rg, i1, st1 = R.sign(Hd, k, s, handle=handle, precision=prec, tol=tol, check=False)
    Y, i2, st2 = R.sign_apply(Hd, torch.from_numpy(Vn).to("cuda:0"), k, s, handle=handle,
                              precision=prec, tol=tol, check=False)
    assert st1 == 0 and st2 == 0 and i1["ns_steps"] == i2["ns_steps"]
    ref = Rg.cpu().numpy() @ Vn
    assert np.abs(Y.cpu().numpy() - ref).max() <= 1e-12 * np.abs(Vn).sum(axis=0).max()
