"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Tolerances:
* FP64 iterates: the library and the oracle run the same recurrence (eq. NS)
  in FP64 with different summation orders; the difference of X_m stays at
  the FP64 rounding level times the growth of the iteration (<= 1e-13 for
  d <= 300 and m <= 20, measured against the spectral closed form in the
  oracle pins).
* FP64 converged: ||X^2 - I||_F < 1e-12 gives ||X - sgn||_F < 1e-12 for a
  commuting iterate (eigenwise |p - s| <= |p^2 - 1|), plus rounding.
* MIXED: the target ||R - R_k||_F <= 1e-8 sqrt(d).
"""
import ctypes
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


def _cfg0():
    H, lam, Q = inputs.planted_hessian(64, 4, 0.1, 0)
    return H, lam, Q, 0.5 * (lam[3] + lam[4])


# ------------------------------------------------------------------ FP64
@pytest.mark.parametrize("m", [1, 2, 5, 10, 17, 20])
def test_fp64_iterates_match_oracle(R, handle, m):
    _say(f"fp64 iterate d=64 k=4 m={m}")
    H, lam, Q, s = _cfg0()
    Rg, info, st = R.sign(_gpu(H), 4, s, handle=handle, precision="fp64", fixed_steps=m)
    assert st == 0
    alpha = oracle.inf_norm_shifted(H, s)
    assert info["alpha"] == pytest.approx(alpha, rel=1e-15)
    Xm = oracle.ns_iterates(H, s, alpha, m)[m]
    err = np.abs(Rg.cpu().numpy() - Xm).max()
    _say(f"  max|X_m - oracle| = {err:.2e}")
    assert err < 1e-13


def test_fp64_ragged_size(R, handle):
    # d = 300: a 3 x 3 grid of 128-tiles (6 upper tiles) with a ragged tail.
    d, k = 300, 7
    _say(f"fp64 iterate d={d} k={k} m=6")
    H, lam, Q = inputs.planted_hessian(d, k, 0.05, 3)
    s = 0.5 * (lam[k - 1] + lam[k])
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="fp64", fixed_steps=6)
    alpha = oracle.inf_norm_shifted(H, s)
    X6 = oracle.ns_iterates(H, s, alpha, 6)[6]
    err = np.abs(Rg.cpu().numpy() - X6).max()
    _say(f"  max|X_6 - oracle| = {err:.2e}")
    assert err < 1e-13
    d2 = oracle.certificates(H, X6, s)
    assert info["trace"] == pytest.approx(d2["trace"], abs=1e-10)
    assert info["resid_fro"] == pytest.approx(d2["resid_fro"], rel=1e-9)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ts", [32, 64, 96, 128])
def test_tile_edges_ragged(R, handle, monkeypatch, ts, prec):
    """Every tile edge of the FP64 / FP32 products on a ragged size (d = 300
    pads to 320, 320, 384 or 384): the same iterate as the oracle, and the
    same (bit for bit in FP64) whichever edge runs."""
    d, k, m = 300, 7, 6
    H, lam, Q = inputs.planted_hessian(d, k, 0.05, 3)
    s = 0.5 * (lam[k - 1] + lam[k])
    X6 = oracle.ns_iterates(H, s, oracle.inf_norm_shifted(H, s), m)[m]
    monkeypatch.setenv("REFL_F_TILE", str(ts))
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision=prec, fixed_steps=m)
    monkeypatch.setenv("REFL_F_TILE", "128")
    R128, _, _ = R.sign(_gpu(H), k, s, handle=handle, precision=prec, fixed_steps=m)
    err = np.abs(Rg.cpu().numpy() - X6).max()
    _say(f"{prec} tile {ts}: max|X_6 - oracle| = {err:.2e}, equal to tile 128: {torch.equal(Rg, R128)}")
    assert st == 0 and err < (1e-13 if prec == "fp64" else 1e-4)
    if prec == "fp64":
        assert torch.equal(Rg, R128)
    assert np.array_equal(Rg.cpu().numpy(), Rg.cpu().numpy().T)


def test_fp64_converged_config0(R, handle):
    _say("fp64 converged d=64 k=4 gap=0.1 midpoint tol=1e-12")
    H, lam, Q, s = _cfg0()
    Rg, info, st = R.sign(_gpu(H), 4, s, handle=handle, precision="fp64", tol=1e-12)
    assert st == 0
    Rk, w, V = oracle.reflector(H, 4)
    err = np.linalg.norm(Rg.cpu().numpy() - Rk)
    pred = oracle.ns_depth_scalar((w - s) / info["alpha"], 1e-12)
    _say(f"  ||R - R_k||_F = {err:.2e} steps={info['ns_steps']} predicted={pred} resid={info['resid_fro']:.2e}")
    assert info["resid_fro"] < 1e-12
    assert err < 2e-12
    assert info["index_j"] == 4
    assert abs(info["ns_steps"] - pred) <= 1


def test_fp64_off_centre_shifts(R, handle):
    H, lam, Q, s_mid = _cfg0()
    Rk, w, V = oracle.reflector(H, 4)
    steps = {}
    for theta in (0.1, 0.5, 0.9):
        s = lam[3] + theta * (lam[4] - lam[3])
        _say(f"fp64 d=64 theta={theta}")
        Rg, info, st = R.sign(_gpu(H), 4, s, handle=handle, precision="fp64", tol=1e-12)
        assert st == 0
        assert np.linalg.norm(Rg.cpu().numpy() - Rk) < 2e-12
        steps[theta] = info["ns_steps"]
    assert steps[0.5] < steps[0.1] and steps[0.5] < steps[0.9]


def test_fp64_symmetric_upper_only_deterministic(R, handle):
    d, k = 200, 5
    _say(f"fp64 upper-triangle-only d={d}")
    H, lam, Q = inputs.planted_hessian(d, k, 0.1, 4)
    s = 0.5 * (lam[k - 1] + lam[k])
    Hg = H.copy()
    Hg[np.tril_indices(d, -1)] = np.nan   # never read
    R1, _, st1 = R.sign(_gpu(Hg), k, s, handle=handle, precision="fp64")
    R2, _, st2 = R.sign(_gpu(H), k, s, handle=handle, precision="fp64")
    a, b = R1.cpu().numpy(), R2.cpu().numpy()
    assert st1 == 0 and st2 == 0
    assert np.array_equal(a, b)
    assert np.array_equal(a, a.T)
    Rk = np.eye(d) - 2 * Q[:, :k] @ Q[:, :k].T
    assert np.linalg.norm(a - Rk) < 2e-12


def test_apply_and_sign_apply(R, handle):
    d, k = 257, 6
    _say(f"apply d={d}")
    H, lam, Q = inputs.planted_hessian(d, k, 0.1, 5)
    s = 0.5 * (lam[k - 1] + lam[k])
    rng = np.random.default_rng(0)
    Vn = rng.standard_normal((d, 3))
    Rg, _, _ = R.sign(_gpu(H), k, s, handle=handle, precision="fp64")
    Y = R.apply(Rg, _gpu(Vn), handle=handle).cpu().numpy()
    ref = Rg.cpu().numpy() @ Vn
    assert np.abs(Y - ref).max() < 1e-12
    y = R.apply(Rg, _gpu(Vn[:, 0].copy()), handle=handle).cpu().numpy()
    assert np.abs(y - ref[:, 0]).max() < 1e-12
    Y2, info, st = R.sign_apply(_gpu(H), _gpu(Vn), k, s, handle=handle, precision="fp64")
    assert st == 0
    assert np.abs(Y2.cpu().numpy() - ref).max() < 1e-12
    # Prop. 3.3: the direction error is bounded by the operator error.
    Rk = np.eye(d) - 2 * Q[:, :k] @ Q[:, :k].T
    g = Vn[:, 0]
    assert np.linalg.norm(y - Rk @ g) <= oracle.spectral_norm_sym(Rg.cpu().numpy() - Rk) * np.linalg.norm(g) + 1e-14


# --------------------------------------------------------------- errors
def test_error_paths(R, handle):
    H, lam, Q, s = _cfg0()
    Hg = _gpu(H)
    _say("errors: bad k")
    for k in (-1, 64):
        _, _, st = R.sign(Hg, k, s, handle=handle, check=False)
        assert R.STATUS[st] == "REFL_ERR_INVALID_ARG"
    _, _, st = R.sign(Hg, 0, None, handle=handle, check=False)   # k = 0 needs a given shift
    assert R.STATUS[st] == "REFL_ERR_INVALID_ARG"
    _say("errors: non-finite H")
    Hn = H.copy()
    Hn[3, 10] = np.nan
    _, _, st = R.sign(_gpu(Hn), 4, s, handle=handle, check=False)
    assert R.STATUS[st] == "REFL_ERR_NOT_FINITE"
    _, _, st = R.sign(Hg, 4, float("nan"), handle=handle, check=False)
    assert R.STATUS[st] == "REFL_ERR_NOT_FINITE"
    _say("errors: shift outside the gap")
    _, info, st = R.sign(Hg, 4, 0.5 * (lam[4] + lam[5]), handle=handle, check=False)
    assert R.STATUS[st] == "REFL_ERR_NOT_ADMISSIBLE" and info["index_j"] == 5
    _say("errors: max_iter too small")
    Rg, info, st = R.sign(Hg, 4, s, handle=handle, max_iter=2, check=False)
    assert R.STATUS[st] == "REFL_ERR_NOT_CONVERGED" and info["ns_steps"] == 2
    alpha = oracle.inf_norm_shifted(H, s)
    assert np.abs(Rg.cpu().numpy() - oracle.ns_iterates(H, s, alpha, 2)[2]).max() < 1e-13
    _say("errors: shift equal to an eigenvalue")
    D = np.diag(np.linspace(-1, 1, 16))
    _, info, st = R.sign(_gpu(D), 8, D[7, 7], handle=handle, check=False, max_iter=60)
    assert R.STATUS[st] == "REFL_ERR_NOT_CONVERGED" and info["index_j"] == -1


def test_symmetry_check(R, handle):
    """params.check_symmetric: H is read in full and rejected with
    NOT_SYMMETRIC when max |H_ij - H_ji| exceeds sym_tol max |H_ij| (or a
    NaN sits anywhere); an exactly symmetric H passes and gives the same R
    as without the check; off by default, when the lower triangle is never
    read.  Also through refl_sign_apply, refl_sign_grad and a batch."""
    H, lam, Q, s = _cfg0()
    Hg = _gpu(H)
    R0, _, st0 = R.sign(Hg, 4, s, handle=handle)
    R1, _, st1 = R.sign(Hg, 4, s, handle=handle, check_symmetric=True)
    assert st0 == 0 and st1 == 0 and torch.equal(R0, R1)
    Ha = H.copy()
    Ha[10, 3] += 1e-9                       # lower triangle only
    amax = float(np.abs(Ha).max())
    for tol, want in ((0.0, "REFL_ERR_NOT_SYMMETRIC"), (0.5e-9 / amax, "REFL_ERR_NOT_SYMMETRIC"),
                      (2e-9 / amax, "REFL_OK")):
        _, _, st = R.sign(_gpu(Ha), 4, s, handle=handle, check_symmetric=True, sym_tol=tol, check=False)
        _say(f"symmetry check tol={tol:.1e}: {R.STATUS[st]}")
        assert R.STATUS[st] == want
    _, _, st = R.sign(_gpu(Ha), 4, s, handle=handle, check=False)
    assert st == 0                          # off: the lower triangle is not read
    Hn = H.copy()
    Hn[40, 2] = np.nan
    _, _, st = R.sign(_gpu(Hn), 4, s, handle=handle, check_symmetric=True, sym_tol=1.0, check=False)
    assert R.STATUS[st] == "REFL_ERR_NOT_SYMMETRIC"
    V = _gpu(np.ones((64, 2)))
    _, _, st = R.sign_apply(_gpu(Ha), V, 4, s, handle=handle, precision="mixed", check_symmetric=True,
                            check=False)
    assert R.STATUS[st] == "REFL_ERR_NOT_SYMMETRIC"
    G = _gpu(np.eye(64))
    *_, st = R.sign_grad(_gpu(Ha), G, 4, s, handle=handle, check_symmetric=True, check=False)
    assert R.STATUS[st] == "REFL_ERR_NOT_SYMMETRIC"
    Rs, infos, sts, st = R.sign_batched([Hg, _gpu(Ha)], [4, 4], [s, s], handle=handle,
                                        precision="fp64", check_symmetric=True, check=False)
    assert [R.STATUS[x] for x in sts] == ["REFL_OK", "REFL_ERR_NOT_SYMMETRIC"]
    assert R.STATUS[st] == "REFL_ERR_NOT_SYMMETRIC" and torch.equal(Rs[0], R0)


def test_index_report_mode(R, handle):
    """k = 0: no target; the certified index j is reported and R = sgn(H - sI)
    for that j (the reflector R_j, Prop. 2.1), including the definite cases
    j = 0 (R = I) and j = d (R = -I)."""
    H, lam, Q, s = _cfg0()
    Hg = _gpu(H)
    R4, i4, st = R.sign(Hg, 4, s, handle=handle)
    R0, i0, st0 = R.sign(Hg, 0, s, handle=handle)
    _say(f"k=0 in gap 4: j={i0['index_j']}")
    assert st0 == 0 and i0["index_j"] == 4 and torch.equal(R0, R4)
    s5 = 0.5 * (lam[4] + lam[5])
    R5, i5, st5 = R.sign(Hg, 0, s5, handle=handle)
    err5 = np.linalg.norm(R5.cpu().numpy() - oracle.reflector_from_eig(Q, 5))
    _say(f"k=0 in gap 5: j={i5['index_j']} err={err5:.2e}")
    assert st5 == 0 and i5["index_j"] == 5 and err5 < 1e-11
    for s_out, j, sign in ((-1.5, 0, 1.0), (1.5, 64, -1.0)):
        for prec in ("fp64", "mixed"):
            Rd, idd, std = R.sign(Hg, 0, s_out, handle=handle, precision=prec, check=False)
            err = float((Rd - sign * torch.eye(64, dtype=torch.float64, device=Rd.device)).abs().max())
            _say(f"k=0 {prec} s={s_out}: status={R.STATUS[std]} j={idd['index_j']} max|R - ({sign:+.0f})I|={err:.1e}")
            assert std == 0 and idd["index_j"] == j
            assert err < (1e-12 if prec == "fp64" else 1e-30)
    Rm, im, stm = R.sign(Hg, 0, s, handle=handle, precision="mixed")
    errm = np.linalg.norm(Rm.cpu().numpy() - oracle.reflector_from_eig(Q, 4))
    _say(f"k=0 mixed in gap 4: j={im['index_j']} err={errm:.2e}")
    assert stm == 0 and im["index_j"] == 4 and errm <= 1e-8 * np.sqrt(64)


def test_frobenius_scale(R, handle):
    H, lam, Q, s = _cfg0()
    Rg, info, st = R.sign(_gpu(H), 4, s, handle=handle, scale="fro")
    fro = oracle.fro_norm_shifted(H, s)
    err = np.linalg.norm(Rg.cpu().numpy() - oracle.reflector_from_eig(Q, 4))
    _say(f"scale fro: alpha={info['alpha']:.15e} oracle={fro:.15e} steps={info['ns_steps']} err={err:.2e}")
    assert st == 0 and abs(info["alpha"] - fro) <= 1e-14 * fro and err < 1e-11


# ------------------------------------------------------------------ FP32
@pytest.mark.parametrize("grel,theta", [(1e-1, 0.5), (1e-2, 0.5), (1e-2, 0.1)])
def test_fp32_controlled_spectra(R, handle, grel, theta):
    d, k = 1024, 8
    _say(f"fp32 d={d} k={k} grel={grel} theta={theta}")
    H, lam, Q = inputs.planted_hessian(d, k, 2 * grel, 0)
    s = lam[k - 1] + theta * (lam[k] - lam[k - 1])
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="fp32", tol=1e-3, check=False)
    Rk = np.eye(d) - 2 * Q[:, :k] @ Q[:, :k].T
    err = np.linalg.norm(Rg.cpu().numpy() - Rk)
    _say(f"  status={R.STATUS[st]} steps={info['ns_steps']} resid={info['resid_fro']:.2e} ||R-R_k||_F={err:.2e}")
    assert info["index_j"] == k
    assert err < 1e-2


def test_fp32_default_tol_stops_at_floor(R, handle):
    """FP32 with the default tol (1e-12, far below the FP32 floor of
    ||X^2 - I||_F): the iteration stops at the floor (a residual below 0.1
    that does not halve over two steps, which exact steps always would)
    within a few steps of the depth the scalar model needs for 1e-3, not at
    the 100-step cap, with the certified index and the FP32 error bound."""
    d, k = 1024, 8
    H, lam, Q = inputs.planted_hessian(d, k, 0.02, 0)
    s = 0.5 * (lam[k - 1] + lam[k])
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="fp32", check=False)
    pred = oracle.ns_depth_scalar((lam - s) / info["alpha"], 1e-3)
    err = np.linalg.norm(Rg.cpu().numpy() - oracle.reflector_from_eig(Q, k))
    gamma = (s - lam[k - 1]) / info["alpha"]
    _say(f"fp32 default tol: status={R.STATUS[st]} steps={info['ns_steps']} (model to 1e-3: {pred}) "
         f"resid={info['resid_fro']:.2e} j={info['index_j']} err={err:.2e}")
    assert R.STATUS[st] == "REFL_ERR_NOT_CONVERGED"
    assert info["ns_steps"] <= pred + 6 and info["resid_fro"] < 0.1
    assert info["index_j"] == k
    assert err <= info["resid_fro"] + 4 * 2.0 ** -24 * np.sqrt(d) / gamma


# ----------------------------------------------------------------- MIXED
def test_mixed_bulk_iterate(R, handle):
    """Split-word bulk iterates against the oracle's model of the same
    arithmetic (oracle.ns_step_words: BF16 words by round-to-nearest-even,
    the kept word products, FP32 results), step by step: the library's X_j
    against one model step from the library's X_{j-1}.  The two differ only
    in the order of the FP32 accumulation of each product, bounded by
    gamma_n = n u32 times sum_k |a_ik||b_kj| <= ||A||_2 ||B||_2 <= 1 (rows
    of X and N have 2-norm at most ||X||_2, ||N||_2 <= 1), with n = the
    number of word products times K; one step has two products and N's
    error enters the second, so each step is within 3 gamma_n.  The FP64
    iterate of eq. NS is then within the model's own distance from it
    plus that bound times the steps."""
    d, k, m = 256, 4, 8
    _say(f"mixed bulk fixed steps d={d}")
    H, lam, Q = inputs.planted_hessian(d, k, 0.2, 1)
    s = 0.5 * (lam[k - 1] + lam[k])
    alpha = oracle.inf_norm_shifted(H, s)
    Hg = _gpu(H)
    X64 = oracle.ns_iterates(H, s, alpha, m)
    for words in (2, 3):
        nprod = 3 if words == 2 else 6
        step_tol = 3.0 * nprod * d * 2.0 ** -24
        model = oracle.ns_iterates_words(H, s, alpha, m, words)
        prev = None
        worst = 0.0
        for j in range(1, m + 1):
            Rg, info, st = R.sign(Hg, k, s, handle=handle, precision="mixed", words=words, fixed_steps=j)
            assert st == 0 and info["ns_steps"] == j
            Xj = Rg.cpu().numpy()
            ref = model[1] if j == 1 else oracle.ns_step_words(prev, words)
            e = float(np.abs(Xj - ref).max())
            worst = max(worst, e)
            assert e <= step_tol, (words, j, e, step_tol)
            prev = Xj
        e_model = float(np.abs(model[m] - X64[m]).max())
        e64 = float(np.abs(prev - X64[m]).max())
        _say(f"  words={words} per-step max|X_j - model step| = {worst:.2e} (bound {step_tol:.1e}); "
             f"max|X_8 - X_8(fp64)| = {e64:.2e}, model {e_model:.2e}")
        assert e64 <= e_model + m * 1.5 ** m * step_tol


@pytest.mark.parametrize("tile", ["128", "192"])
def test_mixed_bulk_ragged_tiles(R, handle, tile, monkeypatch):
    # d = 500 is ragged for both bulk tile edges (4 x 128, 3 x 192 tiles).
    d, k = 500, 6
    monkeypatch.setenv("REFL_BULK_TILE", tile)
    _say(f"mixed bulk fixed steps d={d} tile={tile}")
    H, lam, Q = inputs.planted_hessian(d, k, 0.1, 2)
    s = 0.5 * (lam[k - 1] + lam[k])
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="mixed", words=2, fixed_steps=6)
    alpha = oracle.inf_norm_shifted(H, s)
    X6 = oracle.ns_iterates(H, s, alpha, 6)[6]
    a = Rg.cpu().numpy()
    err = np.abs(a - X6).max()
    _say(f"  max|X_6 - oracle| = {err:.2e}")
    assert np.array_equal(a, a.T)
    assert err < 1e-3
    d2 = oracle.certificates(H, X6, s)
    assert info["trace"] == pytest.approx(d2["trace"], abs=1e-2)


@pytest.mark.parametrize("grel", [1e-1, 1e-2])
def test_mixed_planted_d1024(R, handle, grel):
    d, k = 1024, 8
    _say(f"mixed d={d} k={k} grel={grel}")
    H, lam, Q = inputs.planted_hessian(d, k, 2 * grel, 0)
    s = 0.5 * (lam[k - 1] + lam[k])
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="mixed", check=False)
    Rk = np.eye(d) - 2 * Q[:, :k] @ Q[:, :k].T
    err = np.linalg.norm(Rg.cpu().numpy() - Rk)
    _say(f"  status={R.STATUS[st]} steps={info['ns_steps']} sweeps={info['polish_sweeps']} "
         f"cg={info['cg_iters']} dk={info['dk_bound']:.2e} ||R-R_k||_F={err:.2e}")
    assert st == 0
    assert err <= 1e-8 * np.sqrt(d)


def test_mixed_timing_sampled(R, handle):
    # params.timing on the MIXED bulk: the events change nothing in the
    # result; timing = 1 times the products of every step taken (m + 1
    # residual, m update), timing = 3 those of steps 0, 3, 6, ... only.
    d, k = 1024, 8
    H, lam, Q = inputs.planted_hessian(d, k, 0.02, 0)
    s = 0.5 * (lam[k - 1] + lam[k])
    Hg = _gpu(H)
    _say(f"mixed timing sampled d={d} k={k}")
    runs = {}
    for t in (0, 1, 3):
        Rg, info, st = R.sign(Hg, k, s, handle=handle, precision="mixed", check=False, timing=t)
        assert st == 0
        runs[t] = (Rg.clone(), info)
    m = runs[0][1]["ns_steps"]
    assert m >= 6
    for t in (1, 3):
        assert torch.equal(runs[0][0], runs[t][0])
        assert runs[t][1]["ns_steps"] == m
    assert runs[0][1]["gemm_launches"] == 0
    assert runs[1][1]["gemm_launches"] == 2 * m + 1
    assert runs[3][1]["gemm_launches"] == sum(2 if j < m else 1 for j in range(0, m + 1, 3))
    assert runs[3][1]["ms_gemm"] > 0.0


def _allen_cahn_golden(seed=0):
    path = os.path.join(GOLDEN, f"allen_cahn_n64_seed{seed}.npz")
    if not os.path.exists(path):
        pytest.skip("golden file missing")
    g = np.load(path)
    H, u = inputs.allen_cahn_2d(64, float(g["eps"]), seed)
    np.testing.assert_array_equal(u, g["u"])
    return H, g["w"], g["V"]


@pytest.mark.parametrize("cg_prec", ["fp64", "fp32", "auto"])
def test_mixed_inner_solve_precision(R, handle, cg_prec):
    """The inner solves of the correction read H in FP64 or an FP32 copy; the
    Rayleigh-Ritz step and the certificate use H in FP64 either way, so the
    target holds and the certified bound is a bound."""
    d, k = 1024, 6
    H, lam, Q = inputs.planted_hessian(d, k, 0.02, 5)
    s = 0.5 * (lam[k - 1] + lam[k])
    target = 1e-8 * np.sqrt(d)
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="mixed", tol=target,
                          cg_prec=cg_prec)
    err = np.linalg.norm(Rg.cpu().numpy() - oracle.reflector_from_eig(Q, k))
    _say(f"mixed d={d} inner {cg_prec}: status={R.STATUS[st]} sweeps={info['polish_sweeps']} "
         f"cg={info['cg_iters']} dk={info['dk_bound']:.2e} err={err:.2e}")
    assert st == 0 and err <= target and err <= info["dk_bound"] * 1.0001 + 1e-15


@pytest.mark.parametrize("k,cg_prec", [(12, "fp32"), (20, "fp64"), (32, "fp32"), (32, "fp64")])
def test_mixed_wide_target_blocks(R, handle, k, cg_prec):
    """Wide target spaces take the block widths past 8 columns (12, 24, 32)
    in the subspace extraction, the Rayleigh-Ritz products and the inner
    CG, whose FP32 pass splits its chunks over two wave groups up to 16
    columns and not beyond; d = 700 leaves a ragged chunk and row group."""
    d = 700
    H, lam, Q = inputs.planted_hessian(d, k, 0.1, k)
    s = 0.5 * (lam[k - 1] + lam[k])
    target = 1e-8 * np.sqrt(d)
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="mixed", tol=target,
                          cg_prec=cg_prec)
    err = np.linalg.norm(Rg.cpu().numpy() - oracle.reflector_from_eig(Q, k))
    _say(f"mixed d={d} k={k} inner {cg_prec}: status={R.STATUS[st]} sweeps={info['polish_sweeps']} "
         f"cg={info['cg_iters']} dk={info['dk_bound']:.2e} err={err:.2e}")
    assert st == 0 and info["index_j"] == k
    assert err <= target and err <= info["dk_bound"] * 1.0001 + 1e-15


def test_mixed_inner_iteration_cap(R, handle):
    """The inner CG stops at cg_max_iter (the count reported is the cap);
    with a cap too small for one sweep the certified bound is missed and the
    call says so; with a small cap and more sweeps it still reaches the
    target."""
    d, k = 512, 4
    H, lam, Q = inputs.planted_hessian(d, k, 0.1, 2)
    s = 0.5 * (lam[k - 1] + lam[k])
    Hg = _gpu(H)
    for cap in (1, 3):
        _, info, st = R.sign(Hg, k, s, handle=handle, precision="mixed", tol=1e-14, check=False,
                             polish_sweeps=1, cg_max_iter=cap)
        _say(f"cap {cap}: status={R.STATUS[st]} sweeps={info['polish_sweeps']} cg={info['cg_iters']} "
             f"dk={info['dk_bound']:.2e}")
        assert R.STATUS[st] == "REFL_ERR_NOT_CONVERGED"
        assert info["polish_sweeps"] == 1 and info["cg_iters"] == cap
    target = 1e-8 * np.sqrt(d)
    Rg, info, st = R.sign(Hg, k, s, handle=handle, precision="mixed", tol=target, polish_sweeps=10,
                          cg_max_iter=20)
    err = np.linalg.norm(Rg.cpu().numpy() - oracle.reflector_from_eig(Q, k))
    _say(f"cap 20, up to 10 sweeps: status={R.STATUS[st]} sweeps={info['polish_sweeps']} cg={info['cg_iters']} "
         f"err={err:.2e}")
    assert st == 0 and err <= target and info["cg_iters"] <= 20 * info["polish_sweeps"]


@pytest.mark.parametrize("k", [1, 3, 5])
def test_mixed_allen_cahn_d4096(R, handle, k):
    _say(f"mixed Allen-Cahn d=4096 k={k}")
    H, w, Vk = _allen_cahn_golden(0)
    d = H.shape[0]
    s = 0.5 * (w[k - 1] + w[k])
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="mixed", check=False)
    Rn = Rg.cpu().numpy()
    Rn -= np.eye(d)
    Rn += 2.0 * Vk[:, :k] @ Vk[:, :k].T
    err = np.linalg.norm(Rn)
    _say(f"  status={R.STATUS[st]} steps={info['ns_steps']} sweeps={info['polish_sweeps']} "
         f"cg={info['cg_iters']} dk={info['dk_bound']:.2e} ||R-R_k||_F={err:.2e} "
         f"bulk={info['ms_bulk']:.1f}ms polish={info['ms_polish']:.1f}ms")
    assert st == 0
    assert err <= 1e-8 * np.sqrt(d)


# ------------------------------------------------------ tiny and empty
@pytest.mark.parametrize("d", [2, 3, 5])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_tiny_orders(R, handle, d, prec):
    """Orders far below one tile (the matrices are padded to a tile and zero
    outside d x d), every admissible index k = 1 .. d - 1, against the
    oracle's Jacobi reflector; the index certificate must give k."""
    rng = np.random.default_rng(100 + d)
    lam = np.sort(rng.uniform(-1.0, 1.0, d))
    lam += 0.3 * np.arange(d)                      # gaps of at least 0.3
    Q = inputs.haar_orthogonal(d, rng)
    H = np.ascontiguousarray(0.5 * ((Q * lam) @ Q.T + ((Q * lam) @ Q.T).T))
    Hg = _gpu(H)
    tol = {"fp64": 1e-12, "fp32": 1e-5, "mixed": 1e-8 * np.sqrt(d)}[prec]
    for k in range(1, d):
        Rk, w, V = oracle.reflector(H, k)
        s = oracle.midpoint(w, k)
        Rg, info, st = R.sign(Hg, k, s, handle=handle, precision=prec, tol=tol, check=False)
        err = float(np.linalg.norm(Rg.cpu().numpy() - Rk))
        _say(f"tiny d={d} k={k} {prec}: status={R.STATUS[st]} steps={info['ns_steps']} "
             f"j={info['index_j']} err={err:.1e}")
        # FP32: ||X - sgn(X)||_F <= ||X^2 - I||_F for the symmetric iterate, plus
        # the rounding of the products (u32 = 6e-8 per entry at these orders).
        bound = {"fp64": 1e-12, "fp32": info["resid_fro"] + 1e-6, "mixed": tol}[prec]
        assert st == 0 and info["index_j"] == k and err <= bound


def test_empty_arguments_rejected(R, handle):
    """Empty inputs are argument errors at the boundary: d = 0, nrhs = 0, an
    empty batch."""
    lib = R.load()
    h = handle.h
    buf = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    p = R.make_params(1, 0.0)
    info = R.refl_info_t()
    st = lib.refl_sign(h, 0, buf.data_ptr(), 1, ctypes.byref(p), buf.data_ptr(), 1, ctypes.byref(info))
    assert R.STATUS[st] == "REFL_ERR_INVALID_ARG"
    st = lib.refl_apply(h, 4, buf.data_ptr(), 4, 0, buf.data_ptr(), 4, buf.data_ptr(), 4)
    assert R.STATUS[st] == "REFL_ERR_INVALID_ARG"
    st = lib.refl_sign_batched(h, 0, None, None, None, None, None, None, None, None)
    assert R.STATUS[st] == "REFL_ERR_INVALID_ARG"


@pytest.fixture(scope="module")
def large():
    # d = 12000: three times the Allen-Cahn order, ragged against the 192-row
    # bulk tiles and the 64/128-row FP tiles.  1.15 GB per FP64 matrix.
    d, k = 12000, 8
    H, lam, Qk = inputs.planted_hessian_reflected(d, k, 0.02, 12)
    return H, lam, Qk, k


def _err_on_device(Rg, Qk):
    Qg = torch.from_numpy(Qk).to(Rg.device)
    E = Rg - torch.eye(Rg.shape[0], dtype=Rg.dtype, device=Rg.device)
    E += 2.0 * (Qg @ Qg.T)
    return float(torch.linalg.norm(E))


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
def test_large_order(R, handle, large, prec):
    """A large order through the whole path (d = 12000, k = 8, gap 0.02): the
    MIXED reflector meets 1e-8 sqrt(d) and its certified bound; FP32 meets
    its rounding bound (err <= resid + 4 u32 sqrt(d)/gamma, as for the
    controlled spectra)."""
    H, lam, Qk, k = large
    d = H.shape[0]
    s = 0.5 * (lam[k - 1] + lam[k])
    Hg = _gpu(H)
    tol = 1e-8 * np.sqrt(d) if prec == "mixed" else 1e-3
    Rg, info, st = R.sign(Hg, k, s, handle=handle, precision=prec, tol=tol, check=False)
    err = _err_on_device(Rg, Qk)
    _say(f"large d={d} k={k} {prec}: status={R.STATUS[st]} steps={info['ns_steps']} sweeps={info['polish_sweeps']} "
         f"cg={info['cg_iters']} j={info['index_j']} err={err:.2e} ms={info['ms_total']:.0f}")
    assert st == 0 and info["index_j"] == k
    if prec == "mixed":
        assert err <= tol and err <= info["dk_bound"] * 1.0001 + 1e-15
    else:
        gamma = (s - lam[k - 1]) / info["alpha"]
        assert err <= info["resid_fro"] + 4 * 2.0 ** -24 * np.sqrt(d) / gamma
    del Hg, Rg
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_shift_on_an_eigenvalue(R, handle, prec):
    """s equal to an eigenvalue (lambda_{k+1}): sgn(H - sI) is undefined.  The
    scaled matrix keeps an eigenvalue at rounding level, which each NS step
    multiplies by 1.5 only.  FP64 (60 steps): it stays below the certificate,
    so the call reports NOT_CONVERGED with no index.  FP32 and MIXED: the
    coarser rounding moves it to one side within the steps, and the
    certificate then counts it: either index k (the shift acts as one just
    above lambda_{k+1}, and the result must be R_k, which is defined since
    lambda_k < lambda_{k+1}) or k + 1 (NOT_ADMISSIBLE).  Never a certified
    reflector of the wrong index."""
    d, k = 64, 4
    w = np.linspace(-1.0, 1.0, d)
    Q = inputs.haar_orthogonal(d, np.random.default_rng(64))
    H = np.ascontiguousarray(0.5 * ((Q * w) @ Q.T + ((Q * w) @ Q.T).T))
    s = float(w[k])                      # lambda_{k+1}
    Rg, info, st = R.sign(_gpu(H), k, s, handle=handle, precision=prec, max_iter=60, check=False)
    status = R.STATUS[st]
    err = float(np.linalg.norm(Rg.cpu().numpy() - oracle.reflector_from_eig(Q, k)))
    _say(f"shift on lambda_{k + 1} ({prec}): status={status} steps={info['ns_steps']} "
         f"resid={info['resid_fro']:.3e} j={info['index_j']} ||R - R_k||_F={err:.1e}")
    if prec == "fp64":
        assert status == "REFL_ERR_NOT_CONVERGED" and info["index_j"] == -1
        assert info["resid_fro"] >= 0.5
    elif status == "REFL_OK":
        assert info["index_j"] == k
        assert err <= (1e-8 * np.sqrt(d) if prec == "mixed" else 1e-3)
    elif status == "REFL_ERR_NOT_ADMISSIBLE":
        assert info["index_j"] == k + 1
    else:
        assert status == "REFL_ERR_NOT_CONVERGED" and info["index_j"] == -1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_device_stopping_rule_single_solve(R, handle, prec):
    """FP32/FP64 solves above the small-order limit enqueue their steps four
    at a time and stop by the rule evaluated on the device; the products of
    steps past the stop do nothing.  A repeated call and a timed call give
    the same R, steps, residual and trace bit for bit, the timed call counts
    exactly the products of the steps taken (m + 1 residual, m update), and
    fixed depths that are not multiples of four stop exactly there, at the
    oracle's iterate."""
    d, k = 300, 9
    H, lam, Q = inputs.planted_hessian(d, k, 0.02, 31)
    s = 0.5 * (lam[k - 1] + lam[k])
    Hg = _gpu(H)
    tol = 1e-12 if prec == "fp64" else 1e-3

    def run(**kw):
        Rm, info, st = R.sign(Hg, k, s, handle=handle, precision=prec, tol=tol, check=False, **kw)
        assert st == 0
        return Rm.clone(), info

    _say(f"device stopping rule {prec} d={d}")
    g1, i1 = run()
    g2, i2 = run()
    t1, it = run(timing=True)
    assert i1["ns_steps"] >= 12
    for other, io in ((g2, i2), (t1, it)):
        assert torch.equal(g1, other)
        assert io["ns_steps"] == i1["ns_steps"] and io["resid_fro"] == i1["resid_fro"]
        assert io["trace"] == i1["trace"]
    assert it["gemm_launches"] == 2 * i1["ns_steps"] + 1
    exact = np.eye(d) - 2 * Q[:, :k] @ Q[:, :k].T
    err = float(np.linalg.norm(g1.cpu().numpy() - exact))
    assert err < (1e-9 if prec == "fp64" else 1e-2), err
    for m in (5, 6, 7):
        Rm, info, st = R.sign(Hg, k, s, handle=handle, precision=prec, fixed_steps=m, check=False)
        assert st == 0 and info["ns_steps"] == m
        alpha = oracle.inf_norm_shifted(H, s)
        Xm = oracle.ns_iterates(H, s, alpha, m)[m]
        assert np.abs(Rm.cpu().numpy() - Xm).max() < (1e-12 if prec == "fp64" else 4.0 * m * d * 2.0 ** -24)
