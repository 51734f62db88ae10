"""refl_sign_noalloc (the allocation-free variant of refl_sign, whose workspace
is the library's fixed device scratch) against refl_sign, through the C-ABI.

Each case runs two problems in a row on the shared scratch, the second of a
smaller order, so the second call finds the first one's contents there.  Both
calls use the same kernels on the same input, so R agrees with refl_sign's to
rounding (the bar is ||R_noalloc - R_sign||_F <= 1e-12 sqrt(d)), and each R is
also checked against the exact reflector R_k = I - 2 Q_k Q_k^T of the planted
spectrum (eq. Pk) to the method's bound: 1e-8 sqrt(d) for FP64 and MIXED, the
FP32 floor for FP32.
"""
import numpy as np
import pytest

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


def _exact(Q, k):
    d = Q.shape[0]
    return np.eye(d) - 2.0 * Q[:, :k] @ Q[:, :k].T


def _problem(d, k, gap, seed):
    H, lam, Q = inputs.planted_hessian(d, k, gap, seed)
    return H, 0.5 * (lam[k - 1] + lam[k]), _exact(Q, k)


def _pair(R, handle, d, k, gap, seed, prec, lanczos=False, sign_first=True, **kw):
    H, s, Rk = _problem(d, k, gap, seed)
    Hg = _gpu(H)
    shift = None if lanczos else s
    _say(f"noalloc {prec} d={d} k={k} gap={gap} seed={seed} lanczos={lanczos} sign_first={sign_first}")
    out_na = torch.full((d, d), float("nan"), dtype=torch.float64, device="cuda:0")
    if sign_first:
        Rs, info_s, st_s = R.sign(Hg, k, shift, handle=handle, precision=prec, seed=seed, **kw)
        Rn, info_n, st_n = R.sign_noalloc(Hg, k, shift, handle=handle, out=out_na, precision=prec,
                                          seed=seed, **kw)
    else:
        Rn, info_n, st_n = R.sign_noalloc(Hg, k, shift, handle=handle, out=out_na, precision=prec,
                                          seed=seed, **kw)
        Rs, info_s, st_s = R.sign(Hg, k, shift, handle=handle, precision=prec, seed=seed, **kw)
    torch.cuda.synchronize()
    assert st_s == 0 and st_n == 0, (st_s, st_n)
    a, b = Rn.cpu().numpy(), Rs.cpu().numpy()
    diff = float(np.linalg.norm(a - b))
    err_n = float(np.linalg.norm(a - Rk))
    err_s = float(np.linalg.norm(b - Rk))
    _say(f"  ||R_na - R_sign||_F={diff:.2e} ||R_na - R_k||_F={err_n:.2e} ||R_sign - R_k||_F={err_s:.2e} "
         f"steps {info_n['ns_steps']}/{info_s['ns_steps']}")
    assert np.isfinite(a).all()
    assert diff <= 1e-12 * np.sqrt(d)
    assert info_n["index_j"] == k and info_s["index_j"] == k
    bound = 1e-3 if prec == "fp32" else 1e-8 * np.sqrt(d)
    assert err_n <= bound and err_s <= bound
    return info_n


@pytest.mark.parametrize("prec,big,small", [
    ("fp64", (700, 6, 0.05, 1), (200, 3, 0.05, 2)),
    ("fp64", (300, 5, 0.1, 3), (64, 4, 0.1, 4)),          # tiled, then the one-launch small order
    ("fp32", (900, 8, 0.05, 5), (150, 4, 0.05, 6)),
    ("mixed", (1024, 8, 0.02, 7), (300, 5, 0.05, 8)),
])
def test_noalloc_matches_sign_two_calls(R, handle, prec, big, small):
    kw = {"tol": 1e-3} if prec == "fp32" else {"tol": 1e-12} if prec == "fp64" else {}
    _pair(R, handle, *big, prec, **kw)
    _pair(R, handle, *small, prec, **kw)


def test_noalloc_lanczos_shift_two_calls(R, handle):
    _pair(R, handle, 600, 4, 0.05, 9, "mixed", lanczos=True)
    _pair(R, handle, 257, 2, 0.05, 10, "mixed", lanczos=True)


def test_noalloc_untuned_order_first(R, handle):
    # An order no refl_sign call has tuned yet: the allocation-free call takes
    # the cost model's tile edge; refl_sign then times the candidates.
    _pair(R, handle, 777, 7, 0.05, 11, "fp64", sign_first=False, tol=1e-12)
    _pair(R, handle, 333, 3, 0.05, 12, "fp64", sign_first=False, tol=1e-12)


def test_noalloc_rejects_oversize_and_timing(R, handle):
    d = 2048
    H, s, _ = _problem(d, 3, 0.05, 13)
    Hg = _gpu(H)
    p = R.make_params(3, s, precision="fp64", tol=1e-12)
    need = R.refl_workspace_size(handle.h, d, p)
    _say(f"noalloc oversize d={d}: workspace {need} bytes")
    assert need > (64 << 20)
    out = torch.full((d, d), 7.0, dtype=torch.float64, device="cuda:0")
    _, _, st = R.sign_noalloc(Hg, 3, s, handle=handle, out=out, precision="fp64", tol=1e-12, check=False)
    assert R.STATUS[st] == "REFL_ERR_INVALID_ARG"
    assert "allocation-free" in R.refl_last_error(handle.h)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())   # no device work before the rejection
    _, _, st = R.sign_noalloc(Hg[:300, :300].contiguous(), 3, s, handle=handle, precision="fp64",
                              timing=True, check=False)
    assert R.STATUS[st] == "REFL_ERR_INVALID_ARG"
    # The handle still serves ordinary calls afterwards.
    _pair(R, handle, 400, 3, 0.05, 14, "fp64", tol=1e-12)
