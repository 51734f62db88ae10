"""The bounds-checked debug build (librefl_debug.so, -DREFL_DEBUG) on the
device: on valid inputs no launch-extent guard trips, and every result is
bit for bit the release library's (the guards only add block-uniform entry
checks; the arithmetic and its order are unchanged).

Cases cover each guarded kernel family: FP64 and FP32 products at ragged
orders (FP64/FP32 tiles, mirror, row sums, X_0, reflector), the MIXED path
with its correction (word products, thin passes, inner-solve pass, update
and first partials, Cholesky QR), R V without forming R, the block-Lanczos
shift estimate, a batched call and two gradients (FP64 adjoint, and the
MIXED limit's FP64 block CG).  The release library's
results are themselves checked against the oracle by the other GPU tests.
"""
import numpy as np
import pytest

from paper_2605_24840_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _planted(d, k, gap, seed):
    H, lam, _ = inputs.planted_hessian(d, k, gap, seed)
    return torch.from_numpy(H).to("cuda:0"), 0.5 * (lam[k - 1] + lam[k])


def _run_all(refl):
    """Every case once with the current library; returns name -> (status
    list, host arrays)."""
    out = {}
    h = refl.Handle("cuda:0")
    try:
        for prec, d, k in (("fp64", 300, 4), ("fp32", 517, 7), ("mixed", 1000, 5)):
            _say(f"  sign {prec} d={d} k={k}")
            H, s = _planted(d, k, 0.1, d)
            R, info, st = refl.sign(H, k, s, handle=h, precision=prec,
                                    tol=1e-5 if prec == "fp32" else None)
            out[f"sign_{prec}"] = ([st], [R.cpu().numpy(), np.array([info["ns_steps"], info["cg_iters"]])])
        _say("  sign_apply mixed d=500 k=3 nrhs=33")
        H, s = _planted(500, 3, 0.1, 7)
        V = torch.from_numpy(np.random.default_rng(3).standard_normal((500, 33))).to("cuda:0")
        Y, _, st = refl.sign_apply(H, V, 3, s, handle=h, precision="mixed")
        out["sign_apply"] = ([st], [Y.cpu().numpy()])
        _say("  estimate_shift d=400 k=3")
        H, _ = _planted(400, 3, 0.1, 11)
        vals = refl.estimate_shift(H, 3, handle=h)
        out["estimate"] = ([vals[-1]], [np.array(vals[:-1])])
        _say("  sign_batched fp32 4 problems")
        Hs, ks, ss = [], [], []
        for i, (d, k) in enumerate(((100, 2), (300, 5), (130, 1), (520, 9))):
            Hi, si = _planted(d, k, 0.05, 100 + i)
            Hs.append(Hi), ks.append(k), ss.append(si)
        Rs, _, sts, st = refl.sign_batched(Hs, ks, ss, handle=h, precision="fp32", tol=1e-3)
        out["batched"] = ([st] + [int(x) for x in sts], [R.cpu().numpy() for R in Rs])
        _say("  sign_grad fp64 d=200 k=4")
        H, s = _planted(200, 4, 0.1, 21)
        G = torch.from_numpy(inputs.symmetric_normal(200, 5)).to("cuda:0")
        grad, loss, _, _, st = refl.sign_grad(H, G, 4, s, handle=h, tol=1e-10)
        out["grad"] = ([st], [grad.cpu().numpy(), np.array([loss])])
        _say("  sign_grad mixed d=400 k=3 (FP64 block CG of the gradient)")
        H, s = _planted(400, 3, 0.1, 23)
        G = torch.from_numpy(inputs.symmetric_normal(400, 6)).to("cuda:0")
        grad, loss, _, _, st = refl.sign_grad(H, G, 3, s, handle=h, precision="mixed")
        out["grad_mixed"] = ([st], [grad.cpu().numpy(), np.array([loss])])
    finally:
        h.close()
    return out


def test_debug_build_matches_release_and_trips_no_guard():
    from paper_2605_24840_amd import refl
    rel = refl.load(refl.LIB_PATH)
    assert rel.refl_debug_build() == 0
    _say("release library")
    a = _run_all(refl)
    try:
        dbg = refl.load(refl.DEBUG_LIB_PATH)
        assert dbg.refl_debug_build() == 1
        _say("debug library")
        b = _run_all(refl)
    finally:
        refl.load(refl.LIB_PATH)
    for name in a:
        sa, va = a[name]
        sb, vb = b[name]
        assert all(x == 0 for x in sa), (name, sa)
        assert sb == sa, (name, sb)
        for x, y in zip(va, vb):
            assert x.shape == y.shape and np.array_equal(x, y, equal_nan=True), name
    _say(f"  {len(a)} cases: debug build bit-equal to release, no guard tripped")


def test_refl_log_line():
    """REFL_LOG=1 makes each device entry point write one line to stderr with
    its status and figures.  The variable is read once per process, so the
    call runs in a child process (one small MIXED solve)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = (
        "import sys, torch; sys.path.insert(0, %r)\n"
        "from paper_2605_24840_amd import inputs, refl\n"
        "H, lam, _ = inputs.planted_hessian(300, 4, 0.1, 3)\n"
        "R, info, st = refl.sign(torch.from_numpy(H).to('cuda:0'), 4, 0.5 * (lam[3] + lam[4]), precision='mixed')\n"
        "print('status', st, info['ns_steps'], info['cg_iters'], flush=True)\n" % root)
    _say("child process with REFL_LOG=1: mixed d=300 k=4")
    r = subprocess.run([sys.executable, "-c", script], env=dict(os.environ, REFL_LOG="1"),
                       capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    _, st, steps, cg = r.stdout.split()[-4:]
    lines = [x for x in r.stderr.splitlines() if x.startswith("refl: refl_sign ")]
    assert len(lines) == 1, r.stderr[-2000:]
    assert f"d=300 status=REFL_OK steps={steps} " in lines[0] and f" cg={cg} j=4 " in lines[0], lines[0]
    _say(f"  {lines[0]}")
