"""The outer shifted-sign iteration of Alg. 4.3 (eq. discrete_step) driven
through the library (`paper_2605_24840_amd.outer.descend`: Lanczos midpoint
policy + refl_sign_apply) against the oracle's loop (`oracle.outer_descent`:
exact eigendecomposition), on the paper's synthetic energies.  The paper
states neither eta, nor c_i, nor its starts, so these runs check properties
and agreement with the oracle loop, not the paper's figures (parity of the
figures is unpinned).

* Rotated quartic (section 5.3), d = 64, k in {1, 4, 16}: with the converged
  sign engine the reflector does not depend on the shift inside the gap, so
  both loops follow the same trajectory to rounding (1e-8 over the run) and
  reach the index-k saddle (||g|| < 1e-10, Morse index k).  With the finite
  filter p_4, the oracle is fed the library's shifts and scales the same way
  (inf-norm), and the trajectories agree to 1e-9.
* 1-D Allen-Cahn (section 5.4, n = 41, eps = 0.4): the one-step direction
  error of p_m against the exact reflector falls with m = 2, 4, 6 and equals
  the oracle's to 1e-10 relative; 200 converged-engine steps (dense-eigensolver
  midpoint: block Lanczos does not resolve this small stiff spectrum within
  d/b steps) track the oracle to 1e-9, and ||g|| falls by 100x towards the
  index-one zero state.
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


@pytest.mark.parametrize("k", [1, 4, 16])
def test_quartic_converged_engine_matches_oracle(R, handle, k):
    from paper_2605_24840_amd import outer
    q = inputs.RotatedQuartic(64, k, 0)
    x0 = q.start(1)
    lib = outer.descend(q.grad, q.hess, x0, k, 0.3, 300, handle, tol=1e-13)
    ref = oracle.outer_descent(q.grad, q.hess, x0, k, 0.3, 300)
    idx = int(np.sum(np.linalg.eigvalsh(q.hess(lib["x"])) < 0))
    dx = float(np.linalg.norm(lib["x"] - ref["x"]))
    _say(f"quartic k={k}: steps lib={lib['steps']} oracle={ref['steps']} |g|={lib['gnorm'][-1]:.2e} "
         f"index={idx} |x_lib - x_oracle|={dx:.2e} status={lib['status']}")
    assert lib["status"] == 0 and lib["gnorm"][-1] < 1e-10 and idx == k
    assert abs(lib["steps"] - ref["steps"]) <= 1
    n = min(len(lib["gnorm"]), len(ref["gnorm"]))
    assert np.allclose(lib["gnorm"][:n], ref["gnorm"][:n], rtol=1e-6, atol=1e-8)


def test_quartic_finite_filter_matches_oracle(R, handle):
    from paper_2605_24840_amd import outer
    k, m = 4, 4
    q = inputs.RotatedQuartic(64, k, 0)
    x0 = q.start(2)
    lib = outer.descend(q.grad, q.hess, x0, k, 0.3, 60, handle, fixed_steps=m, gtol=0.0)
    ref = oracle.outer_descent(q.grad, q.hess, x0, k, 0.3, len(lib["shifts"]), shifts=lib["shifts"], m=m,
                               gtol=0.0)
    dx = float(np.linalg.norm(lib["x"] - ref["x"]))
    _say(f"quartic p_{m}: {lib['steps']} steps, |g| {lib['gnorm'][0]:.2e} -> {lib['gnorm'][-1]:.2e}, "
         f"|x_lib - x_oracle|={dx:.2e}")
    assert lib["status"] == 0 and lib["steps"] == 60
    assert dx < 1e-9 * max(1.0, float(np.linalg.norm(ref["x"])))
    assert lib["gnorm"][-1] < 1e-3 * lib["gnorm"][0]


def test_allen_cahn_direction_error_falls_with_depth(R, handle):
    a = inputs.AllenCahn1D()
    u = 1e-3 * np.random.default_rng(5).standard_normal(a.n)
    H, g = a.hess_sym(u), a.grad(u)
    w, V = np.linalg.eigh(H)
    s = oracle.midpoint(w, 1)
    Rex, _ = oracle.shifted_sign_from_eig(w, V, s)
    dex = Rex @ (a.S * g) / a.S
    Hg = torch.from_numpy(H).to("cuda:0")
    v = torch.from_numpy(a.S * g).to("cuda:0")
    errs = []
    for m in (2, 4, 6):
        y, info, st = R.sign_apply(Hg, v, 1, s, handle=handle, fixed_steps=m)
        dm = y.cpu().numpy() / a.S
        Rm = oracle.ns_iterates(H, s, oracle.inf_norm_shifted(H, s), m)[m]
        dref = Rm @ (a.S * g) / a.S
        e = float(np.linalg.norm(dm - dex) / np.linalg.norm(dex))
        _say(f"allen-cahn p_{m}: direction error {e:.4e}, vs oracle filter "
             f"{np.linalg.norm(dm - dref) / np.linalg.norm(dref):.1e}")
        assert st == 0 and np.linalg.norm(dm - dref) <= 1e-10 * np.linalg.norm(dref)
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]
    y, info, st = R.sign_apply(Hg, v, 1, s, handle=handle, tol=1e-13)
    e = float(np.linalg.norm(y.cpu().numpy() / a.S - dex) / np.linalg.norm(dex))
    _say(f"allen-cahn converged engine: direction error {e:.2e}")
    assert st == 0 and e < 1e-10


def test_allen_cahn_outer_steps_track_oracle(R, handle):
    from paper_2605_24840_amd import outer
    a = inputs.AllenCahn1D()
    u0 = a.start(0)
    # Block Lanczos cannot resolve the gap of this stiff 41 x 41 Hessian within its d/b
    # steps, so the shift comes from a dense eigensolver (the paper's other route).
    def mid(Hn):
        w = np.linalg.eigvalsh(Hn)
        return 0.5 * (w[0] + w[1])
    lib = outer.descend(a.grad, a.hess_sym, u0, 1, 1.8e-3, 200, handle, similarity=a.S, tol=1e-13,
                        gtol=0.0, shift_fn=mid)
    ref = oracle.outer_descent(a.grad, a.hess_sym, u0, 1, 1.8e-3, 200, similarity=a.S, gtol=0.0)
    dx = float(np.linalg.norm(lib["x"] - ref["x"]))
    idx = int(np.sum(np.linalg.eigvalsh(a.hess_sym(lib["x"])) < 0))
    _say(f"allen-cahn 200 steps: |g| {lib['gnorm'][0]:.2e} -> {lib['gnorm'][-1]:.2e}, index {idx}, "
         f"|u_lib - u_oracle|={dx:.2e}")
    assert lib["status"] == 0 and lib["steps"] == 200
    assert dx < 1e-9 and idx == 1
    assert lib["gnorm"][-1] < 1e-2 * lib["gnorm"][0]


def test_target_index_scan_matches_oracle(R, handle):
    """The section 5.3 scan (d = 64, k in {1, 2, 4, 8, 16}, matched starts,
    converged engine and midpoint filters m = 2, 4, 6) through the library,
    at reduced breadth (4 starts, 6 perturbations per k), against the oracle's
    loop on the same starts: the same runs succeed, converged runs take the
    same number of steps (+-1), and the one-step direction errors equal the
    oracle filter's to 1e-9 relative.  As the paper reports, m = 2 is not
    robust (no run reaches the saddle within 200 steps here) while m = 4 and 6
    succeed wherever the exact reflector does, and the median direction error
    falls with m."""
    from paper_2605_24840_amd import outer
    ks, ns, ms, npert = (1, 2, 4, 8, 16), 4, (2, 4, 6), 6
    res = outer.target_index_scan(handle, ks=ks, nstarts=ns, ms=ms, npert=npert)
    for k in ks:
        q = inputs.RotatedQuartic(64, k, 0)
        rng = np.random.default_rng(10_000 + k)
        perts = [0.05 * rng.standard_normal(64) for _ in range(npert)]
        line = []
        for m in (0,) + ms:
            lib = res[k][m]
            for st in range(ns):
                ref = oracle.outer_descent(q.grad, q.hess, q.start(st, 0.3), k, 0.3, 200, m=m)
                idx = int(np.sum(np.linalg.eigvalsh(q.hess(ref["x"])) < 0))
                ok = ref["gnorm"][-1] < 1e-10 and idx == k and np.linalg.norm(ref["x"]) < 1e-6
                assert lib["success"][st] == bool(ok), (k, m, st)
                if ok:
                    assert abs(lib["steps"][st] - ref["steps"]) <= 1, (k, m, st)
            for x, e in zip(perts, lib["dir_err"]):
                H, g = q.hess(x), q.grad(x)
                w, V = np.linalg.eigh(H)
                s = 0.5 * (w[k - 1] + w[k])
                dex = g - 2.0 * V[:, :k] @ (V[:, :k].T @ g)
                Rm = oracle.shifted_sign_from_eig(w, V, s)[0] if m == 0 else \
                    oracle.ns_iterates(H, s, oracle.inf_norm_shifted(H, s), m)[m]
                eref = float(np.linalg.norm(Rm @ g - dex) / np.linalg.norm(dex))
                if m == 0:
                    assert e < 1e-10, (k, e)
                else:
                    assert abs(e - eref) <= 1e-9 * eref, (k, m, e, eref)
            line.append(f"m={m}: {sum(lib['success'])}/{ns} err {np.median(lib['dir_err']):.1e}")
        _say(f"k={k}: " + ", ".join(line))
        assert sum(res[k][2]["success"]) == 0
        for m in (4, 6):
            assert res[k][m]["success"] == res[k][0]["success"]
        meds = [np.median(res[k][m]["dir_err"]) for m in ms]
        assert meds[0] > meds[1] > meds[2] > np.median(res[k][0]["dir_err"])
