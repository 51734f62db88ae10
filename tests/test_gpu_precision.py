"""MIXED bulk precision: the device-side stopping rule, escalation to more
BF16 words per operand, and the choice of three words from the Lanczos
estimate of the scaled margin (section 3.3: the margin gamma decides how much
the bulk arithmetic may perturb the eigenvalues nearest the shift before the
index changes).

One BF16 word cannot resolve the Allen-Cahn gap (the rounding of X_0 to one
word moves the spectrum by about 0.15/alpha, against a scaled half-gap of
1e-4), so a bulk started at one word must either fail its index certificate
or escalate; every result is checked against the exact R_k to 1e-8 sqrt(d).
"""
import os

import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def allen_cahn():
    path = os.path.join(GOLDEN, "allen_cahn_n64_seed0.npz")
    if not os.path.exists(path):
        pytest.skip("golden file missing")
    g = np.load(path)
    H, u = inputs.allen_cahn_2d(64, float(g["eps"]), 0)
    np.testing.assert_array_equal(u, g["u"])
    return H, g["w"], g["V"]


def test_one_word_escalates_to_a_certified_result(R, handle, allen_cahn):
    H, w, V = allen_cahn
    d, k = H.shape[0], 5
    s = 0.5 * (w[k - 1] + w[k])
    target = 1e-8 * np.sqrt(d)
    Hg = _gpu(H)
    _say("Allen-Cahn d=4096 k=5, one word, no escalation")
    _, info, st = R.sign(Hg, k, s, handle=handle, precision="mixed", tol=target, words=1, words_max=1,
                         check=False)
    _say(f"  status={R.STATUS[st]} steps={info['ns_steps']} j={info['index_j']} resid={info['resid_fro']:.2e}")
    assert R.STATUS[st] in ("REFL_ERR_NOT_ADMISSIBLE", "REFL_ERR_NOT_CONVERGED")
    assert info["bulk_words"] == 1
    # The device rule stops at the words' floor, long before the step cap.
    assert info["ns_steps"] < 60
    _say("Allen-Cahn d=4096 k=5, one word, escalation up to three")
    Rg, info, st = R.sign(Hg, k, s, handle=handle, precision="mixed", tol=target, words=1, words_max=3,
                          check=False)
    Rn = Rg.cpu().numpy()
    Rn -= np.eye(d)
    Rn += 2.0 * V[:, :k] @ V[:, :k].T
    err = float(np.linalg.norm(Rn))
    _say(f"  status={R.STATUS[st]} words={info['bulk_words']} steps={info['ns_steps']} j={info['index_j']} "
         f"err={err:.2e} dk={info['dk_bound']:.2e}")
    assert st == 0 and info["bulk_words"] >= 2 and info["index_j"] == k
    assert err <= target and err <= info["dk_bound"] * 1.0001


def test_two_words_need_no_escalation_on_the_workload(R, handle, allen_cahn):
    H, w, V = allen_cahn
    d = H.shape[0]
    for k in (1, 3, 5):
        s = 0.5 * (w[k - 1] + w[k])
        _, info, st = R.sign(_gpu(H), k, s, handle=handle, precision="mixed", tol=1e-8 * np.sqrt(d))
        _say(f"Allen-Cahn k={k}: words={info['bulk_words']} steps={info['ns_steps']} j={info['index_j']}")
        assert st == 0 and info["bulk_words"] == 2 and info["index_j"] == k


@pytest.mark.parametrize("gap,words", [(1e-4, 3), (2e-2, 2)])
def test_lanczos_margin_chooses_the_words(R, handle, gap, words):
    d, k = 1024, 8
    H, lam, Q = inputs.planted_hessian(d, k, gap, 11)
    target = 1e-8 * np.sqrt(d)
    Rg, info, st = R.sign(_gpu(H), k, None, handle=handle, precision="mixed", tol=target, seed=3,
                          check=False)
    err = float(np.linalg.norm(Rg.cpu().numpy() - (np.eye(d) - 2 * Q[:, :k] @ Q[:, :k].T)))
    _say(f"planted gap={gap}: status={R.STATUS[st]} gamma={info['gamma']:.2e} words={info['bulk_words']} "
         f"lanczos={info['lanczos_steps']} sweeps={info['polish_sweeps']} err={err:.2e}")
    assert st == 0
    assert info["bulk_words"] == words
    assert (info["gamma"] < 5e-6) == (words == 3)
    assert info["lanczos_steps"] > 0 and np.isfinite(info["lam_k"])
    assert err <= target


def test_words_max_validation(R, handle):
    d, k = 256, 3
    H, lam, Q = inputs.planted_hessian(d, k, 0.1, 1)
    s = 0.5 * (lam[k - 1] + lam[k])
    for wm in (1, 4):
        _, _, st = R.sign(_gpu(H), k, s, handle=handle, precision="mixed", words=2, words_max=wm, check=False)
        assert R.STATUS[st] == "REFL_ERR_INVALID_ARG"


def test_narrow_gap_two_words_fail_three_certify(R, handle):
    """A planted gap of 3e-7 (scaled margin 8.7e-9): the rounding of the
    two-word bulk moves an eigenvalue across the shift and the certificate
    finds j = k - 1; the three-word bulk keeps the index, and the default
    call (words_max = 3) escalates to it and returns the exact reflector."""
    d, k = 1024, 8
    H, lam, Q = inputs.planted_hessian(d, k, 3e-7, 12)
    s = 0.5 * (lam[k - 1] + lam[k])
    Hg = _gpu(H)
    target = 1e-8 * np.sqrt(d)
    _, info, st = R.sign(Hg, k, s, handle=handle, precision="mixed", tol=target, words=2, words_max=2,
                         check=False)
    _say(f"gap 3e-7, two words only: status={R.STATUS[st]} j={info['index_j']} steps={info['ns_steps']}")
    assert R.STATUS[st] == "REFL_ERR_NOT_ADMISSIBLE" and info["index_j"] == k - 1
    Rg, info, st = R.sign(Hg, k, s, handle=handle, precision="mixed", tol=target, polish_sweeps=4,
                          check=False)
    err = float(np.linalg.norm(Rg.cpu().numpy() - (np.eye(d) - 2 * Q[:, :k] @ Q[:, :k].T)))
    _say(f"gap 3e-7, default escalation: status={R.STATUS[st]} words={info['bulk_words']} j={info['index_j']} "
         f"sweeps={info['polish_sweeps']} cg={info['cg_iters']} err={err:.2e}")
    assert st == 0 and info["bulk_words"] == 3 and info["index_j"] == k
    assert err <= target and err <= info["dk_bound"] * 1.0001
