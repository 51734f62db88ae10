"""The outer shifted-sign reflector iteration of Alg. 4.3 in the explicit-
Hessian regime, driven through the library:

    x_{n+1} = x_n - eta R_n g_n      (eq. discrete_step)

with g_n = grad E(x_n), R_n the reflector refl_sign_apply computes for
H_n = hess E(x_n) at the shift a ShiftPolicy returns (Prop. 4.1 midpoint,
damped midpoint, or reuse/refresh with the Prop. 4.2 certificate), either the
finite filter p_m (fixed_steps = m) or the converged sign.  Host-side
sequencing only: every reflector product runs in the library's kernels.
"""
import numpy as np


def descend(grad, hess, x0, k, eta, steps, handle, policy="midpoint", policy_kw=None,
            gtol=1e-10, similarity=None, shift_fn=None, **sign_kw):
    """Run Alg. 4.3 from x0 for at most ``steps`` iterations (stop when
    ||g|| < gtol or when the policy cannot certify a shift).

    ``shift_fn(H)`` (H a numpy array), when given, supplies the shift instead
    of the policy: the paper's other estimate route, a dense eigensolver
    (block Lanczos cannot resolve the gap of a small stiff Hessian within its
    d/b steps).

    ``grad(x)`` and ``hess(x)`` return numpy arrays; ``hess`` must be
    symmetric.  With ``similarity`` = S (a positive vector) the energy's
    Hessian is not symmetric but S H S^-1 is: ``hess`` returns S H S^-1 and
    the direction is S^-1 sgn(S H S^-1) S g = sgn(H) g.  ``sign_kw`` go to
    refl.sign_apply (precision, fixed_steps, tol, ...).

    Returns dict(x, steps, gnorm (history), shifts (history), status)."""
    import torch
    from . import refl

    dev = handle.device
    pol = refl.ShiftPolicy(handle, policy, k, **(policy_kw or {}))
    x = np.array(x0, dtype=np.float64)
    gnorms, shifts = [], []
    status = 0
    try:
        for n in range(steps):
            g = grad(x)
            gn = float(np.linalg.norm(g))
            gnorms.append(gn)
            if gn < gtol:
                break
            Hn = np.ascontiguousarray(hess(x))
            H = torch.from_numpy(Hn).to(dev)
            if shift_fn is not None:
                s = float(shift_fn(Hn))
            else:
                s, info, status = pol.shift(H, check=False)
                if status != 0:
                    break
            shifts.append(s)
            v = g if similarity is None else similarity * g
            y, _, status = refl.sign_apply(H, torch.from_numpy(v).to(dev), k, s, handle=handle,
                                           check=False, **sign_kw)
            if status not in (0, refl.REFL_ERR_NOT_CONVERGED):
                break
            status = 0
            d = y.cpu().numpy()
            if similarity is not None:
                d = d / similarity
            x = x - eta * d
        else:
            gnorms.append(float(np.linalg.norm(grad(x))))
    finally:
        pol.close()
    return {"x": x, "steps": len(shifts), "gnorm": gnorms, "shifts": shifts, "status": status}


def exact_midpoint(k):
    """Shift from a dense eigensolver (the paper's other estimate route):
    the midpoint of lambda_k and lambda_{k+1} (Prop. 4.1)."""
    def mid(Hn):
        w = np.linalg.eigvalsh(Hn)
        return 0.5 * (w[k - 1] + w[k])
    return mid


def target_index_scan(handle, ks=(1, 2, 4, 8, 16), nstarts=32, ms=(2, 4, 6), d=64, eta=0.3,
                      steps=200, npert=32, pert=0.05, seed=0, start_scale=0.3):
    """The target-index scan of section 5.3 on the rotated quartic family
    (inputs.RotatedQuartic, index-k saddle at the origin), driven through
    the library: for each k, ``nstarts`` matched starts (start seeds
    0 .. nstarts - 1, the same for every engine) run Alg. 4.3 with the
    converged sign engine (m = 0) and with the midpoint filters p_m, m in
    ``ms`` (shift: the exact midpoint of a dense eigensolver).  A run
    succeeds when it reaches ||g|| < 1e-10 at a point of Morse index k
    within 1e-6 of the saddle.  The one-step direction error of each engine,
    ||R g - R_k g|| / ||R_k g|| against the exact reflector, is taken at
    ``npert`` seeded perturbations of the saddle of size ``pert``.

    Returns {k: {m: dict(success=[bool per start], steps=[...],
    ms_per_run=[host wall time of each run], ms_per_step=median over runs of
    the wall time per outer step (energy, shift and refl_sign_apply),
    dir_err=[per perturbation])}}."""
    import time

    import torch
    from . import inputs, refl

    dev = handle.device
    out = {}
    for k in ks:
        q = inputs.RotatedQuartic(d, k, seed)
        mid = exact_midpoint(k)
        per_k = {}
        for m in (0,) + tuple(ms):
            kw = dict(fixed_steps=m) if m > 0 else dict(tol=1e-13)
            succ, nsteps, times, runs = [], [], [], []
            for st in range(nstarts):
                x0 = q.start(st, start_scale)
                t0 = time.perf_counter()
                r = descend(q.grad, q.hess, x0, k, eta, steps, handle, shift_fn=mid, **kw)
                dt = time.perf_counter() - t0
                x = r["x"]
                idx = int(np.sum(np.linalg.eigvalsh(q.hess(x)) < 0))
                ok = r["status"] == 0 and r["gnorm"][-1] < 1e-10 and idx == k and np.linalg.norm(x) < 1e-6
                succ.append(bool(ok))
                nsteps.append(r["steps"])
                runs.append(1e3 * dt)
                if r["steps"]:
                    times.append(1e3 * dt / r["steps"])
            errs = []
            rng = np.random.default_rng(10_000 + k)
            for _ in range(npert):
                x = pert * rng.standard_normal(d)
                H, g = q.hess(x), q.grad(x)
                w, V = np.linalg.eigh(H)
                dex = g - 2.0 * V[:, :k] @ (V[:, :k].T @ g)
                s = 0.5 * (w[k - 1] + w[k])
                y, _, stt = refl.sign_apply(torch.from_numpy(np.ascontiguousarray(H)).to(dev),
                                            torch.from_numpy(g).to(dev), k, s, handle=handle, check=False,
                                            **kw)
                errs.append(float(np.linalg.norm(y.cpu().numpy() - dex) / np.linalg.norm(dex)))
            per_k[m] = dict(success=succ, steps=nsteps, ms_per_run=runs,
                            ms_per_step=float(np.median(times)) if times else float("nan"), dir_err=errs)
        out[k] = per_k
    return out
