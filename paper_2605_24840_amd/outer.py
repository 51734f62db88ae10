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
