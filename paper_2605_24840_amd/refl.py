"""Python binding of ``librefl.so`` (include/refl.h): argument marshalling only.

The functions named ``refl_*`` are the C entry points, called with device
pointers.  ``sign``, ``apply``, ``sign_apply``, ``sign_batched`` and
``estimate_shift`` wrap them for torch tensors on a ROCm device (torch provides the device memory and
the stream; every step of the computation runs in the library's kernels).
There is no CPU fallback: if the library is missing, loading raises.
"""
import ctypes
import math
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librefl.so")
# The same library with the kernels' launch-extent guards (-DREFL_DEBUG).
DEBUG_LIB_PATH = os.path.join(_PKG, "librefl_debug.so")

REFL_OK = 0
STATUS = {0: "REFL_OK", 1: "REFL_ERR_INVALID_ARG", 2: "REFL_ERR_DEVICE", 3: "REFL_ERR_NO_MEMORY",
          4: "REFL_ERR_NOT_CONVERGED", 5: "REFL_ERR_NOT_ADMISSIBLE", 6: "REFL_ERR_NO_GAP",
          7: "REFL_ERR_NOT_SYMMETRIC", 8: "REFL_ERR_UNSUPPORTED", 9: "REFL_ERR_NOT_FINITE",
          10: "REFL_ERR_BOUNDS"}
(REFL_ERR_INVALID_ARG, REFL_ERR_DEVICE, REFL_ERR_NO_MEMORY, REFL_ERR_NOT_CONVERGED,
 REFL_ERR_NOT_ADMISSIBLE, REFL_ERR_NO_GAP, REFL_ERR_NOT_SYMMETRIC, REFL_ERR_UNSUPPORTED,
 REFL_ERR_NOT_FINITE, REFL_ERR_BOUNDS) = range(1, 11)
PRECISION = {"fp64": 0, "fp32": 1, "mixed": 2}
SHIFT = {"given": 0, "lanczos": 1}
SCALE = {"inf": 0, "fro": 1, "lanczos": 2, "given": 3}
GRAD_MODE = {"reverse": 0, "tangent": 1}
CG_PREC = {"fp64": 0, "fp32": 1, "auto": 2}
# Largest orders the library runs as one LDS-resident launch (refl_sign and
# the batched solve), by precision; larger orders use the tiled products.
SMALL_MAX = {"fp32": 128, "fp64": 96}

EXPORTS = ["refl_params_default", "refl_create", "refl_destroy", "refl_set_stream",
           "refl_workspace_size", "refl_set_workspace", "refl_estimate_shift", "refl_sign",
           "refl_sign_noalloc", "refl_apply", "refl_sign_apply", "refl_sign_batched",
           "refl_sign_batched_workspace_size", "refl_sign_grad", "refl_policy_create",
           "refl_policy_destroy", "refl_policy_shift", "refl_status_string", "refl_last_error",
           "refl_debug_build"]


class refl_params_t(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("s", ctypes.c_double), ("shift_mode", ctypes.c_int32),
                ("scale_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("fixed_steps", ctypes.c_int32),
                ("words", ctypes.c_int32), ("polish_sweeps", ctypes.c_int32),
                ("cg_tol", ctypes.c_double), ("cg_max_iter", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("timing", ctypes.c_int32), ("grad_mode", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("cg_f32", ctypes.c_int32),
                ("check_symmetric", ctypes.c_int32), ("sym_tol", ctypes.c_double),
                ("words_max", ctypes.c_int32)]


class refl_policy_params_t(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("k", ctypes.c_int32), ("beta", ctypes.c_double),
                ("clip", ctypes.c_double), ("tau", ctypes.c_double),
                ("lanczos_steps", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("warm_start", ctypes.c_int32)]


class refl_policy_info_t(ctypes.Structure):
    _fields_ = [("s", ctypes.c_double), ("lam_k", ctypes.c_double), ("lam_k1", ctypes.c_double),
                ("eps", ctypes.c_double), ("margin", ctypes.c_double), ("drift", ctypes.c_double),
                ("refreshed", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
                ("calls", ctypes.c_int32), ("refreshes", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


POLICY = {"midpoint": 0, "damped": 1, "reuse": 2}


class refl_info_t(ctypes.Structure):
    _fields_ = [("ns_steps", ctypes.c_int32), ("polish_sweeps", ctypes.c_int32),
                ("cg_iters", ctypes.c_int32), ("index_j", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("s", ctypes.c_double),
                ("alpha", ctypes.c_double), ("lam_k", ctypes.c_double),
                ("lam_k1", ctypes.c_double), ("eps", ctypes.c_double),
                ("margin", ctypes.c_double), ("resid_fro", ctypes.c_double),
                ("trace", ctypes.c_double), ("commutator_fro", ctypes.c_double),
                ("dk_bound", ctypes.c_double), ("ms_setup", ctypes.c_double),
                ("ms_bulk", ctypes.c_double), ("ms_polish", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("ms_gemm", ctypes.c_double),
                ("gemm_launches", ctypes.c_int32), ("rho", ctypes.c_double),
                ("gamma", ctypes.c_double), ("bulk_tile", ctypes.c_int32),
                ("bulk_words", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_loaded = {}


def load(path: str = None):
    """The current library: ``librefl.so`` unless ``path`` names another
    build (``DEBUG_LIB_PATH``), which then becomes current; each file is
    opened once and its C signatures declared.  Raises if the file is absent.
    Handles remember the library that created them."""
    global _lib
    if path is None:
        if _lib is not None:
            return _lib
        path = LIB_PATH
    if path in _loaded:
        _lib = _loaded[path]
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2605_24840_amd.build.build()")
    lib = ctypes.CDLL(path)
    H = ctypes.c_void_p
    i64, i32, u64, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
    P = ctypes.POINTER
    sig = {
        "refl_params_default": [P(refl_params_t)],
        "refl_create": [P(H), ctypes.c_int, vp],
        "refl_destroy": [H],
        "refl_set_stream": [H, vp],
        "refl_workspace_size": [H, i64, P(refl_params_t), P(ctypes.c_size_t)],
        "refl_set_workspace": [H, vp, ctypes.c_size_t],
        "refl_estimate_shift": [H, i64, vp, i64, i32, i32, u64, P(dbl), P(dbl), P(dbl), P(dbl), P(dbl)],
        "refl_sign": [H, i64, vp, i64, P(refl_params_t), vp, i64, P(refl_info_t)],
        "refl_sign_noalloc": [H, i64, vp, i64, P(refl_params_t), vp, i64, P(refl_info_t)],
        "refl_apply": [H, i64, vp, i64, i64, vp, i64, vp, i64],
        "refl_sign_apply": [H, i64, vp, i64, P(refl_params_t), i64, vp, i64, vp, i64, P(refl_info_t)],
        "refl_sign_batched": [H, i32, P(i64), P(vp), P(i64), P(refl_params_t), P(vp), P(i64),
                              P(refl_info_t), P(ctypes.c_int)],
        "refl_sign_batched_workspace_size": [H, i32, P(i64), P(refl_params_t), P(ctypes.c_size_t)],
        "refl_sign_grad": [H, i64, vp, i64, P(refl_params_t), vp, i64, vp, i64, P(dbl), vp, i64,
                           P(refl_info_t)],
        "refl_policy_create": [H, P(refl_policy_params_t), P(vp)],
        "refl_policy_destroy": [vp],
        "refl_policy_shift": [H, vp, i64, vp, i64, P(dbl), P(refl_policy_info_t)],
        "refl_status_string": [ctypes.c_int],
        "refl_last_error": [H],
        "refl_debug_build": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name in ("refl_status_string", "refl_last_error") else ctypes.c_int
    _loaded[path] = lib
    _lib = lib
    return lib


# ---------------------------------------------------------------- C names
def refl_params_default():
    p = refl_params_t()
    _check(None, load().refl_params_default(ctypes.byref(p)))
    return p


def refl_create(device: int = 0, stream: int = 0):
    h = ctypes.c_void_p()
    st = load().refl_create(ctypes.byref(h), device, ctypes.c_void_p(stream))
    if st != REFL_OK:
        raise ReflError(st, "refl_create failed")
    return h


def refl_destroy(h):
    return load().refl_destroy(h)


def refl_set_stream(h, stream: int):
    return _check(h, load().refl_set_stream(h, ctypes.c_void_p(stream)))


def refl_workspace_size(h, d: int, params) -> int:
    n = ctypes.c_size_t()
    _check(h, load().refl_workspace_size(h, d, ctypes.byref(params), ctypes.byref(n)))
    return n.value


def refl_set_workspace(h, ptr: int, nbytes: int):
    return _check(h, load().refl_set_workspace(h, ctypes.c_void_p(ptr), nbytes))


def refl_sign(h, d, H_ptr, ldh, params, R_ptr, ldr, info=None, check=True):
    info = info if info is not None else refl_info_t()
    st = load().refl_sign(h, d, ctypes.c_void_p(H_ptr), ldh, ctypes.byref(params),
                          ctypes.c_void_p(R_ptr), ldr, ctypes.byref(info))
    if check:
        _check(h, st)
    return st, info


def refl_sign_noalloc(h, d, H_ptr, ldh, params, R_ptr, ldr, info=None, check=True):
    info = info if info is not None else refl_info_t()
    st = load().refl_sign_noalloc(h, d, ctypes.c_void_p(H_ptr), ldh, ctypes.byref(params),
                                  ctypes.c_void_p(R_ptr), ldr, ctypes.byref(info))
    if check:
        _check(h, st)
    return st, info


def refl_apply(h, d, R_ptr, ldr, nrhs, V_ptr, ldv, Y_ptr, ldy):
    return _check(h, load().refl_apply(h, d, ctypes.c_void_p(R_ptr), ldr, nrhs,
                                       ctypes.c_void_p(V_ptr), ldv, ctypes.c_void_p(Y_ptr), ldy))


def refl_sign_apply(h, d, H_ptr, ldh, params, nrhs, V_ptr, ldv, Y_ptr, ldy, info=None, check=True):
    info = info if info is not None else refl_info_t()
    st = load().refl_sign_apply(h, d, ctypes.c_void_p(H_ptr), ldh, ctypes.byref(params), nrhs,
                                ctypes.c_void_p(V_ptr), ldv, ctypes.c_void_p(Y_ptr), ldy,
                                ctypes.byref(info))
    if check:
        _check(h, st)
    return st, info


def refl_estimate_shift(h, d, H_ptr, ldh, k, steps=0, seed=0, check=True):
    out = [ctypes.c_double() for _ in range(5)]
    st = load().refl_estimate_shift(h, d, ctypes.c_void_p(H_ptr), ldh, k, steps, seed,
                                    *[ctypes.byref(o) for o in out])
    if check:
        _check(h, st)
    return st, tuple(o.value for o in out)


def refl_sign_batched(h, ds, H_ptrs, ldhs, params, R_ptrs, ldrs, check=True):
    """C call over host arrays; returns ``(status, [per-problem status], [info])``."""
    n = len(ds)
    i64a = ctypes.c_int64 * n
    vpa = ctypes.c_void_p * n
    pa = (refl_params_t * n)(*params)
    infos = (refl_info_t * n)()
    sts = (ctypes.c_int * n)()
    st = load().refl_sign_batched(h, n, i64a(*ds), vpa(*H_ptrs), i64a(*ldhs), pa, vpa(*R_ptrs),
                                  i64a(*ldrs), infos, sts)
    if check:
        _check(h, st)
    return st, list(sts), list(infos)


def refl_sign_batched_workspace_size(h, ds, params) -> int:
    n = len(ds)
    nb = ctypes.c_size_t()
    _check(h, load().refl_sign_batched_workspace_size(h, n, (ctypes.c_int64 * n)(*ds),
                                                      (refl_params_t * n)(*params),
                                                      ctypes.byref(nb)))
    return nb.value


def refl_sign_grad(h, d, H_ptr, ldh, params, G_ptr, ldg, grad_ptr, ldgr, R_ptr=None, ldr=0,
                   check=True):
    """C call; returns ``(status, loss, info)``."""
    info = refl_info_t()
    loss = ctypes.c_double()
    st = load().refl_sign_grad(h, d, ctypes.c_void_p(H_ptr), ldh, ctypes.byref(params),
                               ctypes.c_void_p(G_ptr), ldg, ctypes.c_void_p(grad_ptr), ldgr,
                               ctypes.byref(loss), ctypes.c_void_p(R_ptr or 0), ldr,
                               ctypes.byref(info))
    if check:
        _check(h, st)
    return st, loss.value, info


def refl_policy_create(h, mode, k, beta=0.5, clip=0.25, tau=0.5, lanczos_steps=0, seed=0,
                       warm_start=True):
    pp = refl_policy_params_t(POLICY[mode], int(k), float(beta), float(clip), float(tau),
                              int(lanczos_steps), int(seed), int(bool(warm_start)))
    pol = ctypes.c_void_p()
    _check(h, load().refl_policy_create(h, ctypes.byref(pp), ctypes.byref(pol)))
    return pol


def refl_policy_destroy(pol):
    return load().refl_policy_destroy(pol)


def refl_policy_shift(h, pol, d, H_ptr, ldh, check=True):
    """Returns ``(status, s, info)``."""
    s = ctypes.c_double()
    info = refl_policy_info_t()
    st = load().refl_policy_shift(h, pol, d, ctypes.c_void_p(H_ptr), ldh, ctypes.byref(s),
                                  ctypes.byref(info))
    if check:
        _check(h, st)
    return st, s.value, info


class ShiftPolicy:
    """A shift policy over a sequence of Hessians on one handle (torch tensors).
    Keyword arguments are those of ``refl_policy_params_t`` (``warm_start``
    defaults to True here: refreshes start from the previous Ritz block)."""

    def __init__(self, handle, mode, k, **kw):
        self.handle = handle
        self.pol = refl_policy_create(handle.h, mode, k, **kw)

    def shift(self, H, check=True):
        """``(s, info_dict, status)`` for the float64 device tensor H."""
        H = _dev_f64(H)
        self.handle.sync_stream()
        st, s, info = refl_policy_shift(self.handle.h, self.pol, H.shape[0], H.data_ptr(),
                                        H.stride(0), check=check)
        return s, info.as_dict(), st

    def close(self):
        if self.pol is not None:
            refl_policy_destroy(self.pol)
            self.pol = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def refl_status_string(st: int) -> str:
    return load().refl_status_string(st).decode()


def refl_last_error(h) -> str:
    return load().refl_last_error(h).decode()


class ReflError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(h, st):
    if st != REFL_OK:
        raise ReflError(st, refl_last_error(h) if h is not None else "")
    return st


# ------------------------------------------------------------ torch wrapper
class Handle:
    """A library handle bound to a torch device and its current stream."""

    def __init__(self, device=None):
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.lib = load()
        self.h = refl_create(self.device.index or 0, torch.cuda.current_stream(self.device).cuda_stream)
        self._ws = None

    def sync_stream(self):
        import torch
        refl_set_stream(self.h, torch.cuda.current_stream(self.device).cuda_stream)

    def reserve(self, d, params):
        """Give the library a torch-allocated workspace large enough for (d, params)."""
        import torch
        n = refl_workspace_size(self.h, d, params)
        if self._ws is None or self._ws.numel() < n + 256:
            self._ws = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        ptr = self._ws.data_ptr()
        ptr = (ptr + 255) // 256 * 256
        refl_set_workspace(self.h, ptr, n)

    def close(self):
        if self.h is not None:
            self.lib.refl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(k, s=None, precision="fp64", tol=None, max_iter=100, fixed_steps=0, words=2,
                alpha=None, polish_sweeps=2, cg_tol=1e-6, cg_max_iter=400, lanczos_steps=0, seed=0,
                timing=False, scale=None, grad_mode="reverse", ckpt_every=0, cg_prec="auto",
                check_symmetric=False, sym_tol=0.0, words_max=3):
    """refl_params_t from keyword arguments.  s=None estimates the shift by
    block Lanczos; scale is "inf" (default), "given" (with alpha), "lanczos"
    (1.05 times the Lanczos spectral-radius estimate) or "fro"; k=0 with a
    given s reports the certified index instead of testing one;
    check_symmetric reads H in full and rejects max|H - H^T| > sym_tol max|H|;
    words_max bounds the MIXED bulk's escalation to more words per operand."""
    p = refl_params_default()
    p.k = int(k)
    p.shift_mode = SHIFT["lanczos"] if s is None else SHIFT["given"]
    p.s = 0.0 if s is None else float(s)
    p.precision = PRECISION[precision]
    if tol is not None:
        p.tol = float(tol)
    elif precision == "mixed":
        p.tol = 0.0
    p.max_iter = int(max_iter)
    p.fixed_steps = int(fixed_steps)
    p.words = int(words)
    if alpha is not None:
        p.scale_mode = SCALE["given"]
        p.alpha = float(alpha)
    if scale is not None:
        p.scale_mode = SCALE[scale]
    p.polish_sweeps = int(polish_sweeps)
    p.cg_tol = float(cg_tol)
    p.cg_max_iter = int(cg_max_iter)
    p.lanczos_steps = int(lanczos_steps)
    p.seed = int(seed)
    p.timing = (1 if timing else 0) if isinstance(timing, bool) else int(timing)
    p.grad_mode = GRAD_MODE[grad_mode]
    p.ckpt_every = int(ckpt_every)
    p.cg_f32 = CG_PREC[cg_prec]
    p.check_symmetric = 1 if check_symmetric else 0
    p.sym_tol = float(sym_tol)
    p.words_max = int(words_max)
    return p


def _dev_f64(t):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 tensor on a ROCm device")
    return t


def sign(H, k, s=None, handle=None, out=None, check=True, **kw):
    """R_k = sgn(H - sI) for a float64 device tensor H (upper triangle read).

    Returns ``(R, info_dict, status)``."""
    import torch
    H = _dev_f64(H)
    d = H.shape[0]
    if H.dim() != 2 or H.shape[1] < d or H.stride(1) != 1:
        raise ValueError("H must be d x d (or d x ld) with unit column stride")
    h = handle or Handle(H.device)
    h.sync_stream()
    p = make_params(k, s, **kw)
    R = out if out is not None else torch.empty((d, d), dtype=torch.float64, device=H.device)
    st, info = refl_sign(h.h, d, H.data_ptr(), H.stride(0), p, R.data_ptr(), R.stride(0), check=check)
    return R, info.as_dict(), st


def sign_noalloc(H, k, s=None, handle=None, out=None, check=True, **kw):
    """As ``sign``, through refl_sign_noalloc: the library's fixed device
    scratch is the workspace (no allocation inside the call).  ``out`` may be
    preallocated.  Returns ``(R, info_dict, status)``."""
    import torch
    H = _dev_f64(H)
    d = H.shape[0]
    if H.dim() != 2 or H.shape[1] < d or H.stride(1) != 1:
        raise ValueError("H must be d x d (or d x ld) with unit column stride")
    h = handle or Handle(H.device)
    h.sync_stream()
    p = make_params(k, s, **kw)
    R = out if out is not None else torch.empty((d, d), dtype=torch.float64, device=H.device)
    st, info = refl_sign_noalloc(h.h, d, H.data_ptr(), H.stride(0), p, R.data_ptr(), R.stride(0),
                                 check=check)
    return R, info.as_dict(), st


def apply(R, V, handle=None):
    """Y = R V for a d x d float64 R and a d x nrhs (or length-d) float64 V."""
    import torch
    R = _dev_f64(R)
    V = _dev_f64(V)
    vec = V.dim() == 1
    Vc = V.reshape(-1, 1) if vec else V
    d, nrhs = Vc.shape
    Vcm = Vc.t().contiguous()   # column-major d x nrhs == row-major nrhs x d
    Ycm = torch.empty_like(Vcm)
    h = handle or Handle(R.device)
    h.sync_stream()
    refl_apply(h.h, d, R.data_ptr(), R.stride(0), nrhs, Vcm.data_ptr(), d, Ycm.data_ptr(), d)
    Y = Ycm.t()
    return Y.reshape(-1) if vec else Y.contiguous()


def sign_apply(H, V, k, s=None, handle=None, check=True, **kw):
    """Y = R_k V without materialising R.  Returns ``(Y, info_dict, status)``."""
    import torch
    H = _dev_f64(H)
    V = _dev_f64(V)
    vec = V.dim() == 1
    Vc = V.reshape(-1, 1) if vec else V
    d, nrhs = Vc.shape
    Vcm = Vc.t().contiguous()
    Ycm = torch.empty_like(Vcm)
    h = handle or Handle(H.device)
    h.sync_stream()
    p = make_params(k, s, **kw)
    st, info = refl_sign_apply(h.h, d, H.data_ptr(), H.stride(0), p, nrhs, Vcm.data_ptr(), d,
                               Ycm.data_ptr(), d, check=check)
    Y = Ycm.t()
    return (Y.reshape(-1) if vec else Y.contiguous()), info.as_dict(), st


class BatchedCall:
    """The marshalled arguments of one refl_sign_batched call, built once and
    reused (the same H and R buffers solved repeatedly, e.g. by an outer
    iteration that updates the matrices in place)."""

    def __init__(self, Hs, ks, ss, outs, **kw):
        n = len(Hs)
        per = {key: kw.pop(key) for key in ("alpha", "tol", "max_iter", "fixed_steps")
               if isinstance(kw.get(key), (list, tuple))}
        params = [make_params(ks[p], ss[p], **kw, **{key: v[p] for key, v in per.items()})
                  for p in range(n)]
        i64a = ctypes.c_int64 * n
        vpa = ctypes.c_void_p * n
        self.n = n
        self.d = i64a(*[H.shape[0] for H in Hs])
        self.H = vpa(*[H.data_ptr() for H in Hs])
        self.ldh = i64a(*[H.stride(0) for H in Hs])
        self.params = (refl_params_t * n)(*params)
        self.R = vpa(*[R.data_ptr() for R in outs])
        self.ldr = i64a(*[R.stride(0) for R in outs])
        self.infos = (refl_info_t * n)()
        self.status = (ctypes.c_int * n)()
        self._keep = (Hs, outs)

    def run(self, h, check=True):
        """Returns the call's status; per-problem results in .infos / .status."""
        st = load().refl_sign_batched(h, self.n, self.d, self.H, self.ldh, self.params, self.R,
                                      self.ldr, self.infos, self.status)
        if check:
            _check(h, st)
        return st


def sign_batched(Hs, ks, ss, handle=None, outs=None, check=True, **kw):
    """R_k = sgn(H - sI) for a list of float64 device tensors in one call.

    ``ks`` and ``ss`` give each problem's index and (given) shift; the other
    keywords are make_params' and apply to every problem (``alpha``, ``tol``,
    ``max_iter`` and ``fixed_steps`` may also be lists).  Returns
    ``(Rs, [info_dict], [status], status)``."""
    import torch
    n = len(Hs)
    if not (len(ks) == len(ss) == n) or n == 0:
        raise ValueError("Hs, ks and ss must be non-empty and of equal length")
    for H in Hs:
        _dev_f64(H)
        if H.dim() != 2 or H.shape[1] < H.shape[0] or H.stride(1) != 1:
            raise ValueError("each H must be d x d (or d x ld) with unit column stride")
    h = handle or Handle(Hs[0].device)
    h.sync_stream()
    Rs = outs if outs is not None else [torch.empty((H.shape[0], H.shape[0]), dtype=torch.float64,
                                                    device=H.device) for H in Hs]
    call = BatchedCall(Hs, ks, ss, Rs, **kw)
    st = call.run(h.h, check=check)
    return Rs, [i.as_dict() for i in call.infos], list(call.status), st


def sign_grad(H, G, k, s, handle=None, with_R=False, check=True, **kw):
    """Gradient of L = <G, R_m(H)> over symmetric perturbations of H (s and
    the scale fixed).  Returns ``(grad, loss, R or None, info_dict, status)``."""
    import torch
    H = _dev_f64(H)
    G = _dev_f64(G)
    d = H.shape[0]
    if G.shape[0] != d or G.stride(1) != 1 or H.stride(1) != 1:
        raise ValueError("H and G must be d x d with unit column stride")
    h = handle or Handle(H.device)
    h.sync_stream()
    p = make_params(k, s, **kw)
    grad = torch.empty((d, d), dtype=torch.float64, device=H.device)
    R = torch.empty((d, d), dtype=torch.float64, device=H.device) if with_R else None
    st, loss, info = refl_sign_grad(h.h, d, H.data_ptr(), H.stride(0), p, G.data_ptr(), G.stride(0),
                                    grad.data_ptr(), grad.stride(0),
                                    R.data_ptr() if R is not None else None,
                                    R.stride(0) if R is not None else 0, check=check)
    return grad, loss, R, info.as_dict(), st


def _reflsign_class():
    import torch

    class ReflSign(torch.autograd.Function):
        """R = sgn(H - sI) (the prescribed-index reflector of refl_sign) as an
        autograd Function.  forward runs refl_sign; backward runs
        refl_sign_grad with G = grad_R (the forward iteration is recomputed,
        so nothing but H is kept) and returns the symmetric gradient: the
        derivative along symmetric perturbations of H, s and the scale held
        fixed.  Precision "fp64" or "fp32" for a differentiable call."""

        @staticmethod
        def forward(ctx, H, k, s, kw):
            kw = dict(kw or {})
            R, info, st = sign(H, k, s, **kw)
            ctx.save_for_backward(H)
            ctx.k, ctx.s, ctx.kw = k, s, kw
            return R

        @staticmethod
        def backward(ctx, gR):
            (H,) = ctx.saved_tensors
            kw = dict(ctx.kw)
            handle = kw.pop("handle", None)
            grad, _, _, _, _ = sign_grad(H, gR.contiguous(), ctx.k, ctx.s, handle=handle, **kw)
            return grad, None, None, None

    return ReflSign


def __getattr__(name):
    if name == "ReflSign":
        cls = _reflsign_class()
        globals()["ReflSign"] = cls
        return cls
    raise AttributeError(name)


def estimate_shift(H, k, steps=0, seed=0, handle=None, check=True):
    """Block-Lanczos midpoint shift: returns ``(s, lam_k, lam_k1, eps, rho, status)``."""
    H = _dev_f64(H)
    d = H.shape[0]
    h = handle or Handle(H.device)
    h.sync_stream()
    st, vals = refl_estimate_shift(h.h, d, H.data_ptr(), H.stride(0), k, steps, seed, check=check)
    return vals + (st,)


def nan():
    return math.nan
