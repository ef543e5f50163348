"""Radial-SVD rotational image alignment on MI355X (gfx950).

Thin ctypes binding of ``libradsvd.so`` (C ABI in ``include/radsvd.h``).
The functions below carry the C names and only marshal arguments: every step
of the computation runs in the library's HIP kernels.  PyTorch supplies
device memory (workspaces, outputs) and the current stream.

If the library has not been built this module raises on first use; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

__all__ = [
    "RadsvdError", "FP64", "FP32", "BF16", "BF16X3", "OUT_BEST", "OUT_LSE", "OUT_FULL",
    "align_prepare_workspace", "align_prepare", "align_pairs", "align_backward_workspace",
    "align_pairs_backward", "align_batched_workspace", "align_pairs_batched",
    "align_pairs_batched_noalloc", "align_get_U",
    "align_set_tile", "align_set_waves", "align_refine_rotation", "align_pairs_list", "align_top_targets",
    "align_landscape_metrics", "align_plan_destroy", "radsvd_last_error", "library_path", "Plan",
    "PRECISIONS", "RadialAlignLSE", "pairs_batched", "RADSVD_NOALLOC_MAX_JOBS",
]

FP64, FP32, BF16, BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16x3": BF16X3}
OUT_BEST, OUT_LSE, OUT_FULL = 1, 2, 4
RADSVD_NOALLOC_MAX_JOBS = 2048   # include/radsvd.h
_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "WORKSPACE", 4: "DEVICE"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "libradsvd.so")
_lib = None


class RadsvdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"radsvd {_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("Q", ctypes.c_int), ("H", ctypes.c_int), ("T", ctypes.c_int),
                ("k", ctypes.POINTER(ctypes.c_double)), ("w", ctypes.POINTER(ctypes.c_double)),
                ("delta", ctypes.POINTER(ctypes.c_double)), ("prec", ctypes.c_int),
                ("hermitian", ctypes.c_int), ("products", ctypes.c_int), ("sigma_delta", ctypes.c_double)]


class _JobOut(ctypes.Structure):
    _fields_ = [("best_score", ctypes.c_void_p), ("best_m", ctypes.c_void_p), ("best_t", ctypes.c_void_p)]


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2202_07235_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, f32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_size_t
    PP = ctypes.POINTER(_Problem)
    L.align_prepare_workspace.argtypes = [PP, i32, i32]
    L.align_prepare_workspace.restype = sz
    L.align_prepare.argtypes = [PP, i32, vp, i32, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
    L.align_prepare.restype = i32
    L.align_pairs.argtypes = [vp, i32, f32, vp, vp, vp, vp, vp, vp, vp]
    L.align_pairs.restype = i32
    L.align_backward_workspace.argtypes = [vp]
    L.align_backward_workspace.restype = sz
    L.align_pairs_backward.argtypes = [vp, f32, vp, vp, vp, vp, vp, sz, vp]
    L.align_pairs_backward.restype = i32
    L.align_batched_workspace.argtypes = [i32]
    L.align_batched_workspace.restype = sz
    L.align_pairs_batched.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(_JobOut), vp, sz, vp]
    L.align_pairs_batched.restype = i32
    L.align_pairs_batched_noalloc.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(_JobOut), vp]
    L.align_pairs_batched_noalloc.restype = i32
    L.align_get_U.argtypes = [vp, vp, vp, vp]
    L.align_get_U.restype = i32
    L.align_set_tile.argtypes = [vp, i32]
    L.align_set_tile.restype = i32
    L.align_pairs_list.argtypes = [vp, i32, f32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.align_pairs_list.restype = i32
    L.align_top_targets.argtypes = [i32, i32, vp, i32, vp, vp]
    L.align_top_targets.restype = i32
    L.align_landscape_metrics.argtypes = [ctypes.c_longlong, i32, vp, vp, i32, vp, vp, vp, vp]
    L.align_landscape_metrics.restype = i32
    L.align_refine_rotation.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.align_refine_rotation.restype = i32
    L.align_set_waves.argtypes = [vp, i32]
    L.align_set_waves.restype = i32
    L.align_plan_destroy.argtypes = [vp]
    L.vol_prepare_workspace.argtypes = [vp, i32, i32]
    L.vol_prepare_workspace.restype = sz
    L.vol_prepare.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
    L.vol_prepare.restype = i32
    L.vol_align.argtypes = [vp, i32, vp, vp, vp, vp]
    L.vol_align.restype = i32
    L.vol_get_UV.argtypes = [vp, vp, vp, vp, vp, vp]
    L.vol_get_UV.restype = i32
    L.vol_plan_destroy.argtypes = [vp]
    L.vol_plan_destroy.restype = None
    L.align_plan_destroy.restype = None
    L.radsvd_last_error.argtypes = []
    L.radsvd_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def radsvd_last_error() -> str:
    return _load().radsvd_last_error().decode()


def _check(st: int):
    if st != 0:
        raise RadsvdError(st, radsvd_last_error())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def make_problem(K, Q, H, T, k, w, delta, prec, hermitian, products=3, sigma_delta=0.0):
    """Build the C problem struct; the returned tuple keeps the host arrays
    alive (pass element 0 to the ABI)."""
    k = np.ascontiguousarray(k, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    d = None if delta is None else np.ascontiguousarray(delta, dtype=np.float64).reshape(-1)
    dp = ctypes.POINTER(ctypes.c_double)
    pr = _Problem(K, Q, H, T, k.ctypes.data_as(dp), w.ctypes.data_as(dp),
                  d.ctypes.data_as(dp) if d is not None else ctypes.cast(None, dp),
                  int(prec), int(hermitian), int(products), float(sigma_delta))
    return pr, (k, w, d)


# ---------------------------------------------------------------------------
# same-name wrappers of the C ABI
# ---------------------------------------------------------------------------
def align_prepare_workspace(problem: _Problem, n_img: int, n_tgt: int) -> int:
    n = _load().align_prepare_workspace(ctypes.byref(problem), n_img, n_tgt)
    if n == 0:
        raise RadsvdError(1, radsvd_last_error())
    return n


def align_prepare(problem: _Problem, n_img, A_polar, n_tgt, B_polar, U_in, ws, stream=None) -> ctypes.c_void_p:
    plan = ctypes.c_void_p()
    _check(_load().align_prepare(ctypes.byref(problem), n_img, _ptr(A_polar), n_tgt, _ptr(B_polar),
                                 _ptr(U_in), _ptr(ws), ws.numel() * ws.element_size() if ws is not None else 0,
                                 _stream(stream), ctypes.byref(plan)))
    return plan


def align_pairs(plan, out_flags, inv_sigma2, best_score=None, best_m=None, best_t=None,
                lse_pair=None, lse_img=None, X_full=None, stream=None):
    _check(_load().align_pairs(plan, out_flags, float(inv_sigma2), _ptr(best_score), _ptr(best_m),
                               _ptr(best_t), _ptr(lse_pair), _ptr(lse_img), _ptr(X_full), _stream(stream)))


def align_backward_workspace(plan) -> int:
    return _load().align_backward_workspace(plan)


def align_pairs_backward(plan, inv_sigma2, lse_img, grad_lse_img, grad_B_polar, grad_U, bwd_ws, stream=None):
    nbytes = bwd_ws.numel() * bwd_ws.element_size() if bwd_ws is not None else 0
    _check(_load().align_pairs_backward(plan, float(inv_sigma2), _ptr(lse_img), _ptr(grad_lse_img),
                                        _ptr(grad_B_polar), _ptr(grad_U), _ptr(bwd_ws), nbytes,
                                        _stream(stream)))


def align_batched_workspace(n_jobs: int) -> int:
    n = _load().align_batched_workspace(n_jobs)
    if n == 0:
        raise RadsvdError(1, radsvd_last_error())
    return n


def align_pairs_batched(plans, outs, batch_ws, stream=None):
    """plans: list of plan handles; outs: list of (best_score, best_m, best_t) tensors."""
    n = len(plans)
    arr = (ctypes.c_void_p * n)(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    jo = (_JobOut * n)(*[_JobOut(o[0].data_ptr(), o[1].data_ptr(), o[2].data_ptr()) for o in outs])
    nbytes = batch_ws.numel() * batch_ws.element_size()
    _check(_load().align_pairs_batched(arr, n, jo, _ptr(batch_ws), nbytes, _stream(stream)))


def align_pairs_batched_noalloc(plans, outs, stream=None):
    """As align_pairs_batched, with the library's own device scratch (no workspace)."""
    n = len(plans)
    arr = (ctypes.c_void_p * n)(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    jo = (_JobOut * n)(*[_JobOut(o[0].data_ptr(), o[1].data_ptr(), o[2].data_ptr()) for o in outs])
    _check(_load().align_pairs_batched_noalloc(arr, n, jo, _stream(stream)))


def align_get_U(plan, U_dev=None, lambda_dev=None, stream=None):
    _check(_load().align_get_U(plan, _ptr(U_dev), _ptr(lambda_dev), _stream(stream)))


def align_set_tile(plan, band: int):
    _check(_load().align_set_tile(plan, int(band)))


def align_pairs_list(plan, out_flags, inv_sigma2, pairs, best_score=None, best_m=None, best_t=None,
                     lse_pair=None, X_full=None, stream=None):
    _check(_load().align_pairs_list(plan, out_flags, float(inv_sigma2), int(pairs.shape[0]), _ptr(pairs),
                                    _ptr(best_score), _ptr(best_m), _ptr(best_t), _ptr(lse_pair), _ptr(X_full),
                                    _stream(stream)))


def align_top_targets(score, k: int, cand, stream=None):
    _check(_load().align_top_targets(int(score.shape[0]), int(score.shape[1]), _ptr(score), int(k), _ptr(cand),
                                     _stream(stream)))


def align_landscape_metrics(X_est, X_ref, f, pair_stats, summary, stream=None):
    """X_est, X_ref: device [n_pairs, ...] complex64 or complex128 of equal shape."""
    n = int(X_est.shape[0])
    _check(_load().align_landscape_metrics(n, int(X_est.numel() // n), _ptr(X_est), _ptr(X_ref),
                                           int(X_est.dtype == torch.complex128), _ptr(f), _ptr(pair_stats),
                                           _ptr(summary), _stream(stream)))


def align_refine_rotation(plan, best_m, best_t, R: int, fine_score, fine_m, stream=None):
    _check(_load().align_refine_rotation(plan, _ptr(best_m), _ptr(best_t), int(R), _ptr(fine_score), _ptr(fine_m),
                                         _stream(stream)))


def align_set_waves(plan, waves: int):
    _check(_load().align_set_waves(plan, int(waves)))


def align_plan_destroy(plan):
    if plan:
        _load().align_plan_destroy(plan)


# ---------------------------------------------------------------------------
# convenience object
# ---------------------------------------------------------------------------
class Plan:
    """A prepared alignment problem.  Holds the device workspace and keeps the
    polar inputs alive (the backward pass reads them)."""

    def __init__(self, A_polar: torch.Tensor, B_polar: torch.Tensor, k, w, delta, H: int,
                 precision: str = "fp32", hermitian: bool = True, products: int = 3,
                 U: torch.Tensor | None = None, stream=None, sigma_delta: float = 0.0):
        prec = PRECISIONS[precision]
        want = torch.complex128 if prec == FP64 else torch.complex64
        for name, X in (("A_polar", A_polar), ("B_polar", B_polar)):
            if not X.is_cuda or X.dtype != want or not X.is_contiguous() or X.dim() != 3:
                raise ValueError(f"{name} must be a contiguous CUDA {want} tensor [n][K][Q]")
        n_img, K, Q = A_polar.shape
        n_tgt = B_polar.shape[0]
        delta = np.zeros((1, 2)) if delta is None else np.asarray(delta, dtype=np.float64).reshape(-1, 2)
        T = delta.shape[0]
        self.K, self.Q, self.H, self.T = K, Q, H, T
        self.n_img, self.n_tgt = n_img, n_tgt
        self.precision, self.prec, self.hermitian = precision, prec, hermitian
        self.products = products
        self.sigma_delta = float(sigma_delta)
        self.problem, self._keep = make_problem(K, Q, H, T, k, w, delta, prec, hermitian, products, sigma_delta)
        nbytes = align_prepare_workspace(self.problem, n_img, n_tgt)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=A_polar.device)
        self.A, self.B = A_polar, B_polar
        self.U_in = None if U is None else U.to(device=A_polar.device, dtype=torch.float64).contiguous()
        self.handle = align_prepare(self.problem, n_img, A_polar, n_tgt, B_polar, self.U_in, self.ws, stream)
        self.device = A_polar.device
        self.band = 0
        self.waves = 0

    def close(self):
        """Release the plan handle now (the workspace goes with the object)."""
        self.__del__()

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                align_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def pairs(self, out: str = "best", inv_sigma2: float = 1.0, stream=None, outputs: dict | None = None):
        flags = 0
        for tok in out.split("+"):
            flags |= {"best": OUT_BEST, "lse": OUT_LSE, "full": OUT_FULL}[tok]
        dev = self.device
        na, nb = self.n_img, self.n_tgt
        o = outputs if outputs is not None else {}
        if flags & OUT_BEST and "best_score" not in o:
            o["best_score"] = torch.empty((na, nb), dtype=torch.float32, device=dev)
            o["best_m"] = torch.empty((na, nb), dtype=torch.int32, device=dev)
            o["best_t"] = torch.empty((na, nb), dtype=torch.int32, device=dev)
        if flags & OUT_LSE and "lse_pair" not in o:
            o["lse_pair"] = torch.empty((na, nb), dtype=torch.float32, device=dev)
            o["lse_img"] = torch.empty((na,), dtype=torch.float32, device=dev)
        if flags & OUT_FULL and "X" not in o:
            dt = torch.complex128 if self.prec == FP64 else torch.complex64
            o["X"] = torch.empty((na, nb, self.T, self.Q), dtype=dt, device=dev)
        align_pairs(self.handle, flags, inv_sigma2, o.get("best_score"), o.get("best_m"), o.get("best_t"),
                    o.get("lse_pair"), o.get("lse_img"), o.get("X"), stream)
        return o

    def U_lambda(self, stream=None):
        U = torch.empty((self.K, self.K), dtype=torch.float64, device=self.device)
        lam = torch.empty((self.K,), dtype=torch.float64, device=self.device)
        align_get_U(self.handle, U, lam, stream)
        return U, lam

    def set_tile(self, band: int):
        """Tile order of the fast path: image tiles per XCD band (0 = default)."""
        align_set_tile(self.handle, band)
        self.band = band

    def pairs_list(self, pairs: torch.Tensor, out: str = "best", inv_sigma2: float = 1.0, stream=None) -> dict:
        """align_pairs for the listed (image, target) pairs, pairs: device
        [n][2] int32; outputs indexed by list position."""
        flags = 0
        for tok in out.split("+"):
            flags |= {"best": OUT_BEST, "lse": OUT_LSE, "full": OUT_FULL}[tok]
        n, dev = int(pairs.shape[0]), self.device
        o = {}
        if flags & OUT_BEST:
            o["best_score"] = torch.empty(n, dtype=torch.float32, device=dev)
            o["best_m"] = torch.empty(n, dtype=torch.int32, device=dev)
            o["best_t"] = torch.empty(n, dtype=torch.int32, device=dev)
        if flags & OUT_LSE:
            o["lse_pair"] = torch.empty(n, dtype=torch.float32, device=dev)
        if flags & OUT_FULL:
            dt = torch.complex128 if self.prec == FP64 else torch.complex64
            o["X"] = torch.empty((n, self.T, self.Q), dtype=dt, device=dev)
        align_pairs_list(self.handle, flags, inv_sigma2, pairs.contiguous(), o.get("best_score"), o.get("best_m"),
                         o.get("best_t"), o.get("lse_pair"), o.get("X"), stream)
        return o

    def refine_rotation(self, best: dict, R: int, stream=None) -> dict:
        """Best rotation on the R-times finer grid around each pair's grid
        maximum (``align_refine_rotation``); ``best`` holds best_m and best_t
        of a BEST output.  Returns fine_score, fine_m and gamma (radians)."""
        fs = torch.empty((self.n_img, self.n_tgt), dtype=torch.float32, device=self.device)
        fm = torch.empty((self.n_img, self.n_tgt), dtype=torch.int32, device=self.device)
        align_refine_rotation(self.handle, best["best_m"], best["best_t"], R, fs, fm, stream)
        return {"fine_score": fs, "fine_m": fm, "gamma": fm.to(torch.float64) * (2.0 * np.pi / (R * self.Q))}

    def set_waves(self, waves: int):
        """Waves per CU of the fast path: 4, 8 or 0 (default); raises
        RadsvdError (UNSUPPORTED) where this plan has no such layout."""
        align_set_waves(self.handle, waves)
        self.waves = waves

    def backward(self, inv_sigma2: float, lse_img: torch.Tensor, grad_lse_img: torch.Tensor,
                 want_B: bool = True, want_U: bool = True, stream=None):
        nbytes = align_backward_workspace(self.handle)
        if nbytes == 0:
            raise RadsvdError(2, radsvd_last_error() or "backward not available for this plan")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        gB = torch.empty_like(self.B) if want_B else None
        gU = torch.empty((self.K, self.H), dtype=torch.float64, device=self.device) if want_U else None
        align_pairs_backward(self.handle, inv_sigma2, lse_img.contiguous(), grad_lse_img.contiguous(),
                             gB, gU, ws, stream)
        return gB, gU


class RadialAlignLSE(torch.autograd.Function):
    """Soft-alignment score with a hand-written backward.

        lse_img = RadialAlignLSE.apply(A_polar, B_polar, U, k, w, delta, inv_sigma2, precision, hermitian)

    Forward: ``align_prepare`` with the caller's U [K][H] (FP64) and
    ``align_pairs`` with the log-sum-exp output; returns lse_img [n_img] (f32):
    lse_img[a] = log sum_{b,t,m} exp(inv_sigma2 Re X[a][b][t][m]).
    Backward: ``align_pairs_backward``; gradients flow to B_polar (complex,
    dL/dRe + i dL/dIm, every entry free) and U (a free real matrix).  A_polar,
    the grid and the scalars get none.
    """

    @staticmethod
    def forward(ctx, A_polar, B_polar, U, k, w, delta, inv_sigma2=1.0, precision="fp32", hermitian=True):
        plan = Plan(A_polar.detach().contiguous(), B_polar.detach().contiguous(), k, w, delta, U.shape[1],
                    precision=precision, hermitian=hermitian, U=U.detach())
        o = plan.pairs("lse", inv_sigma2=inv_sigma2)
        ctx.plan = plan
        ctx.inv_sigma2 = float(inv_sigma2)
        ctx.U_dtype = U.dtype
        ctx.save_for_backward(o["lse_img"])
        return o["lse_img"].clone()

    @staticmethod
    def backward(ctx, grad_lse_img):
        (lse_img,) = ctx.saved_tensors
        want_B, want_U = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gB = gU = None
        if want_B or want_U:
            gB, gU = ctx.plan.backward(ctx.inv_sigma2, lse_img, grad_lse_img.to(torch.float32).contiguous(),
                                       want_B=want_B, want_U=want_U)
        if gU is not None:
            gU = gU.to(ctx.U_dtype)
        return None, gB, gU, None, None, None, None, None, None


def pairs_batched(plans, outputs=None, batch_ws=None, stream=None):
    """Best (score, m, t) of every job in one persistent launch
    (``align_pairs_batched``).  ``plans``: list of ``Plan``; returns (or fills)
    one dict per job with best_score / best_m / best_t."""
    dev = plans[0].device
    if outputs is None:
        outputs = [{"best_score": torch.empty((p.n_img, p.n_tgt), dtype=torch.float32, device=dev),
                    "best_m": torch.empty((p.n_img, p.n_tgt), dtype=torch.int32, device=dev),
                    "best_t": torch.empty((p.n_img, p.n_tgt), dtype=torch.int32, device=dev)} for p in plans]
    if batch_ws is None:
        batch_ws = torch.empty(align_batched_workspace(len(plans)), dtype=torch.uint8, device=dev)
    align_pairs_batched([p.handle for p in plans],
                        [(o["best_score"], o["best_m"], o["best_t"]) for o in outputs], batch_ws, stream)
    return outputs
