"""Rotational volume alignment with principal volumes (paper section 4).

Thin binding of the ``vol_*`` entry points of ``libradsvd.so``: argument
marshalling only.  Volumes are spherical-harmonic coefficients on K shells,
complex [n][K][(L+1)^2] (index l^2 + l + m), on the GPU; the landscape is
X[a][b][ib][m1'][m2'] = <A_a, R_tau B_b> at tau = (gamma, beta, alpha) =
(2 pi m2'/M, beta[ib], 2 pi m1'/M), M = 2L + 1.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import FP32, FP64, OUT_BEST, OUT_FULL, PRECISIONS, _check, _load, _ptr, _stream

__all__ = ["VolPlan", "vol_prepare_workspace", "vol_prepare", "vol_align", "vol_get_UV", "vol_plan_destroy",
           "make_vol_problem", "euler_angles"]


class _VolProblem(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("L", ctypes.c_int), ("H_C", ctypes.c_int), ("H_D", ctypes.c_int),
                ("n_beta", ctypes.c_int), ("w", ctypes.POINTER(ctypes.c_double)),
                ("beta", ctypes.POINTER(ctypes.c_double)), ("prec", ctypes.c_int), ("real_volumes", ctypes.c_int)]


def make_vol_problem(K, L, H_C, H_D, w, beta, prec, real=0):
    """The C problem struct and the host arrays it points into (keep both)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    pr = _VolProblem(K, L, H_C, H_D, len(beta), w.ctypes.data_as(dp), beta.ctypes.data_as(dp), prec, int(real))
    return pr, (w, beta)


def vol_prepare_workspace(problem: _VolProblem, n_vol: int, n_tgt: int) -> int:
    n = _load().vol_prepare_workspace(ctypes.byref(problem), n_vol, n_tgt)
    if n == 0:
        _check(1)
    return n


def vol_prepare(problem, n_vol, A_sh, n_tgt, B_sh, U_in, V_in, ws, stream=None):
    h = ctypes.c_void_p()
    _check(_load().vol_prepare(ctypes.byref(problem), n_vol, _ptr(A_sh), n_tgt, _ptr(B_sh), _ptr(U_in), _ptr(V_in),
                               _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream), ctypes.byref(h)))
    return h


def vol_align(plan, out_flags, best_score=None, best_idx=None, X_full=None, stream=None):
    _check(_load().vol_align(plan, out_flags, _ptr(best_score), _ptr(best_idx), _ptr(X_full), _stream(stream)))


def vol_get_UV(plan, U=None, lamC=None, V=None, lamD=None, stream=None):
    _check(_load().vol_get_UV(plan, _ptr(U), _ptr(lamC), _ptr(V), _ptr(lamD), _stream(stream)))


def vol_plan_destroy(plan):
    _load().vol_plan_destroy(plan)


def euler_angles(best_idx, beta, L: int):
    """Euler angles (gamma, beta, alpha) of the rotations R_z(alpha) R_y(beta)
    R_z(gamma) that vol_align's best_idx {ib, m1', m2'} name: alpha = 2 pi m1'/M,
    gamma = 2 pi m2'/M, M = 2L + 1, beta = beta[ib].  Host arithmetic on the
    indices only; entries of -1 (pairs without a best) give NaN."""
    idx = np.asarray(best_idx.cpu() if isinstance(best_idx, torch.Tensor) else best_idx)
    beta = np.asarray(beta, dtype=np.float64)
    M = 2 * L + 1
    ok = idx[..., 0] >= 0
    ib = np.where(ok, idx[..., 0], 0)
    alpha = np.where(ok, 2.0 * np.pi * idx[..., 1] / M, np.nan)
    gamma = np.where(ok, 2.0 * np.pi * idx[..., 2] / M, np.nan)
    bet = np.where(ok, beta[ib], np.nan)
    return gamma, bet, alpha


class VolPlan:
    """A prepared volume-alignment problem (holds the device workspace)."""

    def __init__(self, A_sh: torch.Tensor, B_sh: torch.Tensor, w, L: int, H_C: int, H_D: int, beta,
                 precision: str = "fp32", U: torch.Tensor | None = None, V: torch.Tensor | None = None,
                 real: bool = False, stream=None):
        """real=True asserts that every volume and target is real in space
        (conj(A_l^m) = (-1)^(l+m) A_l^-m): X is then real and computed from
        half the orders."""
        prec = PRECISIONS[precision]
        if prec not in (FP32, FP64):
            raise ValueError("volume plans take precision 'fp32' or 'fp64'")
        want = torch.complex128 if prec == FP64 else torch.complex64
        for name, X in (("A_sh", A_sh), ("B_sh", B_sh)):
            if not X.is_cuda or X.dtype != want or not X.is_contiguous() or X.dim() != 3:
                raise ValueError(f"{name} must be a contiguous CUDA {want} tensor [n][K][(L+1)^2]")
            if X.shape[2] != (L + 1) ** 2:
                raise ValueError(f"{name} has {X.shape[2]} coefficients per shell, not (L+1)^2 = {(L + 1) ** 2}")
        self.n_vol, self.K, _ = A_sh.shape
        self.n_tgt = B_sh.shape[0]
        self.L, self.M, self.H_C, self.H_D = L, 2 * L + 1, H_C, H_D
        self.beta = np.asarray(beta, dtype=np.float64).reshape(-1)
        self.n_beta = len(self.beta)
        self.precision, self.prec, self.real = precision, prec, bool(real)
        self.problem, self._keep = make_vol_problem(self.K, L, H_C, H_D, w, self.beta, prec, int(real))
        nbytes = vol_prepare_workspace(self.problem, self.n_vol, self.n_tgt)
        self.device = A_sh.device
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.U_in = None if U is None else U.to(device=self.device, dtype=torch.float64).contiguous()
        self.V_in = None if V is None else V.to(device=self.device, dtype=torch.float64).contiguous()
        self.handle = vol_prepare(self.problem, self.n_vol, A_sh, self.n_tgt, B_sh, self.U_in, self.V_in, self.ws,
                                  stream)

    def close(self):
        self.__del__()

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                vol_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def align(self, out: str = "best", stream=None, outputs: dict | None = None) -> dict:
        flags = 0
        for tok in out.split("+"):
            flags |= {"best": OUT_BEST, "full": OUT_FULL}[tok]
        o = outputs if outputs is not None else {}
        dev, nv, nt = self.device, self.n_vol, self.n_tgt
        if flags & OUT_BEST and "best_score" not in o:
            o["best_score"] = torch.empty((nv, nt), dtype=torch.float32, device=dev)
            o["best_idx"] = torch.empty((nv, nt, 3), dtype=torch.int32, device=dev)
        if flags & OUT_FULL and "X" not in o:
            dt = torch.complex128 if self.prec == FP64 else torch.complex64
            o["X"] = torch.empty((nv, nt, self.n_beta, self.M, self.M), dtype=dt, device=dev)
        vol_align(self.handle, flags, o.get("best_score"), o.get("best_idx"), o.get("X"), stream)
        return o

    def UV(self, stream=None):
        """(U [K][K], eigenvalues of C, V [L+1][L+1], eigenvalues of D), FP64."""
        L1 = self.L + 1
        U = torch.empty((self.K, self.K), dtype=torch.float64, device=self.device)
        lc = torch.empty((self.K,), dtype=torch.float64, device=self.device)
        V = torch.empty((L1, L1), dtype=torch.float64, device=self.device)
        ld = torch.empty((L1,), dtype=torch.float64, device=self.device)
        vol_get_UV(self.handle, U, lc, V, ld, stream)
        return U, lc, V, ld
