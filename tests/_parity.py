"""Shared helpers of the GPU parity tests: run the library on a synthetic
problem and the FP64 oracle on exactly the same (upcast) inputs and the
library's own U (principal vectors are only defined up to sign / rotation
within degenerate eigenspaces, so the landscape is compared for one U and U
is compared separately)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2202_07235_amd as rs
import synth


def to_device(P: synth.Problem, precision: str):
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    A = P.A.to(device="cuda", dtype=dt).contiguous()
    B = P.B.to(device="cuda", dtype=dt).contiguous()
    return A, B


def host_inputs(A: torch.Tensor, B: torch.Tensor):
    """The exact values the GPU received, as complex128 host arrays."""
    return A.cpu().to(torch.complex128).numpy(), B.cpu().to(torch.complex128).numpy()


def rel_err(X, ref):
    """A11: max over (t,m) |X - ref| / max |ref| per pair, max over pairs."""
    X = np.asarray(X)
    ref = np.asarray(ref)
    num = np.abs(X - ref).reshape(X.shape[0], X.shape[1], -1).max(axis=-1)
    den = np.abs(ref).reshape(X.shape[0], X.shape[1], -1).max(axis=-1)
    return float(np.max(num / np.maximum(den, 1e-300)))


def argmax_agrees(Xor, m, t, rel):
    """A11: indices equal, or the oracle value at the GPU argmax within
    rel * max|X| of the oracle maximum (near-ties)."""
    R = np.asarray(Xor).real
    T, Q = R.shape[-2:]
    flat = R.reshape(-1, T * Q)
    best = flat.max(axis=1)
    scale = np.abs(flat).max(axis=1)
    idx = (np.asarray(t).reshape(-1) * Q + np.asarray(m).reshape(-1))
    got = flat[np.arange(flat.shape[0]), idx]
    ok = (idx == flat.argmax(axis=1)) | (best - got <= 4 * rel * scale)
    return ok


def oracle_landscape_for(plan: rs.Plan, A_h, B_h, P: synth.Problem, pairs=None):
    U, lam = plan.U_lambda()
    U = U.cpu().numpy()
    X = oracle.landscape(A_h, B_h, U, plan.H, P.k, P.w, P.delta, pairs=pairs)
    return X, U, lam.cpu().numpy()
