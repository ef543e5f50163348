"""Parity of the fused matrix-core Hermitian path (BEST and LSE outputs)
against the FP64 oracle, for every supported angle count Q, every
contraction precision, ragged image/target counts (not multiples of the
8 x 16 tile) and ranks whose padding to a multiple of 8 exercises the
operand padding.

Error bars (derivation in test_gpu_parity): FP32 and split-BF16 with 3 or 6
products: 1e-5 of max|X|; BF16 (one product): 2e-2.  The LSE of
inv_sigma2 * X changes by at most inv_sigma2 * max|dX|, so its tolerance is
4 * tol with inv_sigma2 = 4 / max|X| (plus FP32 rounding of the sum).
"""
import functools

import numpy as np
import pytest
import torch

import oracle
import paper_2202_07235_amd as rs
import synth
from tests._parity import argmax_agrees, host_inputs, to_device

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16x3_6": 1e-5, "bf16": 2e-2}

#          Q    K    H   n_img n_tgt T
CASES = {64: (16, 10, 11, 37, 9),
         96: (24, 12, 9, 20, 9),
         128: (32, 16, 10, 18, 9),
         192: (48, 20, 9, 17, 4),
         256: (64, 16, 12, 20, 9),
         384: (96, 32, 9, 17, 1),
         512: (128, 24, 9, 17, 4)}


@functools.lru_cache(maxsize=None)
def _problem(Q, H=None):
    K, H0, na, nb, T = CASES[Q]
    H = H0 if H is None else H
    cfg = synth.config("fp32", N=Q // 2, K=K, Q=Q, n_img=na, n_tgt=nb, T=T, H=H,
                       n_blobs=8, snr=0.5)
    P = synth.make_problem(cfg, seed=2000 + Q)
    A, B = to_device(P, "fp32")
    A_h, B_h = host_inputs(A, B)
    # U from the library (FP64 eigensolver on the same inputs for every precision)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, H, precision="fp32", hermitian=True)
    U, _ = plan.U_lambda()
    U = U.cpu().numpy()
    X = oracle.landscape(A_h, B_h, U, H, P.k, P.w, P.delta)
    return cfg, P, A, B, X


@pytest.mark.parametrize("Q", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16x3_6", "bf16"])
def test_fast_path_matches_oracle(Q, precision):
    _check_fast(Q, None, precision)


# Ranks on either side of the operand-register limits that decide whether two
# workgroups share a compute unit (and, at Q = 256, whether the MFMA results
# are staged in one buffer or two): Q = 256 with 24 ranks runs two workgroups
# per CU in FP32, BF16 and 3-product bf16x3, one with 6 products; Q = 192 and
# Q = 128 with 32 ranks.
@pytest.mark.parametrize("Q,H", [(256, 24), (192, 32), (128, 32)])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16x3_6", "bf16"])
def test_fast_path_matches_oracle_across_occupancy_limits(Q, H, precision):
    _check_fast(Q, H, precision)


def _check_fast(Q, H, precision):
    cfg, P, A, B, X = _problem(Q, H)
    prec, products = ("bf16x3", 6) if precision == "bf16x3_6" else (precision, 3)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=prec, hermitian=True, products=products)
    s2 = 4.0 / np.abs(X).max()
    o = plan.pairs("best+lse", inv_sigma2=s2)
    torch.cuda.synchronize()
    sc, m, t = (o[k].cpu().numpy() for k in ("best_score", "best_m", "best_t"))
    na, nb = cfg.n_img, cfg.n_tgt
    # A11: errors relative to each pair's own max|X|
    scale = np.abs(X).reshape(na, nb, -1).max(axis=-1)
    assert ((m >= 0) & (m < Q) & (t >= 0) & (t < cfg.T)).all()
    got_at = np.take_along_axis(X.real.reshape(na, nb, -1), (t * Q + m)[..., None], axis=-1)[..., 0]
    err_score = (np.abs(sc - got_at) / scale).max()
    ref_sc, ref_m, ref_t = oracle.best(X)
    err_best = (np.abs(sc - ref_sc) / scale).max()
    tol = TOL[precision]
    print(f"Q={Q} H={cfg.H} {precision}: score err {err_score:.2e}, best err {err_best:.2e}, "
          f"argmax exact {np.mean((m == ref_m) & (t == ref_t)):.3f}")
    assert err_score <= tol
    assert err_best <= tol
    assert argmax_agrees(X, m, t, tol).all()
    lp, li = oracle.lse(X, s2)
    assert np.abs(o["lse_pair"].cpu().numpy() - lp).max() <= 4 * tol + 1e-5
    assert np.abs(o["lse_img"].cpu().numpy() - li).max() <= 4 * tol + 1e-5


def test_fast_path_best_only_and_lse_only_agree_with_combined():
    cfg, P, A, B, X = _problem(128)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="bf16x3", hermitian=True)
    both = plan.pairs("best+lse", inv_sigma2=0.01)
    b = plan.pairs("best")
    l = plan.pairs("lse", inv_sigma2=0.01)
    assert torch.equal(both["best_score"], b["best_score"])
    assert torch.equal(both["best_m"], b["best_m"])
    assert torch.equal(both["lse_pair"], l["lse_pair"])


def test_fast_path_is_deterministic():
    cfg, P, A, B, X = _problem(256)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="bf16x3", hermitian=True)
    o1 = {k: v.clone() for k, v in plan.pairs("best+lse", inv_sigma2=0.01).items()}
    o2 = plan.pairs("best+lse", inv_sigma2=0.01)
    for k in o1:
        assert torch.equal(o1[k], o2[k]), k


def test_fast_path_nan_target_poisons_only_its_pairs():
    cfg, P, A, B, X = _problem(192)
    B2 = B.clone()
    B2[3, 5, 11] = complex(float("nan"), 0.0)
    U = torch.eye(cfg.K, dtype=torch.float64)[:, :cfg.H].contiguous()
    plan = rs.Plan(A, B2, P.k, P.w, P.delta, cfg.H, precision="bf16x3", hermitian=True, U=U)
    o = plan.pairs("best")
    sc, m = o["best_score"].cpu().numpy(), o["best_m"].cpu().numpy()
    assert np.isnan(sc[:, 3]).all() and (m[:, 3] == -1).all()
    others = np.delete(np.arange(cfg.n_tgt), 3)
    assert np.isfinite(sc[:, others]).all() and (m[:, others] >= 0).all()
