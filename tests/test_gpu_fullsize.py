"""Parity at the full workload sizes, in the launch configuration bench.py
times, on sampled pairs the FP64 oracle evaluates one by one:

* FP32 batch workload:  N=128, K=64, Q=256, 1024 x 1024, T=9, H=16;
* precision workload:   N=256, K=128, Q=512, 4096 x 4096, T=9, H=24
  (FP32, BF16x3 with 3 and with 6 products, BF16);
* differentiation workload forward: 2048 noisy images x 256 templates,
  Q=256, T=9, H=16, log-sum-exp per image checked on whole rows.

The oracle gets the exact complex64 inputs the GPU received (upcast) and the
plan's U; U itself is checked against the oracle's kernel C at 1024 targets
(K = 64) and at 4096 targets (K = 128).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_07235_amd as rs
import synth
from tests._parity import argmax_agrees

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16x3_6": 1e-5, "bf16": 2e-2}


def _gen(name, seed, **over):
    cfg = synth.config(name, **over)
    P = synth.make_problem(cfg, seed=seed, device="cuda")
    A = P.A.to(torch.complex64).contiguous()
    B = P.B.to(torch.complex64).contiguous()
    P.A = P.B = None
    torch.cuda.empty_cache()
    return cfg, P, A, B


def _sample_check(cfg, P, A, B, plan, out, npairs=64, seed=0, tol=1e-5):
    rng = np.random.default_rng(seed)
    ia = rng.integers(0, cfg.n_img, npairs)
    ib = rng.integers(0, cfg.n_tgt, npairs)
    ua, inv_a = np.unique(ia, return_inverse=True)
    ub, inv_b = np.unique(ib, return_inverse=True)
    Ah = A[torch.as_tensor(ua, device=A.device)].cpu().to(torch.complex128).numpy()
    Bh = B[torch.as_tensor(ub, device=B.device)].cpu().to(torch.complex128).numpy()
    U, _ = plan.U_lambda()
    U = U.cpu().numpy()
    X = oracle.landscape(Ah, Bh, U, cfg.H, P.k, P.w, P.delta, pairs=list(zip(inv_a, inv_b)))
    sc, m, t = (out[k].cpu().numpy()[ia, ib] for k in ("best_score", "best_m", "best_t"))
    ref_sc, ref_m, ref_t = oracle.best(X[:, None])
    scale = np.abs(X).reshape(npairs, -1).max(axis=1)
    rel = np.abs(sc - ref_sc[:, 0]) / scale
    at = X.real.reshape(npairs, -1)[np.arange(npairs), t * cfg.Q + m]
    rel_at = np.abs(sc - at) / scale
    ok = argmax_agrees(X[:, None], m[:, None], t[:, None], tol)
    return float(rel.max()), float(rel_at.max()), float(ok.mean()), float(np.mean((m == ref_m[:, 0]) & (t == ref_t[:, 0])))


def test_fp32_workload_sampled_pairs_and_U():
    cfg, P, A, B = _gen("fp32", seed=4001)
    for precision in ("fp32", "bf16x3"):
        plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision, hermitian=True)
        out = plan.pairs("best")
        torch.cuda.synchronize()
        rel, rel_at, ok, exact = _sample_check(cfg, P, A, B, plan, out, tol=TOL[precision])
        print(f"fp32 workload {precision}: rel {rel:.2e} at-argmax {rel_at:.2e} agree {ok:.3f} exact {exact:.3f}")
        assert rel <= TOL[precision] and rel_at <= TOL[precision] and ok == 1.0
    # U against the oracle's kernel C built from the same 1024 targets
    _check_U(plan, B, P.w, cfg.Q, cfg.H)


@pytest.mark.parametrize("precision", ["bf16x3", "fp32", "bf16x3_6", "bf16"])
def test_precision_workload_sampled_pairs(precision):
    cfg, P, A, B = _gen("precision", seed=3003)
    prec, products = ("bf16x3", 6) if precision == "bf16x3_6" else (precision, 3)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=prec, hermitian=True, products=products)
    out = plan.pairs("best")
    torch.cuda.synchronize()
    rel, rel_at, ok, exact = _sample_check(cfg, P, A, B, plan, out, tol=TOL[precision])
    print(f"precision workload {precision}: rel {rel:.2e} at-argmax {rel_at:.2e} agree {ok:.3f} exact {exact:.3f}")
    assert rel <= TOL[precision] and rel_at <= TOL[precision] and ok == 1.0


def _check_U(plan, B, w, Q, H, n_chunk=256):
    """The plan's eigenvalues and leading-H projector against the oracle's
    kernel C of the same targets (the target average is taken chunk by chunk:
    C is a mean over targets, so the chunks' kernels combine by their sizes)."""
    nb = B.shape[0]
    Cor = 0.0
    for i0 in range(0, nb, n_chunk):
        Bh = B[i0:i0 + n_chunk].cpu().to(torch.complex128).numpy()
        Cor = Cor + oracle.kernel_C(Bh, w, Q) * (Bh.shape[0] / nb)
    Uor, lam_or = oracle.principal_vectors(Cor)
    U, lam = plan.U_lambda()
    U, lam = U.cpu().numpy(), lam.cpu().numpy()
    lam_err = np.abs(lam - lam_or).max() / lam_or[0]
    gap = (lam_or[H - 1] - lam_or[H]) / lam_or[0]
    proj = np.linalg.norm(U[:, :H] @ U[:, :H].T - Uor[:, :H] @ Uor[:, :H].T, 2)
    print(f"K={len(lam)}: eigenvalue err {lam_err:.2e} of lambda_0, projector distance {proj:.2e} "
          f"(relative eigengap at H {gap:.2e})")
    assert lam_err <= 1e-10
    assert proj <= 1e-9 / max(gap, 1e-6)


def test_precision_workload_U_against_oracle_kernel():
    """K = 128 from 4096 noisy targets at SNR 0.1 (sections 3.3-3.4: the
    principal vectors are the leading eigenvectors of C), the configuration
    the bench times."""
    cfg, P, A, B = _gen("precision", seed=3003)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="bf16x3", hermitian=True, products=6)
    torch.cuda.synchronize()
    _check_U(plan, B, P.w, cfg.Q, cfg.H)


def test_diff_workload_forward_lse_rows():
    cfg, P, A, B = _gen("diff", seed=5005)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="fp32", hermitian=True)
    out = plan.pairs("lse+best", inv_sigma2=1.0)
    torch.cuda.synchronize()
    U, _ = plan.U_lambda()
    rows = [0, 777, cfg.n_img - 1]
    Ah = A[rows].cpu().to(torch.complex128).numpy()
    Bh = B.cpu().to(torch.complex128).numpy()
    X = oracle.landscape(Ah, Bh, U.cpu().numpy(), cfg.H, P.k, P.w, P.delta)
    lp, li = oracle.lse(X, 1.0)
    glp = out["lse_pair"].cpu().numpy()[rows]
    gli = out["lse_img"].cpu().numpy()[rows]
    scale = np.abs(X).max()
    print(f"diff workload: lse_pair err {np.abs(glp - lp).max():.2e}, lse_img err {np.abs(gli - li).max():.2e}, "
          f"max|X| {scale:.2e}")
    # |d lse| <= inv_sigma2 * max|dX| <= 1e-5 * max|X|, plus FP32 rounding of lse itself
    assert np.abs(glp - lp).max() <= 1e-5 * scale + 1e-6 * np.abs(lp).max()
    assert np.abs(gli - li).max() <= 1e-5 * scale + 1e-6 * np.abs(li).max()
