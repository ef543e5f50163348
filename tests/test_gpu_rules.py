"""The decision rules of align_pairs on every path, checked through the C ABI.

* Ties (section 2.7 takes an argmax; the library's convention fixes which of
  several equal maxima is reported): an image that is identically zero makes
  every landscape value of its pairs exactly 0.0, so every (t, m) ties and the
  smallest t * Q + m, (0, 0), must be reported, on the fused Hermitian path,
  the generic path (FP64 and non-Hermitian FP32) and the batched launch.
* Non-finite values: an infinite or NaN sample poisons exactly the pairs it
  enters (score NaN, indices -1, lse NaN), and a NaN target reaching the
  kernel C (library-computed U) makes U, the eigenvalues and every pair NaN.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_07235_amd as rs
import synth
from tests._parity import host_inputs, to_device

pytestmark = pytest.mark.gpu


def _problem(Q=128, K=32, n_img=11, n_tgt=21, T=9, H=12, seed=910, hermitian=True):
    if hermitian:
        cfg = synth.config("fp32", N=Q // 2, K=K, Q=Q, n_img=n_img, n_tgt=n_tgt, T=T, H=H,
                           n_blobs=8, snr=0.5)
    else:
        cfg = synth.config("tiny", n_img=n_img, n_tgt=n_tgt, H=H)
    return cfg, synth.make_problem(cfg, seed)


def _assert_zero_rows(o, rows, T):
    sc, m, t = (o[k].cpu().numpy() for k in ("best_score", "best_m", "best_t"))
    for r in rows:
        assert (sc[r] == 0.0).all(), sc[r]
        assert (m[r] == 0).all() and (t[r] == 0).all(), (m[r], t[r])
    others = [i for i in range(sc.shape[0]) if i not in rows]
    assert (m[others] >= 0).all() and (t[others] >= 0).all() and (t[others] < T).all()


@pytest.mark.parametrize("precision,products", [("fp32", 3), ("bf16x3", 6), ("bf16x3", 3), ("bf16", 3)])
def test_zero_image_ties_go_to_first_index_fused(precision, products):
    cfg, P = _problem()
    A, B = to_device(P, "fp32")
    A[2] = 0
    A[7] = 0
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision, hermitian=True, products=products)
    o = plan.pairs("best+lse", inv_sigma2=0.5)
    torch.cuda.synchronize()
    _assert_zero_rows(o, [2, 7], cfg.T)
    # every value 0: lse_pair = log(T Q) exactly up to FP32 rounding of the sum
    lp = o["lse_pair"].cpu().numpy()
    assert np.allclose(lp[[2, 7]], np.log(cfg.T * cfg.Q), rtol=0, atol=1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_image_ties_go_to_first_index_generic(precision):
    # FP64 plans and non-Hermitian inputs take the generic kernel
    herm = precision == "fp64"
    cfg, P = _problem(Q=64, K=16, n_img=4, n_tgt=5, T=1, H=7, hermitian=herm)
    A, B = to_device(P, precision)
    A[1] = 0
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision, hermitian=herm)
    o = plan.pairs("best+lse+full", inv_sigma2=0.5)
    torch.cuda.synchronize()
    assert (o["X"][1] == 0).all()
    _assert_zero_rows(o, [1], cfg.T)


def test_zero_image_ties_go_to_first_index_batched():
    jobs = []
    for i, (Q, K, H, na, nb, T) in enumerate([(128, 32, 8, 9, 17, 9), (512, 128, 24, 10, 20, 1)]):
        cfg, P = _problem(Q=Q, K=K, n_img=na, n_tgt=nb, T=T, H=H, seed=920 + i)
        A, B = to_device(P, "fp32")
        A[3] = 0
        jobs.append((cfg, rs.Plan(A, B, P.k, P.w, P.delta, H, precision="bf16x3", products=6)))
    outs = rs.pairs_batched([p for _, p in jobs])
    torch.cuda.synchronize()
    for (cfg, _), o in zip(jobs, outs):
        _assert_zero_rows(o, [3], cfg.T)


@pytest.mark.parametrize("bad", [float("inf"), float("-inf"), float("nan")])
@pytest.mark.parametrize("precision,products", [("fp32", 3), ("bf16x3", 6)])
def test_non_finite_target_sample_poisons_its_pairs(bad, precision, products):
    cfg, P = _problem(Q=256, K=64, n_img=9, n_tgt=18, T=4, H=16, seed=930)
    A, B = to_device(P, "fp32")
    B[5, 7, 40] = complex(bad, 0.0)
    U = torch.eye(cfg.K, dtype=torch.float64)[:, :cfg.H].contiguous()   # row 7 is kept
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision, hermitian=True,
                   products=products, U=U)
    o = plan.pairs("best+lse", inv_sigma2=0.1)
    torch.cuda.synchronize()
    sc, m, t = (o[k].cpu().numpy() for k in ("best_score", "best_m", "best_t"))
    lp, li = o["lse_pair"].cpu().numpy(), o["lse_img"].cpu().numpy()
    assert np.isnan(sc[:, 5]).all() and (m[:, 5] == -1).all() and (t[:, 5] == -1).all()
    assert np.isnan(lp[:, 5]).all() and np.isnan(li).all()
    others = np.delete(np.arange(cfg.n_tgt), 5)
    assert np.isfinite(sc[:, others]).all() and (m[:, others] >= 0).all()
    assert np.isfinite(lp[:, others]).all()


def test_non_finite_image_sample_poisons_its_pairs_generic():
    cfg, P = _problem(Q=64, K=16, n_img=4, n_tgt=5, T=1, H=16, hermitian=False)
    A, B = to_device(P, "fp32")
    A[2, 3, 9] = complex(0.0, float("inf"))
    U = torch.eye(cfg.K, dtype=torch.float64).contiguous()
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="fp32", hermitian=False, U=U)
    o = plan.pairs("best+lse", inv_sigma2=0.1)
    torch.cuda.synchronize()
    sc, m = o["best_score"].cpu().numpy(), o["best_m"].cpu().numpy()
    # the oracle's rule on the same inputs
    A_h, B_h = host_inputs(A, B)
    with np.errstate(invalid="ignore", over="ignore"):
        X = oracle.landscape(A_h, B_h, np.eye(cfg.K), cfg.H, P.k, P.w, P.delta)
        ref, ref_m, _ = oracle.best(X)
    assert np.array_equal(np.isnan(sc), np.isnan(ref))
    assert np.isnan(sc[2]).all() and (m[2] == -1).all()
    assert np.isfinite(sc[[0, 1, 3]]).all()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
def test_nan_target_with_library_U_gives_nan_everywhere(precision):
    cfg, P = _problem(Q=128, K=32, n_img=9, n_tgt=17, T=1, H=8, seed=940)
    A, B = to_device(P, precision)
    B[4, 2, 3] = complex(float("nan"), 0.0)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision, hermitian=True, products=6)
    o = plan.pairs("best+lse", inv_sigma2=0.1)
    U, lam = plan.U_lambda()
    torch.cuda.synchronize()
    assert torch.isnan(lam).all() and torch.isnan(U).all()
    sc, m, t = (o[k].cpu().numpy() for k in ("best_score", "best_m", "best_t"))
    assert np.isnan(sc).all() and (m == -1).all() and (t == -1).all()
    assert np.isnan(o["lse_pair"].cpu().numpy()).all()
