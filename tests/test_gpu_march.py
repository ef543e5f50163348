"""Principal-mode marching and the landscape quality measures through the C ABI.

* align_top_targets against the oracle's candidate order (ties to the smaller
  target, NaN never taken) on seeded score arrays.
* align_landscape_metrics against the oracle's measures on seeded landscapes
  (FP64 and FP32 arrays): f per pair exactly, the summary to rounding.
* align_pairs_list against the oracle landscape of the listed pairs, with
  entries outside the plan.
* march: candidates and their high-rank alignments against the oracle's
  composition of the same steps (low-rank landscapes, top targets, high-rank
  landscapes of the candidates with the same U); and the quality of the
  low-rank landscape against the full-rank one, on the GPU and in the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_07235_amd as rs
import synth
from paper_2202_07235_amd import march as mr
from tests._parity import argmax_agrees, host_inputs, to_device

pytestmark = pytest.mark.gpu


def test_top_targets_matches_oracle():
    rng = np.random.default_rng(41)
    S = rng.standard_normal((9, 300)).astype(np.float32)
    S[2, ::7] = np.nan
    S[4, :] = np.nan
    S[4, 10] = 0.5
    S[5, 20:40] = 3.0   # ties
    for k in (1, 5, 64):
        cand = torch.empty((9, k), dtype=torch.int32, device="cuda")
        rs.align_top_targets(torch.tensor(S, device="cuda"), k, cand)
        torch.cuda.synchronize()
        assert np.array_equal(cand.cpu().numpy(), oracle.top_targets(S, k)), k


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_landscape_metrics_match_oracle(dtype):
    rng = np.random.default_rng(42)
    R = rng.standard_normal((6, 5, 4, 48)) + 1j * rng.standard_normal((6, 5, 4, 48))
    E = R + 0.4 * (rng.standard_normal(R.shape) + 1j * rng.standard_normal(R.shape))
    if dtype == torch.complex64:   # the oracle sees the values the GPU sees
        R, E = R.astype(np.complex64).astype(np.complex128), E.astype(np.complex64).astype(np.complex128)
    out = mr.landscape_metrics(torch.tensor(E, dtype=dtype, device="cuda"), torch.tensor(R, dtype=dtype, device="cuda"))
    rel, corr, f = oracle.landscape_metrics(E.reshape(30, -1), R.reshape(30, -1))
    assert np.array_equal(out["f"].cpu().numpy().ravel(), f.astype(np.float32))
    assert abs(out["rel_fro"] - rel) <= 1e-12 * rel
    assert abs(out["corr"] - corr) <= 1e-12
    assert abs(out["mean_f"] - float(np.mean(f.astype(np.float32).astype(np.float64)))) <= 1e-12


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_pairs_list_matches_oracle(precision):
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=6, n_tgt=9, T=4, H=7, n_blobs=8, snr=0.5)
    P = synth.make_problem(cfg, seed=1600)
    A, B = to_device(P, precision)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision)
    pl = np.array([[0, 0], [5, 8], [3, 2], [3, 2], [7, 1], [1, -1], [2, 4]], dtype=np.int32)
    o = plan.pairs_list(torch.tensor(pl, device="cuda"), "best+full")
    torch.cuda.synchronize()
    A_h, B_h = host_inputs(A, B)
    U = plan.U_lambda()[0].cpu().numpy()
    ok = [i for i in range(len(pl)) if 0 <= pl[i, 0] < 6 and 0 <= pl[i, 1] < 9]
    X = oracle.landscape(A_h, B_h, U, cfg.H, P.k, P.w, P.delta, pairs=[tuple(pl[i]) for i in ok])
    sc, m, t = o["best_score"].cpu().numpy(), o["best_m"].cpu().numpy(), o["best_t"].cpu().numpy()
    tol = 1e-12 if precision == "fp64" else 1e-5
    Xg = o["X"].cpu().numpy()
    for j, i in enumerate(ok):
        scale = np.abs(X[j]).max()
        assert np.abs(Xg[i] - X[j]).max() <= tol * scale
        assert argmax_agrees(X[j][None, None], m[i:i + 1][None], t[i:i + 1][None], tol).all()
    bad = [i for i in range(len(pl)) if i not in ok]
    assert np.isnan(sc[bad]).all() and (m[bad] == -1).all() and (t[bad] == -1).all()


def test_march_matches_oracle_and_quality():
    cfg = synth.config("fp32", N=64, K=32, Q=128, n_img=12, n_tgt=40, T=4, H=16, n_blobs=8, snr=0.5)
    P = synth.make_problem(cfg, seed=1700)
    A, B = to_device(P, "fp32")
    H_low, H_high, n_cand = 4, 16, 6
    res = mr.march(A, B, P.k, P.w, P.delta, H_low, H_high, n_cand)
    torch.cuda.synchronize()
    low, high = res["plans"]
    A_h, B_h = host_inputs(A, B)
    U = low.U_lambda()[0].cpu().numpy()
    X_low = oracle.landscape(A_h, B_h, U, H_low, P.k, P.w, P.delta)
    s_low, _, _ = oracle.best(X_low)
    cand = res["cand"].cpu().numpy()
    c_or = oracle.top_targets(s_low, n_cand)
    scale_low = np.abs(X_low).reshape(12, 40, -1).max(axis=-1)
    for a in range(12):
        if not np.array_equal(cand[a], c_or[a]):   # near-ties in the low-rank scores only
            kth = np.sort(s_low[a])[::-1][n_cand - 1]
            assert np.all(s_low[a, cand[a]] >= kth - 2e-5 * scale_low[a].max()), a
    # the candidates' high-rank alignments
    X_hi = oracle.landscape(A_h, B_h, U, H_high, P.k, P.w, P.delta,
                            pairs=[(a, int(b)) for a in range(12) for b in cand[a]])
    sc_or, m_or, t_or = oracle.best(X_hi[:, None])
    sc = res["score"].cpu().numpy().ravel()
    scale = np.abs(X_hi).reshape(len(sc), -1).max(axis=-1)
    assert np.all(np.abs(sc - sc_or[:, 0]) <= 1e-5 * scale)
    assert argmax_agrees(X_hi[:, None], res["m"].cpu().numpy().reshape(-1, 1),
                         res["t"].cpu().numpy().reshape(-1, 1), 1e-5).all()
    # quality of the rank-4 landscape against rank K, on the GPU and in the oracle
    full = rs.Plan(A, B, P.k, P.w, P.delta, cfg.K, precision="fp32", U=low.U_lambda()[0].contiguous())
    lo4 = rs.Plan(A, B, P.k, P.w, P.delta, H_low, precision="fp32", U=low.U_lambda()[0][:, :H_low].contiguous())
    q = mr.landscape_metrics(lo4.pairs("full")["X"], full.pairs("full")["X"])
    X_full = oracle.landscape(A_h, B_h, U, cfg.K, P.k, P.w, P.delta)
    rel, corr, f = oracle.landscape_metrics(X_low.reshape(480, -1), X_full.reshape(480, -1))
    print(f"rank {H_low} vs {cfg.K}: rel Frobenius {q['rel_fro']:.4f} (oracle {rel:.4f}), "
          f"corr {q['corr']:.4f} ({corr:.4f}), mean f {q['mean_f']:.4f} ({np.mean(f):.4f})")
    assert abs(q["rel_fro"] - rel) <= 1e-4 * rel
    assert abs(q["corr"] - corr) <= 1e-5
    assert abs(q["mean_f"] - np.mean(f)) <= 0.02
