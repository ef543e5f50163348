"""Persistent multi-job launch (align_pairs_batched), its HIP-graph capture and
the tile-order autotuner.

* Bitwise equality with one align_pairs call per job, for jobs of every
  supported angle count and rank class, T in {1, 9, 25}, ragged counts, in
  FP32, bf16x3 (3 and 6 products) and BF16.
* Parity of the batched outputs with the FP64 oracle on sampled pairs.
* Graph capture: replays with eager work in between, every replay checked.
* Wave layouts (align_set_waves): 4 and 8 waves per CU give bitwise the
  outputs of the default, alone and in a batch that mixes layouts (the
  batched launch runs each class of items at its own occupancy); layouts a
  plan does not have are refused and leave it unchanged.
* The batching workload (64 jobs: N in {64..256}, K = N/2, Q = 2N, N_A in
  [128, 2048], N_B in [64, 1024], T in {1, 9, 25}, H in [8, 32]) with
  autotuned layouts and bands: equal to one launch per job, and timed
  against it; the whole step (prepare of every job + the batched launch)
  captured in a HIP graph, every replay equal to the eager step.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_07235_amd as rs
import synth
from paper_2202_07235_amd import autotune
from paper_2202_07235_amd.batch import BatchStep
from tests._parity import argmax_agrees, host_inputs

pytestmark = pytest.mark.gpu

#        Q    K   H  n_img n_tgt T
JOBS = [(128, 32, 8, 37, 21, 9),
        (192, 48, 13, 20, 40, 25),
        (256, 64, 24, 9, 17, 1),
        (384, 96, 31, 16, 16, 9),
        (512, 128, 19, 25, 33, 9),
        (128, 32, 32, 8, 70, 1),
        (512, 128, 8, 40, 8, 25)]


def _plans(precision, products=3, jobs=JOBS, seed=600):
    out = []
    for i, (Q, K, H, na, nb, T) in enumerate(jobs):
        cfg = synth.config("fp32", N=Q // 2, K=K, Q=Q, n_img=na, n_tgt=nb, T=T, H=H, n_blobs=8, snr=0.5)
        P = synth.make_problem(cfg, seed=seed + i, device="cuda")
        A = P.A.to(torch.complex64).contiguous()
        B = P.B.to(torch.complex64).contiguous()
        out.append((cfg, P, rs.Plan(A, B, P.k, P.w, P.delta, H, precision=precision, products=products)))
    return out


def _same(o1, o2):
    return all(torch.equal(o1[k], o2[k]) for k in ("best_score", "best_m", "best_t"))


@pytest.mark.parametrize("precision,products", [("fp32", 3), ("bf16x3", 3), ("bf16x3", 6), ("bf16", 3)])
def test_batched_equals_one_launch_per_job(precision, products):
    jobs = _plans(precision, products)
    plans = [p for _, _, p in jobs]
    for i, p in enumerate(plans):
        p.set_tile([1, 2, 4, 8, 16, 0, 4][i])
    outs = rs.pairs_batched(plans)
    torch.cuda.synchronize()
    for p, o in zip(plans, outs):
        assert _same(p.pairs("best"), o)


def test_batched_matches_oracle_on_sampled_pairs():
    jobs = _plans("bf16x3", 6, seed=700)
    plans = [p for _, _, p in jobs]
    outs = rs.pairs_batched(plans)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for (cfg, P, plan), o in zip(jobs, outs):
        ia = rng.integers(0, cfg.n_img, 6)
        ib = rng.integers(0, cfg.n_tgt, 6)
        A_h, B_h = host_inputs(plan.A, plan.B)
        U = plan.U_lambda()[0].cpu().numpy()
        X = oracle.landscape(A_h, B_h, U, cfg.H, P.k, P.w, P.delta, pairs=list(zip(ia, ib)))
        sc = o["best_score"].cpu().numpy()[ia, ib]
        m = o["best_m"].cpu().numpy()[ia, ib]
        t = o["best_t"].cpu().numpy()[ia, ib]
        ref, _, _ = oracle.best(X[:, None])
        scale = np.abs(X).reshape(len(ia), -1).max(axis=1)
        assert (np.abs(sc - ref[:, 0]) / scale).max() <= 1e-5
        assert argmax_agrees(X[:, None], m[:, None], t[:, None], 1e-5).all()


def test_batched_launch_replays_from_a_graph():
    jobs = _plans("bf16x3", 3, jobs=JOBS[:4], seed=800)
    plans = [p for _, _, p in jobs]
    ref = [p.pairs("best") for p in plans]
    outs = [{k: torch.empty_like(v) for k, v in r.items()} for r in ref]
    ws = torch.empty(rs.align_batched_workspace(len(plans)), dtype=torch.uint8, device="cuda")
    rs.pairs_batched(plans, outputs=outs, batch_ws=ws)   # eager warm-up before capture
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rs.pairs_batched(plans, outputs=outs, batch_ws=ws)
    for rep in range(3):
        for o in outs:   # eager work between replays: poison the outputs
            o["best_score"].fill_(float("nan"))
            o["best_m"].fill_(-7)
            o["best_t"].fill_(-7)
        plans[rep % len(plans)].pairs("best")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for r, o in zip(ref, outs):
            assert _same(r, o), f"replay {rep}"


def test_batched_rejects_unsupported_plans():
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=8, n_tgt=16, T=1, H=8)
    P = synth.make_problem(cfg, seed=1, device="cuda")
    p64 = rs.Plan(P.A.to(torch.complex64).contiguous(), P.B.to(torch.complex64).contiguous(),
                  P.k, P.w, P.delta, 8, precision="fp32")
    with pytest.raises(rs.RadsvdError, match="UNSUPPORTED"):
        rs.pairs_batched([p64])


def test_batching_workload_autotuned_vs_one_launch_per_job():
    cfgs = synth.batch_configs(64, seed=4000)
    plans, keep = [], []
    for i, cfg in enumerate(cfgs):
        P = synth.make_problem(cfg, seed=4000 + i, device="cuda")
        A = P.A.to(torch.complex64).contiguous()
        B = P.B.to(torch.complex64).contiguous()
        P.A = P.B = None
        plans.append(rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="bf16x3", products=6))
    torch.cuda.synchronize()
    autotune.tune_jobs(plans)
    print("autotuned:", autotune.describe(plans))
    ref = [p.pairs("best") for p in plans]
    outs = rs.pairs_batched(plans)
    torch.cuda.synchronize()
    for i, (r, o) in enumerate(zip(ref, outs)):
        assert _same(r, o), f"job {i}"
    # timing: one persistent launch vs one launch per job (same outputs)
    ws = torch.empty(rs.align_batched_workspace(len(plans)), dtype=torch.uint8, device="cuda")

    def per_job():
        for p, r in zip(plans, ref):
            p.pairs("best", outputs=r)

    def batched():
        rs.pairs_batched(plans, outputs=outs, batch_ws=ws)

    times = {}
    for name, fn in (("one launch per job", per_job), ("persistent batched", batched)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            fn()
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / 3
    pairs = sum(c.n_img * c.n_tgt for c in cfgs)
    print({k: f"{v:.2f} ms ({pairs / v * 1e3:.3e} pairs/s)" for k, v in times.items()})


#              Q    K   H  n_img n_tgt T
LAYOUT_JOBS = [(128, 32, 24, 30, 40, 4),
               (192, 48, 32, 17, 33, 9),
               (256, 64, 16, 24, 20, 9),
               (256, 64, 24, 9, 35, 4)]


@pytest.mark.parametrize("precision,products", [("fp32", 3), ("bf16x3", 6), ("bf16", 3), ("bf16x3", 3)])
def test_wave_layouts_give_the_same_outputs(precision, products):
    jobs = _plans(precision, products, jobs=LAYOUT_JOBS, seed=1100)
    plans = [p for _, _, p in jobs]
    ref = [p.pairs("best+lse", inv_sigma2=0.3) for p in plans]
    for w in (4, 8):
        for p, r in zip(plans, ref):
            p.set_waves(w)
            o = p.pairs("best+lse", inv_sigma2=0.3)
            for k in r:
                assert torch.equal(r[k], o[k]), (w, p.Q, p.H, k)
    # a batch mixing both layouts: equal to the per-job outputs
    for i, p in enumerate(plans):
        p.set_waves((4, 8)[i % 2])
    outs = rs.pairs_batched(plans)
    torch.cuda.synchronize()
    for r, o in zip(ref, outs):
        for k in ("best_score", "best_m", "best_t"):
            assert torch.equal(r[k], o[k])


def test_wave_layouts_refused_where_absent():
    jobs = _plans("bf16x3", 6, jobs=[(512, 128, 24, 9, 17, 1), (64, 16, 8, 9, 17, 1)], seed=1200)
    (_, _, wide), (_, _, small) = jobs
    ref = wide.pairs("best")
    with pytest.raises(rs.RadsvdError, match="UNSUPPORTED"):
        wide.set_waves(4)           # operands in the eight-wave layout
    wide.set_waves(8)
    assert all(torch.equal(ref[k], v) for k, v in wide.pairs("best").items())
    with pytest.raises(rs.RadsvdError, match="UNSUPPORTED"):
        small.set_waves(4)          # Q = 64: only the default (two workgroups per CU)
    with pytest.raises(rs.RadsvdError, match="INVALID_ARG"):
        small.set_waves(6)
    small.set_waves(8)
    p384 = _plans("fp32", 3, jobs=[(384, 96, 16, 9, 17, 1)], seed=1300)[0][2]
    with pytest.raises(rs.RadsvdError, match="UNSUPPORTED"):
        p384.set_waves(8)           # Q = 384 four-wave: the LDS holds one workgroup
    p384.set_waves(4)


def test_batching_workload_step_replays_from_a_graph():
    cfgs = synth.batch_configs(64, seed=4000)
    plans = []
    for i, cfg in enumerate(cfgs):
        P = synth.make_problem(cfg, seed=4000 + i, device="cuda")
        A = P.A.to(torch.complex64).contiguous()
        B = P.B.to(torch.complex64).contiguous()
        P.A = P.B = None
        plans.append(rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="bf16x3", products=6))
        plans[-1].set_waves((0, 4, 8)[i % 3] if cfg.Q in (128, 192, 256) else 0)
    ref = [p.pairs("best") for p in plans]
    bs = BatchStep(plans)
    bs.run()
    torch.cuda.synchronize()
    for i, (r, o) in enumerate(zip(ref, bs.outs)):
        assert all(torch.equal(r[k], o[k]) for k in r), f"eager step, job {i}"
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bs.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for o in bs.outs:   # eager work between replays
            o["best_score"].fill_(float("nan"))
            o["best_m"].fill_(-7)
        plans[rep].pairs("best")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (r, o) in enumerate(zip(ref, bs.outs)):
            assert all(torch.equal(r[k], o[k]) for k in r), f"replay {rep}, job {i}"
    del g
    bs.close()
