"""align_pairs_batched_noalloc: the batched launch with the library's own
device scratch instead of a caller workspace, for callers that cannot
allocate.  Checked against align_pairs_batched (the workspace entry point,
itself checked against one align_pairs call per job and the FP64 oracle) to
the bit, on two calls in a row, the second with fewer and smaller jobs, so
that the second call runs over what the first left in the scratch."""
import numpy as np
import pytest
import torch

import paper_2202_07235_amd as rs
import synth

pytestmark = pytest.mark.gpu

#             Q    K   H  n_img n_tgt T
FIRST = [(128, 32, 8, 37, 21, 9),
         (256, 64, 24, 19, 40, 9),
         (512, 128, 19, 25, 33, 9),
         (384, 96, 31, 16, 16, 1),
         (192, 48, 13, 20, 40, 25)]
SECOND = [(256, 64, 16, 9, 17, 1),
          (128, 32, 32, 8, 20, 9)]


def _plans(specs, seed):
    out = []
    for i, (Q, K, H, na, nb, T) in enumerate(specs):
        cfg = synth.config("fp32", N=Q // 2, K=K, Q=Q, n_img=na, n_tgt=nb, T=T, H=H, n_blobs=8, snr=0.5)
        P = synth.make_problem(cfg, seed=seed + i, device="cuda")
        A = P.A.to(torch.complex64).contiguous()
        B = P.B.to(torch.complex64).contiguous()
        out.append(rs.Plan(A, B, P.k, P.w, P.delta, H, precision="bf16x3", products=6))
    return out


def _poisoned(plans):
    return [{"best_score": torch.full((p.n_img, p.n_tgt), float("nan"), device="cuda"),
             "best_m": torch.full((p.n_img, p.n_tgt), -7, dtype=torch.int32, device="cuda"),
             "best_t": torch.full((p.n_img, p.n_tgt), -7, dtype=torch.int32, device="cuda")} for p in plans]


def test_noalloc_batched_equals_workspace_batched_on_two_calls():
    for specs, seed in ((FIRST, 7100), (SECOND, 7200)):
        plans = _plans(specs, seed)
        ref = rs.pairs_batched(plans)
        outs = _poisoned(plans)
        rs.align_pairs_batched_noalloc([p.handle for p in plans],
                                       [(o["best_score"], o["best_m"], o["best_t"]) for o in outs])
        torch.cuda.synchronize()
        for j, (r, o) in enumerate(zip(ref, outs)):
            for k in ("best_score", "best_m", "best_t"):
                assert torch.equal(r[k], o[k]), (len(specs), j, k)
            m = o["best_m"].cpu().numpy()
            assert (m >= 0).all() and (m < specs[j][0]).all()


def test_noalloc_batched_rejects_more_jobs_than_its_scratch_holds():
    plans = _plans(SECOND[:1], 7300)
    n = rs.RADSVD_NOALLOC_MAX_JOBS + 1
    outs = _poisoned(plans) * n
    with pytest.raises(rs.RadsvdError, match="UNSUPPORTED"):
        rs.align_pairs_batched_noalloc([plans[0].handle] * n,
                                       [(o["best_score"], o["best_m"], o["best_t"]) for o in outs])
