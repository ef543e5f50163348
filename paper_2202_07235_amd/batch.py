"""A whole multi-job alignment step as one re-runnable, graph-capturable call.

``BatchStep`` owns fixed buffers for a list of jobs (their ``Plan`` objects
give the problem, the polar inputs and the tuned layout and band): each
``run()`` enqueues ``align_prepare`` of every job, spread over a few side
streams (the prepare kernels of small jobs, the single-workgroup eigensolver
above all, leave most of the GPU idle when run one after another), joins
them, and enqueues one ``align_pairs_batched`` for all jobs.  Nothing in a
step allocates or synchronises with the host, so the step can be captured
once in a HIP graph (``torch.cuda.graph``) and replayed.
"""
from __future__ import annotations

import torch

from . import (align_batched_workspace, align_pairs_batched, align_plan_destroy, align_prepare, align_set_tile,
               align_set_waves)


class BatchStep:
    def __init__(self, plans, n_streams: int = 4):
        self.plans = list(plans)
        dev = self.plans[0].device
        self.ws = [torch.empty_like(p.ws) for p in self.plans]
        self.handles = [None] * len(self.plans)
        self.outs = [{"best_score": torch.empty((p.n_img, p.n_tgt), dtype=torch.float32, device=dev),
                      "best_m": torch.empty((p.n_img, p.n_tgt), dtype=torch.int32, device=dev),
                      "best_t": torch.empty((p.n_img, p.n_tgt), dtype=torch.int32, device=dev)}
                     for p in self.plans]
        self.batch_ws = torch.empty(align_batched_workspace(len(self.plans)), dtype=torch.uint8, device=dev)
        # default-priority side streams
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(max(1, n_streams))]
        # largest prepares first, dealt round-robin (eigensolver K^3, rings per item)
        cost = [p.K ** 3 + (p.n_img + p.n_tgt * p.T) * p.K * p.Q for p in self.plans]
        self.order = sorted(range(len(self.plans)), key=lambda i: -cost[i])

    def run(self):
        cur = torch.cuda.current_stream()
        for s in self.streams:
            s.wait_stream(cur)
        for n, i in enumerate(self.order):
            p = self.plans[i]
            s = self.streams[n % len(self.streams)]
            h = align_prepare(p.problem, p.n_img, p.A, p.n_tgt, p.B, p.U_in, self.ws[i], stream=s)
            align_set_tile(h, p.band)
            align_set_waves(h, p.waves)
            old, self.handles[i] = self.handles[i], h
            if old:
                align_plan_destroy(old)   # host object only: the enqueued work uses the workspace
        for s in self.streams:
            cur.wait_stream(s)
        align_pairs_batched(self.handles, [(o["best_score"], o["best_m"], o["best_t"]) for o in self.outs],
                            self.batch_ws, cur)
        return self.outs

    def close(self):
        for i, h in enumerate(self.handles):
            if h:
                align_plan_destroy(h)
            self.handles[i] = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
