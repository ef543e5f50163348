"""Tile-order autotuner of the fused pair kernel.

The fast Hermitian path computes tiles of 8 images x 16 targets; the order in
which the tiles run (``band``: image tiles each XCD walks before the target
tile advances, see ``align_set_tile``) decides how much operand data the
workgroups resident on one XCD share in its L2, and never the results.  The
tuner times each candidate band on the job itself (``align_pairs`` with the
best-score output, HIP events on the current stream) and keeps the fastest.
Choices are cached per job class (Q, rank rounded to 8, T, tile counts rounded
to a power of two, precision), so a batch of similar jobs is tuned once.
"""
from __future__ import annotations

import math

import torch

BANDS = (1, 2, 4, 8, 16)
_cache: dict = {}


def _key(plan) -> tuple:
    nta = (plan.n_img + 7) // 8
    ntb = (plan.n_tgt + 15) // 16
    return (plan.Q, (plan.H + 7) // 8 * 8, plan.T, 1 << max(0, int(math.log2(nta))),
            1 << max(0, int(math.log2(ntb))), plan.precision, plan.products)


def _time_ms(plan, outputs, reps: int) -> float:
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    plan.pairs("best", outputs=outputs)   # warm
    for e0, e1 in ev:
        e0.record()
        plan.pairs("best", outputs=outputs)
        e1.record()
    torch.cuda.synchronize()
    return min(e0.elapsed_time(e1) for e0, e1 in ev)


def tune_band(plan, bands=BANDS, reps: int = 3, use_cache: bool = True) -> int:
    """Pick the fastest tile band for ``plan`` (a ``Plan``), set it on the plan
    and return it."""
    key = _key(plan)
    if use_cache and key in _cache:
        plan.set_tile(_cache[key])
        return _cache[key]
    out = {}
    best, best_t = None, float("inf")
    for b in bands:
        plan.set_tile(b)
        t = _time_ms(plan, out, reps)
        if t < best_t:
            best, best_t = b, t
    plan.set_tile(best)
    _cache[key] = best
    return best


def tune_jobs(plans, bands=BANDS, reps: int = 3) -> list[int]:
    """Tune every plan of a batch (one measurement per job class)."""
    return [tune_band(p, bands, reps) for p in plans]


def clear_cache():
    _cache.clear()
