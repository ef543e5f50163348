"""Autotuner of the fused pair kernel's tiling: wave layout and tile order.

The fast Hermitian path computes tiles of 8 images x 16 targets.  Two knobs
change how they run, never the results:

* ``waves`` (``align_set_waves``): the waves resident on one compute unit, 4
  (one four-wave workgroup per CU, the deepest operand prefetch) or 8 (two
  workgroups, each wave hiding the other's memory waits, at a smaller
  register budget; or the eight-wave workgroup at Q = 384 and 512 for split
  bf16 with six products);
* ``band`` (``align_set_tile``): the image tiles each XCD walks before the
  target tile advances, which decides how much operand data the workgroups
  resident on one XCD share in its L2.

The tuner times every layout the plan has, each with the default band, keeps
the fastest, then times the bands in that layout (``align_pairs`` with the
best-score output, HIP events on the current stream).  Choices are cached per
job class (Q, rank rounded to 8, T, tile counts rounded to a power of two,
precision), so a batch of similar jobs is tuned once.
"""
from __future__ import annotations

import math

import torch

BANDS = (1, 2, 4, 8, 16)
WAVES = (4, 8)
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


def _layouts(plan, waves):
    """Wave layouts this plan has (set_waves raises UNSUPPORTED for the others)."""
    from . import RadsvdError
    out = []
    for w in waves:
        try:
            plan.set_waves(w)
        except RadsvdError:
            continue
        out.append(w)
    plan.set_waves(0)
    return out


def tune(plan, bands=BANDS, waves=WAVES, reps: int = 3, use_cache: bool = True) -> tuple[int, int]:
    """Pick the fastest (waves, band) for ``plan`` (a ``Plan``), set both on
    the plan and return them."""
    key = _key(plan)
    if use_cache and key in _cache:
        w, b = _cache[key]
        plan.set_waves(w)
        plan.set_tile(b)
        return w, b
    out = {}
    lay = _layouts(plan, waves)
    best_w, best_t = 0, float("inf")
    plan.set_tile(0)
    if len(lay) > 1:
        for w in lay:
            plan.set_waves(w)
            t = _time_ms(plan, out, reps)
            if t < best_t:
                best_w, best_t = w, t
    else:
        best_w = lay[0] if lay else 0
    plan.set_waves(best_w)
    best_b, best_t = 0, float("inf")
    for b in bands:
        plan.set_tile(b)
        t = _time_ms(plan, out, reps)
        if t < best_t:
            best_b, best_t = b, t
    plan.set_tile(best_b)
    _cache[key] = (best_w, best_b)
    return best_w, best_b


def tune_band(plan, bands=BANDS, reps: int = 3, use_cache: bool = True) -> int:
    """Tile order only (the plan's wave layout unchanged)."""
    key = ("band",) + _key(plan) + (plan.waves,)
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


def tune_jobs(plans, bands=BANDS, waves=WAVES, reps: int = 3) -> list[tuple[int, int]]:
    """Tune every plan of a batch (one measurement per job class)."""
    return [tune(p, bands, waves, reps) for p in plans]


def describe(plans) -> dict:
    """Counts of the chosen settings over a batch, e.g. {"band=4": 12, ...}."""
    out: dict = {}
    for p in plans:
        k = f"waves={p.waves or 'default'},band={p.band}"
        out[k] = out.get(k, 0) + 1
    return dict(sorted(out.items()))


def clear_cache():
    _cache.clear()
