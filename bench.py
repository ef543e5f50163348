"""Benchmark of the radial-SVD alignment hot path on one MI355X.

Workload (the precision study of the paper's image-alignment method, on
synthetic Gaussian-blob images standing in for cryo-EM data): N = 256 px,
K = 128 radial rings, Q = 512 angles, N_A = N_B = 4096 images/targets, T = 9
translations (3 x 3, 1 px), rank H = 24.  One step = align_prepare (kernel
C, FP64 eigensolver, principal rings of every image and translated target)
+ align_pairs with the best (gamma, delta) and score per pair.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Prints one JSON line.  value = image pairs (all gamma x delta) per second of
whole steps with inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "image-pairs/s (all γ×δ), N=256 H=24: bf16x3 MFMA vs FP32, rel err ≤1e-5"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP32_MATRIX_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--precision", default="bf16x3")
    ap.add_argument("--products", type=int, default=6,
                    help="bf16x3 cross products: 6 uses all three split terms (hi, mid, lo), "
                         "3 only the two leading terms")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="fraction of N_A and N_B (for quick local runs; 1.0 = the full workload)")
    ap.add_argument("--only", choices=["plain", "batching", "differentiation", "volume"], default=None,
                    help="run only that other workload and print its record as one JSON line")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (plain FP32 batch, batching, differentiation, volume)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the same-GPU comparison runs (FP32, bf16x3 with 3 products)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB streaming kernel (x -> -x) whose HBM counters calibrate FETCH_SIZE / "
                         "WRITE_SIZE of the pair kernel")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="summarise rocprofv3 --pmc runs (any counters) of the pair kernel at the precision "
                         "workload into the counter profile text and exit (needs --kernel-ms)")
    ap.add_argument("--summarize-kernel-stats", metavar="CSV",
                    help="summarise a rocprofv3 --kernel-trace --stats kernel_stats.csv of bench.py runs "
                         "(library kernels only) and exit")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="HBM bytes per dispatch of every kernel matching --kernel-regex in two rocprofv3 --pmc "
                         "runs (FETCH_SIZE, then WRITE_SIZE) made with --copy-probe, scaled by the copy kernel's "
                         "readings, and exit")
    ap.add_argument("--kernel-regex", default=None,
                    help="kernel-name pattern for --summarize-traffic and --summarize-pmc")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="DIR",
                    help="per-kernel averages of every counter in rocprofv3 --pmc runs, for the kernels matching "
                         "--kernel-regex, and exit")
    ap.add_argument("--kernel-ms", type=float, default=None,
                    help="the pair kernel's duration (from a kernel-trace run), for the derived rates")
    ap.add_argument("--reduce-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "`bench.py --copy-probe` into the traffic profile text and exit")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_pairs_wide_precision_bf16x3_6_traffic.txt")
TRAFFIC_CONFIG = "bf16x3 products=6"
TRAFFIC_KERNEL = "k_pairs_wide"
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2202_07235_amd", "csrc", f)
                  for f in ("pairs_wide.h", "pairs_wide.hip", "pairs_fast.h", "pairs_fast.hip", "common.h",
                            "internal.h")]
COPY_BYTES = 1 << 30


def pair_kernel_name(Q, precision, products):
    """The fused kernel align_pairs(BEST) dispatches for a Hermitian plan: the
    eight-wave kernel for split bf16 with six products at Q = 384 and 512, the
    four-wave one otherwise."""
    if precision == "bf16x3" and products == 6 and Q in (384, 512):
        return f"k_pairs_wide<Q={Q},bf16x3,6 products>"
    return f"k_pairs_fast<Q={Q},{precision}{',%d products' % products if precision == 'bf16x3' else ''}>"


def kernel_source_hash():
    """Hash of the pair kernel's sources with comments and blank lines removed
    (a changed comment does not invalidate measured counters)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f) as fh:
            txt = fh.read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        h.update("\n".join(l.rstrip() for l in txt.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def reduce_counters(fetch_dir, write_dir):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the pair kernel, scaled by
    what the same counters read for the 1 GiB streaming kernel (read 1 GiB,
    write 1 GiB), as HBM bytes per launch."""
    out = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        pair, copy = [], []
        for r in _counter_rows(d):
            if r.get("Counter_Name") != name:
                continue
            kn, v = r.get("Kernel_Name", ""), float(r["Counter_Value"])
            if TRAFFIC_KERNEL in kn:
                pair.append(v)
            elif "neg" in kn and "elementwise" in kn:
                copy.append(v)
        if not pair or not copy:
            raise SystemExit(f"{d}: no {name} rows for the pair kernel ({len(pair)}) or the copy kernel ({len(copy)})")
        cp = max(copy)   # the 1 GiB launch (smaller neg launches, if any, read less)
        out[name] = (sum(pair) / len(pair), len(pair), cp, COPY_BYTES / (cp * 1024.0))
    fa, na, fc, ff = out["FETCH_SIZE"]
    wa, nw, wc, wf = out["WRITE_SIZE"]
    traffic = fa * 1024.0 * ff + wa * 1024.0 * wf
    lines = [
        f"# HBM traffic of {TRAFFIC_KERNEL}, precision workload (N=256 K=128 Q=512 N_A=N_B=4096 T=9 H=24)",
        "# kernel_source_sha256_16: hash of the pair kernel sources with comments removed (bench.kernel_source_hash)",
        f"config: {TRAFFIC_CONFIG}",
        f"kernel_source_sha256_16: {kernel_source_hash()}",
        f"pair kernel FETCH_SIZE per dispatch: {fa:.6g} KiB ({na} dispatches)",
        f"pair kernel WRITE_SIZE per dispatch: {wa:.6g} KiB ({nw} dispatches)",
        f"copy kernel (1 GiB read + 1 GiB write) FETCH_SIZE: {fc:.6g} KiB -> scale {ff:.4f}",
        f"copy kernel (1 GiB read + 1 GiB write) WRITE_SIZE: {wc:.6g} KiB -> scale {wf:.4f}",
        f"traffic_bytes_per_launch: {traffic:.6g}",
    ]
    return "\n".join(lines)


def summarize_counters(dirs, kernel_ms):
    """Per-dispatch averages of every counter of the pair kernel in the given
    rocprofv3 --pmc output folders, with the rates they imply on MI355X (256
    CUs x 4 SIMDs at 2.4 GHz; one wave64 VALU instruction issues over 4
    cycles)."""
    import collections
    acc = collections.defaultdict(list)
    for d in dirs:
        for r in _counter_rows(d):
            if TRAFFIC_KERNEL in r.get("Kernel_Name", ""):
                acc[r["Counter_Name"]].append(float(r["Counter_Value"]))
    if not acc:
        raise SystemExit(f"no {TRAFFIC_KERNEL} dispatches in {dirs}")
    v = {k: sum(x) / len(x) for k, x in acc.items()}
    n_tiles = (4096 // 8) * (4096 // 16)
    waves, T = n_tiles * 8, 9
    simd_cycles = 1024 * 2.4e9 * kernel_ms * 1e-3
    lines = [f"# SQ/TCC counters of {TRAFFIC_KERNEL}, precision workload (N=256 K=128 Q=512 N_A=N_B=4096 "
             f"T=9 H=24), bf16x3 with 6 products",
             "# kernel_source_sha256_16: hash of the pair kernel sources with comments removed "
             "(bench.kernel_source_hash)",
             f"config: {TRAFFIC_CONFIG}",
             f"kernel_source_sha256_16: {kernel_source_hash()}",
             f"kernel_ms (kernel-trace run): {kernel_ms:.2f}",
             f"waves per dispatch: {waves} ({n_tiles} workgroups x 8), translations: {T}",
             "", "counter (average per dispatch)"]
    for k in sorted(v):
        lines.append(f"  {k:28s} {v[k]:.6g}  ({len(acc[k])} dispatches)")
    lines += ["", "derived"]

    def have(*ks):
        return all(k in v for k in ks)
    if have("SQ_VALU_MFMA_BUSY_CYCLES"):
        lines.append(f"  MFMA busy, fraction of SIMD cycles: {v['SQ_VALU_MFMA_BUSY_CYCLES'] / simd_cycles:.3f}")
    if have("SQ_INSTS_VALU"):
        lines.append(f"  VALU issue, fraction of SIMD cycles (4 cycles each): {4 * v['SQ_INSTS_VALU'] / simd_cycles:.3f}")
        lines.append(f"  VALU instructions per wave and translation: {v['SQ_INSTS_VALU'] / waves / T:.0f}")
    if have("SQ_INSTS_MFMA"):
        lines.append(f"  MFMA instructions per wave and translation: {v['SQ_INSTS_MFMA'] / waves / T:.0f}")
    if have("SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES"):
        lines.append(f"  SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES: {v['SQ_ACTIVE_INST_VALU'] / v['SQ_WAVE_CYCLES']:.3f}")
    if have("SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"):
        lines.append(f"  SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES: {v['SQ_WAIT_INST_ANY'] / v['SQ_WAVE_CYCLES']:.3f}")
    if have("SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS"):
        lines.append(f"  SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS: "
                     f"{v['SQ_LDS_BANK_CONFLICT'] / v['SQ_ACTIVE_INST_LDS']:.3f}")
    if have("TCC_HIT_sum", "TCC_MISS_sum"):
        lines.append(f"  L2 hit rate: {v['TCC_HIT_sum'] / (v['TCC_HIT_sum'] + v['TCC_MISS_sum']):.3f}")
    if have("TA_BUSY_avr", "GRBM_GUI_ACTIVE"):
        lines.append(f"  TA busy (TA_BUSY_avr / (GRBM_GUI_ACTIVE / 8 XCDs)): "
                     f"{v['TA_BUSY_avr'] / (v['GRBM_GUI_ACTIVE'] / 8):.3f}")
    return "\n".join(lines)


def summarize_traffic(fetch_dir, write_dir, pattern):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of every library kernel whose
    name matches the pattern, averaged per kernel, as HBM bytes via the scale
    the same counters give for the 1 GiB copy kernel of --copy-probe."""
    import collections
    import re
    rx = re.compile(pattern)
    lines = []
    per = {}
    scale = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        acc = collections.defaultdict(list)
        copy = []
        for r in _counter_rows(d):
            if r.get("Counter_Name") != name:
                continue
            kn, v = r.get("Kernel_Name", ""), float(r["Counter_Value"])
            if "neg" in kn and "elementwise" in kn:
                copy.append(v)
            elif rx.search(kn):
                short = kn.replace("void ", "").replace("(anonymous namespace)::", "").replace("radsvd::", "")
                short = short[:short.index("(")] if "(" in short else short
                acc[short].append(v)
        if not copy:
            raise SystemExit(f"{d}: no copy-kernel rows (run with --copy-probe)")
        scale[name] = COPY_BYTES / (max(copy) * 1024.0)
        per[name] = acc
    lines.append(f"copy kernel scale: FETCH_SIZE x {scale['FETCH_SIZE']:.4f}, WRITE_SIZE x {scale['WRITE_SIZE']:.4f}")
    lines.append(f"{'kernel':56s} {'dispatches':>10s} {'fetch B':>12s} {'write B':>12s}")
    for k in sorted(set(per["FETCH_SIZE"]) | set(per["WRITE_SIZE"])):
        f = per["FETCH_SIZE"].get(k, [])
        w = per["WRITE_SIZE"].get(k, [])
        fb = sum(f) / len(f) * 1024.0 * scale["FETCH_SIZE"] if f else float("nan")
        wb = sum(w) / len(w) * 1024.0 * scale["WRITE_SIZE"] if w else float("nan")
        lines.append(f"{k[:56]:56s} {len(f):10d} {fb:12.4g} {wb:12.4g}")
    return "\n".join(lines)


def summarize_pmc(dirs, pattern):
    """Average per dispatch of every counter of every library kernel whose name
    matches the pattern, in the given rocprofv3 --pmc output folders."""
    import collections
    import re
    rx = re.compile(pattern)
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for r in _counter_rows(d):
            kn = r.get("Kernel_Name", "")
            if not rx.search(kn):
                continue
            short = kn.replace("void ", "").replace("(anonymous namespace)::", "").replace("radsvd::", "")
            short = short[:short.index("(")] if "(" in short else short
            acc[short][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = []
    for k in sorted(acc):
        lines.append(k)
        for c in sorted(acc[k]):
            v = acc[k][c]
            lines.append(f"  {c:28s} {sum(v) / len(v):.6g}  ({len(v)} dispatches)")
    return "\n".join(lines)


def summarize_kernel_stats(path):
    """Library kernels of a rocprofv3 kernel_stats.csv: calls, average, min and
    max duration (ms), sorted by total time."""
    import csv
    with open(path) as fh:
        rows = [r for r in csv.DictReader(fh) if "radsvd::" in r["Name"]]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"{'kernel':72s} {'calls':>5s} {'avg ms':>9s} {'min ms':>9s} {'max ms':>9s}"]
    for r in rows:
        name = r["Name"].replace("void ", "").replace("(anonymous namespace)::", "").replace("radsvd::", "")
        name = name[:name.index("(")] if "(" in name else name
        lines.append(f"{name[:72]:72s} {int(r['Calls']):5d} {float(r['AverageNs']) / 1e6:9.3f} "
                     f"{float(r['MinNs']) / 1e6:9.3f} {float(r['MaxNs']) / 1e6:9.3f}")
    return "\n".join(lines)


def traffic_from_profile():
    """HBM bytes per pair-kernel launch from the committed counter profile, or
    None when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            txt = fh.read()
    except OSError:
        return None
    kv = dict(l.split(": ", 1) for l in txt.splitlines() if ": " in l and not l.startswith("#"))
    if kv.get("kernel_source_sha256_16") != kernel_source_hash() or kv.get("config") != TRAFFIC_CONFIG:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Step:
    """One reusable workspace; each step re-runs prepare + pairs."""

    def __init__(self, rs, A, B, P, H, precision, products):
        import torch
        self.rs, self.torch = rs, torch
        self.A, self.B = A, B
        self.n_img, self.n_tgt = A.shape[0], B.shape[0]
        prec = rs.PRECISIONS[precision]
        self.problem, self._keep = rs.make_problem(A.shape[1], A.shape[2], H, P.delta.shape[0], P.k, P.w,
                                                   P.delta, prec, 1, products)
        nbytes = rs.align_prepare_workspace(self.problem, self.n_img, self.n_tgt)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dev = "cuda"
        self.out = {"best_score": torch.empty((self.n_img, self.n_tgt), dtype=torch.float32, device=dev),
                    "best_m": torch.empty((self.n_img, self.n_tgt), dtype=torch.int32, device=dev),
                    "best_t": torch.empty((self.n_img, self.n_tgt), dtype=torch.int32, device=dev)}
        self.plan = None
        self.ev = []

    def run(self, record=False):
        rs, torch = self.rs, self.torch
        if self.plan is not None:
            rs.align_plan_destroy(self.plan)
        self.plan = rs.align_prepare(self.problem, self.n_img, self.A, self.n_tgt, self.B, None, self.ws)
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        rs.align_pairs(self.plan, rs.OUT_BEST, 1.0, self.out["best_score"], self.out["best_m"],
                       self.out["best_t"])
        if record:
            e1.record()
            self.ev.append((e0, e1))

    def pairs_ms(self):
        return [a.elapsed_time(b) for a, b in self.ev]

    def close(self):
        if self.plan is not None:
            self.rs.align_plan_destroy(self.plan)
            self.plan = None


def timed(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step.run()
    torch.cuda.synchronize()
    step.ev.clear()
    t0 = time.perf_counter()
    for _ in range(steps):
        step.run(record=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, step.pairs_ms()


def cpu_baseline(P, A, B, U, H, gpu_out, budget_s=12.0):
    """The FP64 oracle (direct psi-space sums, OpenMP) on a random sample of
    pairs of the same workload: principal rings of the sampled images and
    translated targets, the landscape of every sampled pair and its best.
    Also returns the GPU's error on the sample."""
    import numpy as np
    import oracle
    oracle.build()
    rng = np.random.default_rng(12345)
    na, nb = A.shape[0], B.shape[0]

    def run(n):
        ia = rng.integers(0, na, n)
        ib = rng.integers(0, nb, n)
        ua, inv_a = np.unique(ia, return_inverse=True)
        ub, inv_b = np.unique(ib, return_inverse=True)
        Ah = A[ua].cpu().to(dtype=__import__("torch").complex128).numpy()
        Bh = B[ub].cpu().to(dtype=__import__("torch").complex128).numpy()
        t0 = time.perf_counter()
        Ar = oracle.principal_rings(Ah, U, H, P.w, A.shape[2])
        Br = oracle.principal_rings(Bh, U, H, P.w, A.shape[2], k=P.k, delta=P.delta)
        X = oracle.landscape_rings(Ar, Br, pairs=list(zip(inv_a, inv_b)))
        sc, m, t = oracle.best(X[:, None])
        dt = time.perf_counter() - t0
        return dt, ia, ib, X, sc[:, 0], m[:, 0], t[:, 0]

    dt, ia, ib, X, sc, m, t = run(16)
    n = int(min(4096, max(16, 16 * budget_s / max(dt, 1e-3))))
    dt, ia, ib, X, sc, m, t = run(n)
    g_sc = gpu_out["best_score"].cpu().numpy()[ia, ib]
    g_m = gpu_out["best_m"].cpu().numpy()[ia, ib]
    g_t = gpu_out["best_t"].cpu().numpy()[ia, ib]
    Q = A.shape[2]
    scale = np.abs(X).reshape(n, -1).max(axis=1)
    at = X.real.reshape(n, -1)[np.arange(n), g_t * Q + g_m]
    rel = float(np.max(np.abs(g_sc - sc) / scale))
    rel_at = float(np.max(np.abs(g_sc - at) / scale))
    agree = float(np.mean((g_m == m) & (g_t == t)))
    near = float(np.mean((g_m == m) & (g_t == t) | ((sc - at) <= 4e-5 * scale)))
    return {"value": n / dt, "unit": "image-pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} random pairs of the workload, all 9 translations x 512 rotations each; "
                      f"principal rings of the sampled items + FP64 direct psi-space landscape + best; "
                      f"U from the GPU plan; {dt:.1f} s",
            "seconds": dt}, {"pairs": n, "max_rel_err_best_score": rel, "max_rel_err_score_at_argmax": rel_at,
                             "argmax_exact": agree, "argmax_within_tol": near}


def roofline(cfg, precision, products, kernel_ms):
    """Roofline of the fused pair kernel on one launch over a workload: the
    contraction's algorithmic flops (8 H (Q/2 + 1) per pair-translation, times
    the split products), the half-spectrum transform's 2.5 Q log2 Q on the
    vector unit, and the minimum operand + output bytes; the bound is the unit
    with the largest time at its published peak."""
    n_pairs = cfg.n_img * cfg.n_tgt
    pair_delta = n_pairs * cfg.T
    H, Q = cfg.H, cfg.Q
    M1 = Q // 2 + 1
    nprod = {"fp32": 1, "bf16": 1, "bf16x3": products}[precision]
    flops_contract = 8.0 * H * M1 * pair_delta                # conj(a) b over h, q in [0, Q/2]
    flops_fft = 2.5 * Q * math.log2(Q) * pair_delta           # half-spectrum inverse transform
    t_s = kernel_ms * 1e-3
    t_mfma = flops_contract * nprod / (PEAK_BF16_TFLOPS * 1e12) if precision != "fp32" else \
        flops_contract / (PEAK_FP32_MATRIX_TFLOPS * 1e12)
    t_valu = flops_fft / (PEAK_FP32_VECTOR_TFLOPS * 1e12)
    H8 = (H + 7) // 8 * 8
    # operand bytes per real value (images, targets): FP32 4 B; bf16 2 B; bf16x3 with 3 products
    # two bf16 planes (4 B); with 6 products the images' three bf16 planes (6 B) and the
    # targets' FP32 values, split in registers (4 B)
    bpr_a, bpr_b = {"fp32": (4, 4), "bf16": (2, 2), "bf16x3": (4, 4) if products == 3 else (6, 4)}[precision]
    bytes_min = (cfg.n_img * bpr_a + cfg.n_tgt * cfg.T * bpr_b) * M1 * 2 * H8 + n_pairs * 12
    t_hbm = bytes_min / (PEAK_HBM_GBS * 1e9)
    bound = max(("mfma", t_mfma), ("alu", t_valu), ("hbm", t_hbm), key=lambda kv: kv[1])
    if bound[0] == "alu":
        roof = {"bound": "alu", "achieved": flops_fft / t_s / 1e12, "peak": PEAK_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s"}
    elif bound[0] == "mfma":
        pk = PEAK_BF16_TFLOPS if precision != "fp32" else PEAK_FP32_MATRIX_TFLOPS
        roof = {"bound": "mfma", "achieved": flops_contract * nprod / t_s / 1e12, "peak": pk, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": bytes_min / t_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = pair_kernel_name(Q, precision, products)
    roof["kernel_ms"] = kernel_ms
    roof["per_unit"] = {"unit": "pair-translation", "units_per_launch": pair_delta,
                        "contraction_flops": 8 * H * M1, "fft_flops": 2.5 * Q * math.log2(Q),
                        "products": nprod, "operand_bytes_min_total": bytes_min}
    roof["unit_times_ms"] = {"mfma": 1e3 * t_mfma, "valu_fft": 1e3 * t_valu, "hbm": 1e3 * t_hbm}
    return roof


def _make_inputs(synth, torch, cfg, seed):
    P = synth.make_problem(cfg, seed=seed, device="cuda")
    A = P.A.to(torch.complex64).contiguous()
    B = P.B.to(torch.complex64).contiguous()
    P.A = P.B = None
    return P, A, B


def plain_workload(rs, synth, torch, steps=5):
    """The plain FP32 batch (N 128, K 64, Q 256, 1024 x 1024 pairs, T 9, H 16),
    one step = align_prepare + align_pairs(BEST), in FP32 and in split bf16
    with six products, each with the pair kernel's roofline."""
    cfg = synth.config("fp32")
    P, A, B = _make_inputs(synth, torch, cfg, 2002)
    out = {"workload": f"plain FP32 batch: N={cfg.N} K={cfg.K} Q={cfg.Q} N_A={cfg.n_img} N_B={cfg.n_tgt} "
                       f"T={cfg.T} H={cfg.H}"}
    for prec, prod in (("fp32", 3), ("bf16x3", 6)):
        st = Step(__import__("paper_2202_07235_amd"), A, B, P, cfg.H, prec, prod)
        wall, pms = timed(st, steps, 2)
        st.close()
        kms = float(sum(pms) / len(pms))
        roof = roofline(cfg, prec, prod, kms)
        key = prec if prec == "fp32" else f"{prec}_{prod}products"
        out[key] = {"image_pairs_per_s": cfg.n_img * cfg.n_tgt * steps / wall, "ms_per_step": 1e3 * wall / steps,
                    "pairs_kernel_ms": kms,
                    "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "kernel")}}
        print(f"[bench] plain workload {key}: {out[key]['ms_per_step']:.2f} ms/step, pairs kernel {kms:.2f} ms, "
              f"frac {roof['frac']:.3f}", file=sys.stderr, flush=True)
    return out


def batching_workload(rs, synth, torch, reps=3):
    """The batching workload (64 jobs: N in {64 .. 256}, K = N/2, Q = 2N,
    N_A in [128, 2048], N_B in [64, 1024] log-uniform, T in {1, 9, 25}, H in
    [8, 32]; split bf16, six products): the pair step as one launch per job
    and as the persistent batched launch, both after the autotuner; and the
    whole step (prepare of every job + the batched launch) replayed from a
    HIP graph."""
    from paper_2202_07235_amd import autotune
    cfgs = synth.batch_configs(64, seed=4000)
    plans = []
    for i, cfg in enumerate(cfgs):
        P, A, B = _make_inputs(synth, torch, cfg, 4000 + i)
        plans.append(rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="bf16x3", products=6))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    autotune.tune_jobs(plans)
    tune_s = time.perf_counter() - t0
    outs = [p.pairs("best") for p in plans]
    bouts = [{k: torch.empty_like(v) for k, v in o.items()} for o in outs]
    ws = torch.empty(rs.align_batched_workspace(len(plans)), dtype=torch.uint8, device="cuda")

    def per_job():
        for p, o in zip(plans, outs):
            p.pairs("best", outputs=o)

    def batched():
        rs.pairs_batched(plans, outputs=bouts, batch_ws=ws)

    times = {}
    for name, fn in (("one_launch_per_job_ms", per_job), ("batched_ms", batched)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / reps
    same = all(torch.equal(o[k], b[k]) for o, b in zip(outs, bouts) for k in o)
    pairs = sum(c.n_img * c.n_tgt for c in cfgs)
    res = {"workload": "batching: 64 jobs, N in {64,96,128,192,256}, K=N/2, Q=2N, N_A in [128,2048], "
                       "N_B in [64,1024], T in {1,9,25}, H in [8,32], bf16x3 (6 products)",
           "image_pairs": pairs, **times, "speedup_batched_vs_per_job": times["one_launch_per_job_ms"] / times["batched_ms"],
           "batched_equals_per_job": same, "autotune_s": tune_s, "tuned": autotune.describe(plans)}
    try:
        res.update(graph_step(rs, torch, plans, outs, reps))
    except Exception as ex:   # reported, not hidden: the key says why the graph figure is missing
        res["graph_error"] = repr(ex)
    print(f"[bench] batching workload: {res}", file=sys.stderr, flush=True)
    for p in plans:
        p.close()
    return res


def graph_step(rs, torch, plans, ref, reps):
    """The whole step (prepare of every job on 4 side streams + the batched
    pair launch), eager and replayed from a HIP graph (each replay checked
    against the eager outputs), against prepare + pairs one job at a time."""
    from paper_2202_07235_amd.batch import BatchStep
    bs = BatchStep(plans)

    def one_by_one():
        for p, o in zip(plans, ref):
            h = rs.align_prepare(p.problem, p.n_img, p.A, p.n_tgt, p.B, p.U_in, p.ws)
            rs.align_set_tile(h, p.band)
            rs.align_set_waves(h, p.waves)
            rs.align_pairs(h, rs.OUT_BEST, 1.0, o["best_score"], o["best_m"], o["best_t"])
            rs.align_plan_destroy(h)

    def timed_ms(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    per_job_ms = timed_ms(one_by_one)
    eager_ms = timed_ms(bs.run)
    eager = [{k: v.clone() for k, v in o.items()} for o in bs.outs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bs.run()
    torch.cuda.synchronize()
    graph_ms = timed_ms(g.replay)
    for o in bs.outs:
        o["best_score"].fill_(float("nan"))
    g.replay()
    torch.cuda.synchronize()
    ok = all(torch.equal(e[k], o[k]) for e, o in zip(eager, bs.outs) for k in e)
    ok_ref = all(torch.equal(r[k], o[k]) for r, o in zip(ref, bs.outs) for k in r)
    del g
    bs.close()
    return {"step_one_job_at_a_time_ms": per_job_ms, "step_batched_eager_ms": eager_ms,
            "step_batched_graph_ms": graph_ms, "speedup_step_graph_vs_one_job_at_a_time": per_job_ms / graph_ms,
            "graph_replay_equals_eager": ok, "graph_equals_one_job_at_a_time": ok_ref}


def differentiation_workload(rs, synth, torch, reps=3):
    """The differentiation workload (N 128, K 64, Q 256, 2048 images, 256
    templates, T 9, H 16, sigma^2 = 1): forward LSE and the backward pass with
    respect to the templates' polar coefficients and U, FP32 plan."""
    cfg = synth.config("diff")
    P, A, B = _make_inputs(synth, torch, cfg, 5005)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="fp32")
    g = torch.ones(cfg.n_img, dtype=torch.float32, device="cuda")
    o = plan.pairs("lse", inv_sigma2=1.0)
    plan.backward(1.0, o["lse_img"], g)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fw, bw = [], []
    for _ in range(reps):
        ev[0].record()
        o = plan.pairs("lse", inv_sigma2=1.0)
        ev[1].record()
        plan.backward(1.0, o["lse_img"], g)
        ev[2].record()
        torch.cuda.synchronize()
        fw.append(ev[0].elapsed_time(ev[1]))
        bw.append(ev[1].elapsed_time(ev[2]))
    res = {"workload": f"differentiation: N={cfg.N} K={cfg.K} Q={cfg.Q} N_A={cfg.n_img} N_B={cfg.n_tgt} T={cfg.T} "
                       f"H={cfg.H}, loss = sum_a logsumexp(X / sigma^2), FP32 plan",
           "forward_lse_ms": min(fw), "backward_ms": min(bw)}
    print(f"[bench] differentiation workload: {res}", file=sys.stderr, flush=True)
    plan.close()
    return res


def volume_flops(cfg):
    """Algorithmic flops of one volume-target pair at ranks H_C, H_D (section
    4.9): step 1 (complex MACs over the principal shells), step 1b (real x
    complex over the degrees), step 2 per interior angle, and step 3 counted
    as a 2-D FFT (5 n log2 n, n = M^2); also the flops the library executes
    for step 3, a direct length-M DFT along rows then columns."""
    L, M, nb = cfg.L, 2 * cfg.L + 1, cfg.n_beta
    lm2 = sum((2 * l + 1) ** 2 for l in range(L + 1))
    s1 = 8.0 * cfg.H_C * lm2
    s1b = 4.0 * cfg.H_D * lm2
    s2 = 4.0 * nb * cfg.H_D * M * M
    s3 = nb * 5.0 * M * M * math.log2(M * M)
    s3_exec = nb * 2.0 * M ** 3 * 8.0
    return {"step1": s1, "step1b": s1b, "step2": s2, "step3_fft": s3, "step3_executed": s3_exec,
            "algorithmic": s1 + s1b + s2 + s3, "executed": s1 + s1b + s2 + s3_exec}


def volume_workload(rs, synth, torch, reps=3):
    """Volume alignment (section 4): 96 noisy rotated copies of one target
    (real blob volumes standing in for the paper's reconstructions), K = 48
    shells, degrees to L = 48 (M = 97 orders), 97 interior angles,
    H_C = H_D = 16, FP32 plan with the real-volume mode; the general complex
    mode and an FP64 plan are timed beside it.  One step = vol_prepare +
    vol_align(BEST)."""
    from paper_2202_07235_amd import volume as rv
    from synth import volumes as sv
    cfg = sv.vol_config("volume")
    P = sv.make_volume_problem(cfg, 6006)
    A = torch.tensor(P.A, dtype=torch.complex64, device="cuda")
    B = torch.tensor(P.B, dtype=torch.complex64, device="cuda")
    A64 = torch.tensor(P.A, dtype=torch.complex128, device="cuda")
    B64 = torch.tensor(P.B, dtype=torch.complex128, device="cuda")

    def make(real, fp64=False):
        if fp64:
            return rv.VolPlan(A64, B64, P.w, cfg.L, cfg.H_C, cfg.H_D, P.beta, precision="fp64", real=real)
        return rv.VolPlan(A, B, P.w, cfg.L, cfg.H_C, cfg.H_D, P.beta, precision="fp32", real=real)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def run(real, fp64=False):
        plan = make(real, fp64)
        plan.align("best")
        torch.cuda.synchronize()
        plan.close()
        prep, al = [], []
        for _ in range(reps):
            ev[0].record()
            plan = make(real, fp64)
            ev[1].record()
            plan.align("best")
            ev[2].record()
            torch.cuda.synchronize()
            prep.append(ev[0].elapsed_time(ev[1]))
            al.append(ev[1].elapsed_time(ev[2]))
            plan.close()
        return prep, al

    prep_c, al_c = run(False)
    prep_64, al_64 = run(True, fp64=True)
    prep, al = run(True)
    n_pairs = cfg.n_vol * cfg.n_tgt
    # quality of the compressed landscape against the full sum over shells and
    # degrees (the measures of the paper's volume example), at several ranks
    from paper_2202_07235_amd import march
    full = rv.VolPlan(A, B, P.w, cfg.L, cfg.K, cfg.L + 1, P.beta, precision="fp32", real=True)
    X_ref = full.align("full")["X"]
    quality = {}
    for h in (4, 8, cfg.H_C, 24):
        pl = rv.VolPlan(A, B, P.w, cfg.L, h, h, P.beta, precision="fp32", real=True)
        X_est = pl.align("full")["X"]
        mq = march.landscape_metrics(X_est, X_ref)
        quality[f"H_C=H_D={h}"] = {"rel_fro": mq["rel_fro"], "corr": mq["corr"], "mean_f": mq["mean_f"]}
        pl.close()
        del X_est
    full.close()
    del X_ref
    fl = volume_flops(cfg)
    t = min(al) * 1e-3
    res = {"workload": f"volume: {cfg.n_vol} volumes x {cfg.n_tgt} target, K={cfg.K} L={cfg.L} (M={2 * cfg.L + 1}), "
                       f"n_beta={cfg.n_beta}, H_C={cfg.H_C} H_D={cfg.H_D}, FP32 plan",
           "vol_prepare_ms": min(prep), "vol_align_ms": min(al),
           "complex_mode": {"vol_prepare_ms": min(prep_c), "vol_align_ms": min(al_c),
                            "pairs_per_s": n_pairs / (min(al_c) * 1e-3)},
           "fp64_real_mode": {"vol_prepare_ms": min(prep_64), "vol_align_ms": min(al_64),
                              "pairs_per_s": n_pairs / (min(al_64) * 1e-3)},
           "pairs_per_s": n_pairs / t, "pairs_per_s_with_prepare": n_pairs / ((min(al) + min(prep)) * 1e-3),
           "quality_vs_full_rank": quality,
           "flops_per_pair": fl,
           "roofline": {"bound": "alu", "achieved": n_pairs * fl["algorithmic"] / t / 1e12, "peak": 157.3,
                        "unit": "TFLOP/s", "frac": n_pairs * fl["algorithmic"] / t / 1e12 / 157.3,
                        "executed_tflops": n_pairs * fl["executed"] / t / 1e12, "kernel": "vol_align (all kernels)"}}
    print(f"[bench] volume workload: {res}", file=sys.stderr, flush=True)
    return res


def main():
    a = parse()
    if a.reduce_counters:
        print(reduce_counters(*a.reduce_counters))
        return 0
    if a.summarize_kernel_stats:
        print(summarize_kernel_stats(a.summarize_kernel_stats))
        return 0
    if a.summarize_pmc:
        if not a.kernel_regex:
            raise SystemExit("--summarize-pmc needs --kernel-regex")
        print(summarize_pmc(a.summarize_pmc, a.kernel_regex))
        return 0
    if a.summarize_traffic:
        if not a.kernel_regex:
            raise SystemExit("--summarize-traffic needs --kernel-regex")
        print(summarize_traffic(*a.summarize_traffic, a.kernel_regex))
        return 0
    if a.summarize_counters:
        if a.kernel_ms is None:
            raise SystemExit("--summarize-counters needs --kernel-ms")
        print(summarize_counters(a.summarize_counters, a.kernel_ms))
        return 0
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); the library has no multi-GPU "
              f"path.", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import paper_2202_07235_amd as rs
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.only:
        if a.copy_probe:   # a 1 GiB streaming kernel whose counters calibrate the HBM counters
            src = torch.randn(COPY_BYTES // 4, device="cuda")
            torch.neg(src, out=torch.empty_like(src))
            torch.cuda.synchronize()
            del src
        fn = {"plain": plain_workload, "batching": batching_workload,
              "differentiation": differentiation_workload, "volume": volume_workload}[a.only]
        print(json.dumps(fn(rs, synth, torch)))
        return 0
    cfg = synth.config("precision")
    if a.scale != 1.0:
        cfg = synth.config("precision", n_img=max(16, int(cfg.n_img * a.scale)),
                           n_tgt=max(16, int(cfg.n_tgt * a.scale)))
    print(f"[bench] generating inputs: {cfg}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    P = synth.make_problem(cfg, seed=3003, device="cuda")
    A = P.A.to(torch.complex64).contiguous()
    B = P.B.to(torch.complex64).contiguous()
    del P.A, P.B
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    print(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    n_pairs = cfg.n_img * cfg.n_tgt
    pair_delta = n_pairs * cfg.T
    H, Q = cfg.H, cfg.Q

    step = Step(rs, A, B, P, H, a.precision, a.products)
    print(f"[bench] {a.precision}: {a.warmup} warmup + {a.steps} timed steps", file=sys.stderr, flush=True)
    wall, pairs_ms = timed(step, a.steps, a.warmup)
    ms_step = 1e3 * wall / a.steps
    value = n_pairs * a.steps / wall
    pairs_avg = float(np.mean(pairs_ms))
    U_dev = torch.empty((cfg.K, cfg.K), dtype=torch.float64, device="cuda")
    rs.align_get_U(step.plan, U_dev, None)
    torch.cuda.synchronize()
    gpu_out = {k: v.clone() for k, v in step.out.items()}
    step.close()
    print(f"[bench] {a.precision}: {ms_step:.2f} ms/step, pairs kernel {pairs_avg:.2f} ms", file=sys.stderr,
          flush=True)

    if a.copy_probe:
        src = torch.randn(COPY_BYTES // 4, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        print("[bench] copy probe done", file=sys.stderr, flush=True)

    # the same step in plain FP32 and, for bf16x3, with the two-term split (3 products), on this GPU
    alt = {}
    alt_runs = [] if a.no_fp32 else [("fp32", 3)]
    if not a.no_fp32 and a.precision == "bf16x3" and a.products == 6:
        alt_runs.append(("bf16x3", 3))
    for prec, prod in alt_runs:
        if prec == a.precision and prod == a.products:
            continue
        s2 = Step(rs, A, B, P, H, prec, prod)
        n2 = max(2, a.steps // 2)
        w2, p2 = timed(s2, n2, 1)
        s2.close()
        key = prec if prec == "fp32" else f"{prec}_{prod}products"
        alt[key] = {"value": n_pairs * n2 / w2, "ms_per_step": 1e3 * w2 / n2, "pairs_kernel_ms": float(np.mean(p2))}
        print(f"[bench] {key}: {alt[key]['ms_per_step']:.2f} ms/step, pairs kernel {alt[key]['pairs_kernel_ms']:.2f} ms",
              file=sys.stderr, flush=True)

    # roofline of the dominant kernel (the fused pair kernel)
    roof = roofline(cfg, a.precision, a.products, pairs_avg)
    tr = traffic_from_profile() if f"{a.precision} products={a.products}" == TRAFFIC_CONFIG else None
    roof = {**{k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac")}, "traffic": tr,
            **{k: v for k, v in roof.items() if k not in ("bound", "achieved", "peak", "unit", "frac")}}

    extras = {}
    if not a.no_extras:
        del step
        torch.cuda.empty_cache()
        extras["plain_fp32_workload"] = plain_workload(rs, synth, torch)
        extras["batching_workload"] = batching_workload(rs, synth, torch)
        extras["differentiation_workload"] = differentiation_workload(rs, synth, torch)
        extras["volume_workload"] = volume_workload(rs, synth, torch)

    cpu = None
    accuracy = None
    if not a.no_cpu:
        print("[bench] cpu baseline (oracle on a sample)", file=sys.stderr, flush=True)
        cpu, accuracy = cpu_baseline(P, A, B, U_dev.cpu().numpy(), H, gpu_out)

    try:
        gpu_name = torch.cuda.get_device_name(0)
    except Exception:
        gpu_name = "?"
    rec = {
        "metric": METRIC, "value": value, "unit": "image-pairs/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": a.precision if a.precision != "bf16x3" else f"bf16x3({a.products} products)",
        "data": "synthetic (seeded Gaussian-blob images, closed-form polar FT, Hermitian noise SNR 0.1)",
        "config": {"workload": f"precision: N={cfg.N} K={cfg.K} Q={cfg.Q} N_A={cfg.n_img} N_B={cfg.n_tgt} "
                               f"T={cfg.T} H={cfg.H}", "N": cfg.N, "K": cfg.K, "Q": cfg.Q, "n_img": cfg.n_img,
                   "n_tgt": cfg.n_tgt, "T": cfg.T, "H": cfg.H, "precision": a.precision,
                   "products": a.products, "step": "align_prepare + align_pairs(BEST)"},
        "pairs_only_per_s": n_pairs / (pairs_avg * 1e-3),
        "pairs_kernel_ms": pairs_avg,
        "same_gpu_comparison": alt,
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": accuracy,
        "other_workloads": extras,
        "gpu": gpu_name,
        "host": platform.node(),
    }
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
