"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/radsvd.h, and rejects invalid arguments with the
documented status before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2202_07235_amd as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "radsvd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(align_\w+|vol_\w+|radsvd_\w+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = rs._load()
    names = _declared()
    assert "align_prepare" in names and "align_pairs" in names and "align_pairs_backward" in names
    assert "vol_prepare" in names and "vol_align" in names and "vol_get_UV" in names
    for n in names:
        assert hasattr(lib, n), n


def _prob(**kw):
    K, Q, H, T = kw.get("K", 16), kw.get("Q", 64), kw.get("H", 8), kw.get("T", 1)
    k = kw.get("k", np.linspace(0.5, 16, K))
    w = kw.get("w", np.ones(K))
    delta = kw.get("delta", np.zeros((T, 2)))
    return rs.make_problem(K, Q, H, T, k, w, delta, kw.get("prec", rs.FP32), kw.get("herm", 1),
                           kw.get("products", 3), kw.get("sigma_delta", 0.0))


@pytest.mark.parametrize("bad", [
    dict(K=1), dict(K=129), dict(Q=63), dict(Q=70), dict(Q=1024), dict(Q=4), dict(H=0), dict(H=17),
    dict(K=64, H=33), dict(T=0), dict(T=65), dict(prec=7), dict(herm=2),
    dict(prec=rs.BF16X3, products=4), dict(k=np.r_[np.linspace(0.5, 16, 15), -1.0]),
    dict(w=np.r_[np.ones(15), 0.0]), dict(T=2, delta=np.array([[0.0, np.nan], [0, 0]])),
    dict(sigma_delta=-0.1), dict(sigma_delta=float("nan")), dict(sigma_delta=float("inf")),
])
def test_invalid_problem_rejected(bad):
    pr, keep = _prob(**bad)
    assert rs._load().align_prepare_workspace(ctypes.byref(pr), 4, 4) == 0
    assert rs.radsvd_last_error() != ""


def test_workspace_size_is_positive_and_monotone():
    pr, keep = _prob()
    a = rs.align_prepare_workspace(pr, 4, 4)
    b = rs.align_prepare_workspace(pr, 8, 40)
    assert 0 < a < b
    assert rs._load().align_prepare_workspace(ctypes.byref(pr), 0, 4) == 0


def _prepare_status(pr, n_img=4, n_tgt=4, A=0x10000, B=0x20000, U=None, ws=0x40000, ws_bytes=None):
    lib = rs._load()
    plan = ctypes.c_void_p()
    if ws_bytes is None:
        ws_bytes = 1 << 40
    return lib.align_prepare(ctypes.byref(pr), n_img, ctypes.c_void_p(A), n_tgt, ctypes.c_void_p(B),
                             ctypes.c_void_p(U) if U else None, ctypes.c_void_p(ws) if ws else None,
                             ws_bytes, None, ctypes.byref(plan))


def test_prepare_argument_errors_before_launch():
    pr, keep = _prob()
    assert _prepare_status(pr, A=0) == 1
    assert _prepare_status(pr, A=0x10008) == 1            # misaligned input
    assert _prepare_status(pr, n_img=0) == 1
    assert _prepare_status(pr, U=0x30004) == 1            # misaligned U
    assert _prepare_status(pr, ws=0) == 3
    assert _prepare_status(pr, ws=0x40010) == 3           # misaligned workspace
    need = rs.align_prepare_workspace(pr, 4, 4)
    assert _prepare_status(pr, ws_bytes=need - 1) == 3
    assert "too small" in rs.radsvd_last_error()


def test_pairs_and_backward_argument_errors():
    lib = rs._load()
    assert lib.align_pairs(None, 1, 1.0, None, None, None, None, None, None, None) == 1
    assert lib.align_pairs_backward(None, 1.0, None, None, None, None, None, 0, None) == 1
    assert lib.align_get_U(None, None, None, None) == 1
    assert lib.align_set_tile(None, 0) == 1
    assert lib.align_set_waves(None, 0) == 1
    assert lib.align_refine_rotation(None, None, None, 4, None, None, None) == 1
    assert lib.align_pairs_list(None, 1, 1.0, 1, None, None, None, None, None, None, None) == 1
    assert lib.align_top_targets(1, 1, None, 1, None, None) == 1
    assert lib.align_top_targets(4, 4, None, 0, None, None) == 1
    assert lib.align_landscape_metrics(0, 1, None, None, 0, None, None, None, None) == 1
    assert lib.align_set_waves(None, 8) == 1
    assert lib.align_batched_workspace(0) == 0
    assert lib.align_pairs_batched(None, 1, None, None, 0, None) == 1
    assert lib.align_pairs_batched_noalloc(None, 1, None, None) == 1
    assert lib.align_pairs_batched_noalloc(None, 0, None, None) == 1
    # the job limit of the library's own scratch is checked before anything else
    assert lib.align_pairs_batched_noalloc(None, rs.RADSVD_NOALLOC_MAX_JOBS + 1, None, None) == 2
    assert "no-allocation limit" in rs.radsvd_last_error()


def test_noalloc_job_limit_matches_header():
    src = open(os.path.join(ROOT, "include", "radsvd.h")).read()
    assert f"#define RADSVD_NOALLOC_MAX_JOBS {rs.RADSVD_NOALLOC_MAX_JOBS}" in src


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(rs, "_lib", None)
    monkeypatch.setattr(rs, "_LIB_PATH", "/nonexistent/libradsvd.so")
    with pytest.raises(ImportError):
        rs._load()


def _vprob(**kw):
    from paper_2202_07235_amd import volume as rv
    K, L = kw.get("K", 8), kw.get("L", 6)
    return rv.make_vol_problem(K, L, kw.get("H_C", 4), kw.get("H_D", 4), kw.get("w", np.ones(K)),
                               kw.get("beta", np.linspace(0, 6, 5)), kw.get("prec", rs.FP32), kw.get("real", 0))


@pytest.mark.parametrize("bad", [
    dict(K=1), dict(K=129), dict(L=0), dict(L=65), dict(L=49, prec=rs.FP64), dict(prec=rs.BF16),
    dict(prec=rs.BF16X3), dict(H_C=0), dict(H_C=9), dict(H_D=0), dict(H_D=8), dict(beta=np.zeros(0)),
    dict(beta=np.zeros(257)), dict(beta=np.array([0.0, np.inf])), dict(w=np.r_[np.ones(7), 0.0]),
    dict(w=np.r_[np.ones(7), np.nan]), dict(real=2), dict(real=-1),
])
def test_invalid_volume_problem_rejected(bad):
    pr, keep = _vprob(**bad)
    assert rs._load().vol_prepare_workspace(ctypes.byref(pr), 4, 4) == 0
    assert rs.radsvd_last_error() != ""


def test_volume_workspace_and_argument_errors():
    from paper_2202_07235_amd import volume as rv
    lib = rs._load()
    pr, keep = _vprob()
    a = rv.vol_prepare_workspace(pr, 4, 1)
    b = rv.vol_prepare_workspace(pr, 40, 2)
    assert 0 < a < b
    assert lib.vol_prepare_workspace(ctypes.byref(pr), 0, 1) == 0
    assert lib.vol_prepare_workspace(ctypes.byref(pr), 1 << 20, 1 << 20) == 0   # n_vol * n_tgt > 2^31
    # the largest FP32 and FP64 degrees are accepted
    for L, prec in ((64, rs.FP32), (48, rs.FP64)):
        p2, k2 = _vprob(L=L, prec=prec)
        assert rv.vol_prepare_workspace(p2, 2, 1) > 0
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    st = lib.vol_prepare(ctypes.byref(pr), 4, None, 1, fake, None, None, ws, a, None, ctypes.byref(out))
    assert st == 1 and "NULL" in rs.radsvd_last_error()
    st = lib.vol_prepare(ctypes.byref(pr), 4, ctypes.c_void_p(4100), 1, fake, None, None, ws, a, None,
                         ctypes.byref(out))
    assert st == 1 and "aligned" in rs.radsvd_last_error()
    st = lib.vol_prepare(ctypes.byref(pr), 4, fake, 1, fake, None, None, ws, a - 1, None, ctypes.byref(out))
    assert st == 3
    st = lib.vol_prepare(ctypes.byref(pr), 4, fake, 1, fake, None, None, ctypes.c_void_p((1 << 20) + 8), a, None,
                         ctypes.byref(out))
    assert st == 3
    assert lib.vol_align(None, 1, fake, fake, None, None) == 1
    assert lib.vol_get_UV(None, None, None, None, None, None) == 1


def test_volume_euler_angles():
    """best_idx {ib, m1', m2'} -> (gamma, beta, alpha); -1 entries give NaN."""
    from paper_2202_07235_amd import volume as rv
    L, beta = 4, np.array([0.0, 0.5, 1.5])
    M = 2 * L + 1
    idx = np.array([[[2, 3, 7], [-1, -1, -1]]])
    g, b, a = rv.euler_angles(idx, beta, L)
    assert np.allclose([g[0, 0], b[0, 0], a[0, 0]], [2 * np.pi * 7 / M, 1.5, 2 * np.pi * 3 / M])
    assert np.isnan(g[0, 1]) and np.isnan(b[0, 1]) and np.isnan(a[0, 1])
