"""Volume alignment (vol_prepare / vol_align) against the FP64 volume oracle.

* Kernels and principal vectors: the eigenvalues of C and D against the
  oracle's (built from the same, possibly complex64-rounded, coefficients),
  and the principal subspaces by projector distance where the eigenvalue gap
  allows.
* Landscape: the library's U and V are fed to the oracle (any orthonormal
  eigenbasis of a degenerate cluster is as correct as another), and the FULL
  landscape is compared element by element: per pair, max |X_gpu - X_or| /
  max |X_or| <= 1e-5 (FP32) or 1e-10 (FP64).  At H_C = K and H_D = L + 1 the
  comparison is against the direct sum of section 4.4, with no U or V from
  the library at all.
* BEST: the index agrees, or the oracle's value at the library's index is
  within the tolerance of the oracle's maximum (a near-tie).
* Sizes: small cases spanning several workgroups and ragged order grids; the
  largest degrees (L = 64 in FP32 with two blocks of pairs, L = 48 in FP64);
  the paper-shaped workload (96 volumes, one target, K = L = 48, 97 interior
  angles) on every pair's BEST and sampled pairs' landscapes, plus recovery of
  each copy's true rotation to within the grid.
* Edges: L = 1, ranks 1, one interior angle, a NaN volume (its pairs give NaN
  and -1, the others are unaffected), recovery of an exact grid rotation.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import volume as ov
from paper_2202_07235_amd import volume as rv
from synth import volumes as sv

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-10}


def _dev(X, precision):
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    return torch.tensor(np.ascontiguousarray(X), dtype=dt, device="cuda")


def _host(t):
    return t.cpu().to(torch.complex128).numpy()


def _plan(P, precision, H_C=None, H_D=None, betas=None, **kw):
    cfg = P.cfg
    A, B = _dev(P.A, precision), _dev(P.B, precision)
    plan = rv.VolPlan(A, B, P.w, cfg.L, H_C or cfg.H_C, H_D or cfg.H_D,
                      P.beta if betas is None else betas, precision=precision, **kw)
    return plan, _host(A), _host(B)


def _compare(Xg, Xo, tol, label):
    worst = 0.0
    for idx in np.ndindex(Xo.shape[:2]):
        scale = np.abs(Xo[idx]).max()
        err = np.abs(Xg[idx] - Xo[idx]).max() / scale
        worst = max(worst, err)
        assert err <= tol, (label, idx, err)
    print(f"{label}: worst rel err {worst:.2e}")
    return worst


def _check_best(bs, bi, Xo, tol):
    so, io = ov.best(Xo)
    R = Xo.real
    for idx in np.ndindex(so.shape):
        scale = np.abs(Xo[idx]).max()
        if tuple(bi[idx]) != tuple(io[idx]):
            at = R[idx][tuple(bi[idx])]
            assert so[idx] - at <= 2 * tol * scale, (idx, bi[idx], io[idx])
        assert abs(bs[idx] - so[idx]) <= tol * scale + 1e-7 * abs(so[idx]), (idx, bs[idx], so[idx])


def _proj_dist(U1, U2, H):
    return np.abs(U1[:, :H] @ U1[:, :H].T - U2[:, :H] @ U2[:, :H].T).max()


@pytest.mark.parametrize("name,precision,real", [("vtiny", "fp64", False), ("vtiny", "fp32", False),
                                                 ("vsmall", "fp32", False), ("vsmall", "fp64", False),
                                                 ("vtiny", "fp32", True), ("vsmall", "fp32", True),
                                                 ("vsmall", "fp64", True)])
def test_volume_matches_oracle(name, precision, real):
    """real=True: the volumes are real in space (blob maps plus real noise), the
    library computes X from half the orders; the oracle's complex X has an
    imaginary part at rounding level, the library's is exactly zero."""
    cfg = sv.vol_config(name)
    P = sv.make_volume_problem(cfg, seed=2000 + len(name))
    plan, A, B = _plan(P, precision, real=real)
    out = plan.align("best+full")
    U, lc, V, ld = (t.cpu().numpy() for t in plan.UV())
    torch.cuda.synchronize()
    # kernels and principal vectors
    Co, Do = ov.vol_kernel_C(B, P.w, cfg.L), ov.vol_kernel_D(B, P.w, cfg.L)
    lco, ldo = np.linalg.eigvalsh(Co)[::-1], np.linalg.eigvalsh(Do)[::-1]
    assert np.abs(lc - lco).max() <= 1e-11 * lco[0], (lc, lco)
    assert np.abs(ld - ldo).max() <= 1e-11 * ldo[0], (ld, ldo)
    Uo, Vo = np.linalg.eigh(Co)[1][:, ::-1], np.linalg.eigh(Do)[1][:, ::-1]
    if cfg.H_C < cfg.K and lco[cfg.H_C - 1] - lco[cfg.H_C] > 1e-6 * lco[0]:
        assert _proj_dist(U, Uo, cfg.H_C) < 1e-7
    if cfg.H_D <= cfg.L and ldo[cfg.H_D - 1] - ldo[cfg.H_D] > 1e-6 * ldo[0]:
        assert _proj_dist(V, Vo, cfg.H_D) < 1e-7
    # landscape with the library's U, V
    Xo = ov.landscape_all(A, B, P.w, U, cfg.H_C, V, cfg.H_D, cfg.L, P.beta)
    Xg = _host(out["X"])
    if real:
        assert np.all(Xg.imag == 0)
    _compare(Xg, Xo, TOL[precision], f"{name}-{precision}{'-real' if real else ''}")
    _check_best(out["best_score"].cpu().numpy(), out["best_idx"].cpu().numpy(), Xo, TOL[precision])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_volume_complex_inputs(precision):
    """Coefficients that belong to no real volume (independent complex Gaussian
    entries): X is complex, and the general mode must match the oracle in both
    parts."""
    cfg = sv.vol_config("vtiny", n_vol=3, n_tgt=2, L=7, K=5, H_C=4, H_D=6)
    rng = np.random.default_rng(2150)
    nc = (cfg.L + 1) ** 2
    A = rng.standard_normal((cfg.n_vol, cfg.K, nc)) + 1j * rng.standard_normal((cfg.n_vol, cfg.K, nc))
    B = rng.standard_normal((cfg.n_tgt, cfg.K, nc)) + 1j * rng.standard_normal((cfg.n_tgt, cfg.K, nc))
    k, w = sv.shell_grid(cfg.k_max, cfg.K)
    P = sv.VolProblem(cfg, k, w, sv.beta_grid(9), A, B, {})
    plan, Ah, Bh = _plan(P, precision)
    out = plan.align("best+full")
    U, _, V, _ = (t.cpu().numpy() for t in plan.UV())
    Xo = ov.landscape_all(Ah, Bh, w, U, cfg.H_C, V, cfg.H_D, cfg.L, P.beta)
    assert np.abs(Xo.imag).max() > 0.1 * np.abs(Xo).max()   # genuinely complex
    _compare(_host(out["X"]), Xo, TOL[precision], f"complex inputs {precision}")
    _check_best(out["best_score"].cpu().numpy(), out["best_idx"].cpu().numpy(), Xo, TOL[precision])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_volume_full_rank_equals_direct_sum(precision):
    cfg = sv.vol_config("vtiny", n_vol=3, n_tgt=2)
    P = sv.make_volume_problem(cfg, seed=2100)
    betas = np.array([0.0, 0.4, 1.7, 3.0, 5.5])
    plan, A, B = _plan(P, precision, H_C=cfg.K, H_D=cfg.L + 1, betas=betas)
    X = _host(plan.align("full")["X"])
    Xd = np.stack([np.stack([ov.landscape_direct(A[a], B[b], P.w, cfg.L, betas) for b in range(2)])
                   for a in range(3)])
    _compare(X, Xd, TOL[precision], f"full-rank {precision}")


def test_volume_recovers_grid_rotation():
    L, K = 10, 8
    M = 2 * L + 1
    rng = np.random.default_rng(2200)
    mu, s, c = sv.blob_params_3d(rng, 1, 10, 0.5)
    k, w = sv.shell_grid(8.0, K)
    Bc = sv.sh_coeffs(mu, s, c, k, L)
    rots = [(3, 5, 17), (0, 1, 2), (20, 10, 7)]
    Ac = np.concatenate([sv.sh_coeffs((sv.rotation_matrix(2 * math.pi * p / M, 2 * math.pi * q / M,
                                                          2 * math.pi * t / M) @ mu[0].T).T[None], s, c, k, L)
                         for p, q, t in rots])
    plan = rv.VolPlan(_dev(Ac, "fp64"), _dev(Bc, "fp64"), w, L, K, L + 1, sv.beta_grid(M), precision="fp64")
    out = plan.align("best")
    bi = out["best_idx"].cpu().numpy()
    # <A, R_tau B> with A = R0 B is largest where R_tau = R0: (ib, m1', m2') = (q, p, t)
    for i, (p, q, t) in enumerate(rots):
        assert tuple(bi[i, 0]) == (q, p, t), (i, bi[i, 0])


def test_volume_edges():
    # L = 1, ranks 1, one interior angle
    cfg = sv.vol_config("vtiny", L=1, K=3, H_C=1, H_D=1, n_vol=3, n_tgt=1, n_beta=1)
    P = sv.make_volume_problem(cfg, seed=2300)
    plan, A, B = _plan(P, "fp64", betas=np.array([0.9]))
    out = plan.align("best+full")
    U, _, V, _ = (t.cpu().numpy() for t in plan.UV())
    Xo = ov.landscape_all(A, B, P.w, U, 1, V, 1, 1, [0.9])
    _compare(_host(out["X"]), Xo, 1e-10, "L=1")
    _check_best(out["best_score"].cpu().numpy(), out["best_idx"].cpu().numpy(), Xo, 1e-10)
    # a NaN in one volume: its pairs are NaN / -1, the rest as before
    cfg = sv.vol_config("vtiny", n_vol=4, n_tgt=2)
    P = sv.make_volume_problem(cfg, seed=2301)
    plan, A, B = _plan(P, "fp32")
    ref = plan.align("best")
    ref = {k: v.clone() for k, v in ref.items()}
    A2 = P.A.copy()
    A2[2, 1, 5] = np.nan
    P2 = sv.VolProblem(cfg, P.k, P.w, P.beta, A2, P.B, P.truth)
    U, _, V, _ = plan.UV()
    plan2, _, _ = _plan(P2, "fp32", U=U[:, :cfg.H_C], V=V[:, :cfg.H_D])
    out = plan2.align("best")
    bs, bi = out["best_score"].cpu().numpy(), out["best_idx"].cpu().numpy()
    assert np.isnan(bs[2]).all() and (bi[2] == -1).all()
    keep = [0, 1, 3]
    assert np.array_equal(bs[keep], ref["best_score"].cpu().numpy()[keep])
    assert np.array_equal(bi[keep], ref["best_idx"].cpu().numpy()[keep])
    # caller-supplied U, V: eigenvalues reported NaN
    _, lc, _, ld = plan2.UV()
    assert torch.isnan(lc).all() and torch.isnan(ld).all()
    # only U supplied: V (and its eigenvalues) from the degree kernel, results as before
    plan3, _, _ = _plan(P, "fp32", U=U[:, :cfg.H_C])
    out3 = plan3.align("best")
    _, lc3, V3, ld3 = plan3.UV()
    assert torch.isnan(lc3).all() and torch.isfinite(ld3).all()
    assert torch.equal(V3[:, :cfg.H_D], V[:, :cfg.H_D])
    assert np.array_equal(out3["best_score"].cpu().numpy(), ref["best_score"].cpu().numpy())


@pytest.mark.parametrize("L,precision,n_vol,real", [(64, "fp32", 130, False), (48, "fp64", 3, False),
                                                    (64, "fp32", 130, True)])
def test_volume_largest_degree(L, precision, n_vol, real):
    """The largest supported degree; for FP32 at H_D = L + 1 the 130 pairs span
    two blocks of pairs (the per-pair intermediates take 11.8 MB, so a block of
    the 1 GiB scratch holds 90 pairs)."""
    cfg = sv.vol_config("vtiny", K=12, L=L, k_max=L / 2, n_vol=n_vol, n_tgt=1, n_blobs=8, H_C=6, H_D=L + 1,
                        n_beta=2)
    P = sv.make_volume_problem(cfg, seed=2400 + L)
    betas = np.array([0.8, 2.6])
    plan, A, B = _plan(P, precision, betas=betas, real=real)
    out = plan.align("best+full")
    U, _, V, _ = (t.cpu().numpy() for t in plan.UV())
    pairs = [(0, 0), (n_vol // 2, 0), (n_vol - 1, 0)]
    if n_vol > 92:
        pairs += [(89, 0), (90, 0), (91, 0)]
    Xo = ov.landscape_all(A, B, P.w, U, cfg.H_C, V, cfg.H_D, L, betas, pairs=pairs)
    Xg = np.stack([_host(out["X"][a, b]) for a, b in pairs])
    _compare(Xg[:, None], Xo[:, None], TOL[precision], f"L={L} {precision}")
    _check_best(np.array([out["best_score"][a, b].item() for a, b in pairs])[:, None],
                np.stack([out["best_idx"][a, b].cpu().numpy() for a, b in pairs])[:, None], Xo[:, None],
                TOL[precision])


@pytest.mark.parametrize("L,precision", [(15, "fp32"), (17, "fp32"), (20, "fp32"), (17, "fp64")])
def test_volume_real_row_blocks(L, precision):
    """Real volumes: the L + 1 rows of the first product in blocks of 16 on the
    matrix cores, with one or two rows past the last full block on the vector
    units: 16 rows (one block), 18 (one block and two rows), 21 (two blocks,
    the second partly masked)."""
    cfg = sv.vol_config("vtiny", K=6, L=L, k_max=L / 2, n_vol=4, n_tgt=2, n_blobs=6, H_C=6, H_D=8, n_beta=5)
    P = sv.make_volume_problem(cfg, seed=2600 + L)
    plan, A, B = _plan(P, precision, real=True)
    out = plan.align("best+full")
    U, _, V, _ = (t.cpu().numpy() for t in plan.UV())
    Xo = ov.landscape_all(A, B, P.w, U, cfg.H_C, V, cfg.H_D, L, P.beta)
    Xg = _host(out["X"])
    assert np.all(Xg.imag == 0)
    _compare(Xg, Xo, TOL[precision], f"real L={L} {precision}")
    _check_best(out["best_score"].cpu().numpy(), out["best_idx"].cpu().numpy(), Xo, TOL[precision])


def _rot_angle(R):
    return math.acos(max(-1.0, min(1.0, (np.trace(R) - 1) / 2)))


@pytest.mark.parametrize("real", [False, True])
def test_volume_paper_shaped_workload(real):
    """96 noisy rotated copies against one target, K = L = 48, 97 angles."""
    cfg = sv.vol_config("volume")
    P = sv.make_volume_problem(cfg, seed=2500)
    plan, A, B = _plan(P, "fp32", real=real)
    out = plan.align("best+full")
    U, _, V, _ = (t.cpu().numpy() for t in plan.UV())
    bs, bi = out["best_score"].cpu().numpy(), out["best_idx"].cpu().numpy()
    sample = [0, 47, 95]
    Xo = ov.landscape_all(A, B, P.w, U, cfg.H_C, V, cfg.H_D, cfg.L, P.beta, pairs=[(a, 0) for a in sample])
    Xg = np.stack([_host(out["X"][a, 0]) for a in sample])
    _compare(Xg[:, None], Xo[:, None], 1e-5, "volume workload (sampled)")
    _check_best(bs[sample], bi[sample], Xo[:, None], 1e-5)
    # every pair: the best grid rotation is close to the copy's true rotation
    # (A = R_true B + noise; noise, rank and grid allow a few grid steps)
    M = 2 * cfg.L + 1
    step = 2 * math.pi / M
    worst = 0.0
    gam, bet, alp = rv.euler_angles(out["best_idx"], P.beta, cfg.L)
    for a in range(cfg.n_vol):
        Rb = sv.rotation_matrix(alp[a, 0], bet[a, 0], gam[a, 0])
        ang = _rot_angle(Rb @ P.truth["rot"][a].T)
        worst = max(worst, ang)
        assert ang <= 3 * step, (a, ang)
    print(f"worst rotation error {worst:.3f} rad (grid step {step:.3f})")


def test_volume_quality_measures():
    """The quality measures of the paper's volume example (section 4.10: relative
    Frobenius error, correlation and percentile f of a low-rank landscape against
    the full sum), computed by the library's metrics kernel on volume landscapes,
    against the oracle's measures of the same arrays; at full rank they are exact
    (0, 1, 1)."""
    from paper_2202_07235_amd import march
    cfg = sv.vol_config("vsmall", n_vol=8, n_tgt=2)
    P = sv.make_volume_problem(cfg, seed=2600)
    full, A, B = _plan(P, "fp32", H_C=cfg.K, H_D=cfg.L + 1, real=True)
    Xr = full.align("full")["X"]
    low, _, _ = _plan(P, "fp32", H_C=4, H_D=4, real=True)
    Xe = low.align("full")["X"]
    m = march.landscape_metrics(Xe, Xr)
    n = cfg.n_vol * cfg.n_tgt
    rel, corr, f = oracle.landscape_metrics(_host(Xe).reshape(n, -1), _host(Xr).reshape(n, -1))
    assert abs(m["rel_fro"] - rel) <= 1e-9 * max(1.0, rel)
    assert abs(m["corr"] - corr) <= 1e-9
    assert np.array_equal(m["f"].cpu().numpy().ravel(), f.astype(np.float32))
    print(f"rank 4/4 of {cfg.K}/{cfg.L + 1}: rel fro {m['rel_fro']:.3f}, corr {m['corr']:.4f}, mean f {m['mean_f']:.4f}")
    assert m["rel_fro"] > 0.0
    same = march.landscape_metrics(Xr, Xr)
    assert same["rel_fro"] == 0.0 and abs(same["corr"] - 1.0) < 1e-12 and same["mean_f"] == 1.0
    # a non-finite value makes that pair's f NaN (landscapes this long take the
    # workgroup-per-pair kernel)
    Xn = Xe.clone()
    Xn[3, 1, 5, 7, 2] = float("nan")
    mn = march.landscape_metrics(Xn, Xr)
    fn = mn["f"].cpu().numpy()
    assert np.isnan(fn[3, 1]) and np.isfinite(np.delete(fn.ravel(), 3 * cfg.n_tgt + 1)).all()


def test_volume_largest_shell_and_angle_counts():
    """K = 128 shells (the eigensolver's largest matrix) and 256 interior angles,
    FP64: eigenvalues of C against the oracle's and the landscape of every pair."""
    cfg = sv.vol_config("vtiny", K=128, L=5, k_max=8.0, n_vol=2, n_tgt=2, n_blobs=6, H_C=12, H_D=5, n_beta=256)
    P = sv.make_volume_problem(cfg, seed=2700)
    plan, A, B = _plan(P, "fp64", betas=sv.beta_grid(256), real=True)
    out = plan.align("best+full")
    U, lc, V, _ = (t.cpu().numpy() for t in plan.UV())
    lco = np.linalg.eigvalsh(ov.vol_kernel_C(B, P.w, cfg.L))[::-1]
    assert np.abs(lc - lco).max() <= 1e-11 * lco[0]
    Xo = ov.landscape_all(A, B, P.w, U, cfg.H_C, V, cfg.H_D, cfg.L, sv.beta_grid(256))
    _compare(_host(out["X"]), Xo, 1e-10, "K=128, 256 angles")
    _check_best(out["best_score"].cpu().numpy(), out["best_idx"].cpu().numpy(), Xo, 1e-10)


def test_volume_align_graph_replays():
    """vol_align launches kernels only (no allocation, no memset), so it can be
    captured in a HIP graph: three replays, with eager work on the outputs in
    between, each equal bitwise to the eager call."""
    cfg = sv.vol_config("vsmall", n_vol=5, n_tgt=2)
    P = sv.make_volume_problem(cfg, seed=2800)
    plan, _, _ = _plan(P, "fp32", real=True)
    ref = plan.align("best+full")
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    outs = {k: torch.empty_like(v) for k, v in ref.items()}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.align("best+full", outputs=outs)   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.align("best+full", outputs=outs)
    for rep in range(3):
        for v in outs.values():
            v.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(outs[k], ref[k]), (rep, k)


def test_volume_block_boundary_inside_a_row():
    """Several targets per volume with a block-of-pairs boundary inside one
    volume's row (L = 64, H_D = 65: 90 pairs per block; 14 x 7 pairs split at
    pair 90 = volume 12, target 6)."""
    cfg = sv.vol_config("vtiny", K=10, L=64, k_max=32.0, n_vol=14, n_tgt=7, n_blobs=6, H_C=5, H_D=65, n_beta=2)
    P = sv.make_volume_problem(cfg, seed=2900)
    betas = np.array([0.7, 2.2])
    plan, A, B = _plan(P, "fp32", betas=betas, real=True)
    out = plan.align("best+full")
    U, _, V, _ = (t.cpu().numpy() for t in plan.UV())
    pairs = [(12, 4), (12, 5), (12, 6), (13, 0), (0, 0), (13, 6)]
    Xo = ov.landscape_all(A, B, P.w, U, cfg.H_C, V, cfg.H_D, cfg.L, betas, pairs=pairs)
    Xg = np.stack([_host(out["X"][a, b]) for a, b in pairs])
    _compare(Xg[:, None], Xo[:, None], 1e-5, "block boundary inside a row")
    _check_best(np.array([out["best_score"][a, b].item() for a, b in pairs])[:, None],
                np.stack([out["best_idx"][a, b].cpu().numpy() for a, b in pairs])[:, None], Xo[:, None], 1e-5)
