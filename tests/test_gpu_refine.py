"""Rotations off the grid (align_refine_rotation) against the oracle.

* For each pair, the oracle's own best grid pose (m, t) is handed to the
  library, which evaluates the landscape at 2R - 1 rotations within one grid
  step; the oracle evaluates the same rotations by rotating the target's
  principal rings with the Fourier-Bessel phase (section 2.2) and summing in
  psi-space.  The fine index must agree (or, at a near-tie, the library's
  choice must be within the tolerance of the oracle's maximum), and the score
  to 1e-5 of the pair's max |X| (FP32 sums) or 1e-7 (FP64 sums; the score
  is returned in f32, whose rounding is 6e-8 of its value).
* Recovery: targets that are exactly band-limited rotations of the images by
  angles off the grid; the refined angle lands within one fine step of the
  true one (the nearest fine rotation, or the other one that brackets the
  peak), never farther than the grid angle.
* R = 1 reproduces the grid landscape; pairs without a best give NaN and -1;
  R outside [1, 64] is refused.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2202_07235_amd as rs
import synth
from tests._parity import host_inputs, to_device

pytestmark = pytest.mark.gpu


def _oracle_refine(Ar, Br, m, t, R, Q):
    """argmax over j of Re X(2 pi (R m + j) / (R Q)), |j| < R (first max)."""
    js = np.arange(-R + 1, R)
    g = 2 * math.pi * (R * m + js) / (R * Q)
    X = oracle.landscape_offgrid(Ar, Br[t], g).real
    i = int(np.argmax(X))
    return X, i, js


@pytest.mark.parametrize("precision,products,hermitian,Q,R", [
    ("fp32", 3, True, 128, 8), ("fp64", 3, True, 64, 4), ("fp32", 3, False, 64, 8),
    ("bf16x3", 6, True, 512, 4), ("bf16x3", 3, True, 96, 16)])
def test_refine_matches_oracle(precision, products, hermitian, Q, R):
    if hermitian:
        cfg = synth.config("fp32", N=Q // 2, K=Q // 4, Q=Q, n_img=7, n_tgt=11, T=4, H=10, n_blobs=8, snr=0.5)
    else:
        cfg = synth.config("tiny", n_img=5, n_tgt=6, H=9)
    P = synth.make_problem(cfg, seed=1300 + Q)
    A, B = to_device(P, precision)
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision, products=products, hermitian=hermitian)
    U = plan.U_lambda()[0].cpu().numpy()
    A_h, B_h = host_inputs(A, B)
    Ar = oracle.principal_rings(A_h, U, cfg.H, P.w, cfg.Q)
    Br = oracle.principal_rings(B_h, U, cfg.H, P.w, cfg.Q, k=P.k, delta=P.delta)
    X = oracle.landscape_rings(Ar, Br)
    _, m_or, t_or = oracle.best(X)
    best = {"best_m": torch.tensor(m_or, dtype=torch.int32, device="cuda"),
            "best_t": torch.tensor(t_or, dtype=torch.int32, device="cuda")}
    out = plan.refine_rotation(best, R)
    torch.cuda.synchronize()
    fs, fm = out["fine_score"].cpu().numpy(), out["fine_m"].cpu().numpy()
    tol = 1e-7 if precision == "fp64" else 1e-5
    worst = 0.0
    for a in range(cfg.n_img):
        for b in range(cfg.n_tgt):
            m, t = int(m_or[a, b]), int(t_or[a, b])
            Xj, i, js = _oracle_refine(Ar[a], Br[b], m, t, R, cfg.Q)
            scale = np.abs(X[a, b]).max()
            want = (R * m + js[i]) % (R * cfg.Q)
            if fm[a, b] != want:   # a near-tie: the library's choice must be (almost) as good
                k = (fm[a, b] - R * m + R * cfg.Q // 2) % (R * cfg.Q) - R * cfg.Q // 2
                assert -R < k < R, (a, b, fm[a, b], want)
                assert Xj[i] - Xj[k + R - 1] <= 2 * tol * scale
            err = abs(fs[a, b] - Xj[i]) / scale
            worst = max(worst, err)
            assert err <= tol, (a, b, err)
    print(f"{precision}-{products} Q={Q} R={R}: worst score err {worst:.2e}")


def test_refine_recovers_off_grid_rotations():
    Q, K, H, R = 128, 32, 12, 16
    cfg = synth.config("fp32", N=Q // 2, K=K, Q=Q, n_img=6, n_tgt=6, T=1, H=H, n_blobs=8, snr=0.5)
    P = synth.make_problem(cfg, seed=1401)
    A = P.A.numpy()
    # remove each ring's q = Q/2 term: the rotation below is then an exact
    # band-limited rotation and composes exactly
    c = np.fft.fft(A, axis=-1)
    c[..., Q // 2] = 0.0
    A = np.fft.ifft(c, axis=-1)
    rng = np.random.default_rng(7)
    g0 = 2 * math.pi * rng.random(cfg.n_tgt)
    B = np.stack([oracle.rotate_ring(A[i], g0[i]) for i in range(cfg.n_tgt)])
    At = torch.tensor(A, dtype=torch.complex64, device="cuda")
    Bt = torch.tensor(B, dtype=torch.complex64, device="cuda")
    plan = rs.Plan(At, Bt, P.k, P.w, None, H, precision="fp32")
    best = plan.pairs("best")
    out = plan.refine_rotation(best, R)
    torch.cuda.synchronize()
    g = out["gamma"].cpu().numpy()
    m = best["best_m"].cpu().numpy()
    for i in range(cfg.n_tgt):
        truth = (-g0[i]) % (2 * math.pi)
        d_fine = abs((g[i, i] - truth + math.pi) % (2 * math.pi) - math.pi)
        d_grid = abs((2 * math.pi * m[i, i] / Q - truth + math.pi) % (2 * math.pi) - math.pi)
        print(f"target {i}: grid error {d_grid:.2e}, refined error {d_fine:.2e} rad")
        assert d_fine <= 2 * math.pi / (R * Q) * 1.0001
        assert d_fine <= d_grid + 1e-12


def test_refine_edges():
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=3, n_tgt=5, T=4, H=6, n_blobs=8, snr=0.5)
    P = synth.make_problem(cfg, seed=1500)
    A, B = to_device(P, "fp32")
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="fp32")
    best = plan.pairs("best+full")
    X = best["X"].real.cpu().numpy()
    bm = best["best_m"].clone()
    bm[1, 3] = -1
    out = plan.refine_rotation({"best_m": bm, "best_t": best["best_t"]}, 1)
    torch.cuda.synchronize()
    fs, fm = out["fine_score"].cpu().numpy(), out["fine_m"].cpu().numpy()
    m, t = best["best_m"].cpu().numpy(), best["best_t"].cpu().numpy()
    assert np.isnan(fs[1, 3]) and fm[1, 3] == -1
    mask = np.ones_like(fm, dtype=bool)
    mask[1, 3] = False
    assert np.array_equal(fm[mask], m[mask])
    at = np.take_along_axis(X.reshape(3, 5, -1), (t * cfg.Q + m)[..., None], axis=-1)[..., 0]
    assert np.allclose(fs[mask], at[mask], rtol=0, atol=1e-5 * np.abs(X).max())
    for bad in (0, 65):
        with pytest.raises(rs.RadsvdError, match="INVALID_ARG"):
            plan.refine_rotation(best, bad)
