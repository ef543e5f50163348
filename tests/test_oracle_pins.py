"""Pins of the FP64 oracle against facts that the paper and the mathematics
fix, computed by routes independent of the oracle's own code:

* closed-form blob transform vs brute-force real-space quadrature;
* the semi-analytic landscape (angular integral of a plane wave = 2 pi J_0);
* the paper's two-step FFT evaluation (section 2.4) at full rank;
* exact rotation / translation equivariance on the grid;
* Hermitian symmetry; swap symmetry;
* kernel C against its q-sum form and against the brute-force
  rotation-averaged objective of section 3.3;
* truncation identity and error bound for H < K;
* best / lse decisions against hand-made landscapes and scipy.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special
import torch

import oracle
import synth


def _rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(1e-300, np.max(np.abs(np.asarray(b))))


# --------------------------------------------------------------------------
# inputs: closed-form transform
# --------------------------------------------------------------------------
def test_closed_form_ft_matches_realspace_quadrature():
    rng = np.random.default_rng(1)
    mu, s, c = synth.blob_params(rng, 1, 16)
    h = 0.005
    x = np.arange(-1.0, 1.0 + 0.5 * h, h)
    X, Y = np.meshgrid(x, x, indexing="ij")
    img = np.zeros_like(X)
    for i in range(16):
        img += c[0, i] * np.exp(-((X - mu[0, i, 0]) ** 2 + (Y - mu[0, i, 1]) ** 2) / (2 * s[0, i] ** 2))
    k, w = synth.gl_grid(32, 16)
    Q = 64
    F = synth.polar_ft(mu, s, c, k, Q).numpy()[0]
    psi = 2 * math.pi * np.arange(Q) / Q
    for (r, j) in [(0, 0), (3, 5), (7, 17), (11, 33), (15, 63)]:
        kx, ky = k[r] * math.cos(psi[j]), k[r] * math.sin(psi[j])
        brute = (img * np.exp(-1j * (kx * X + ky * Y))).sum() * h * h
        assert abs(brute - F[r, j]) <= 1e-12 * np.max(np.abs(F))


def test_gl_grid_integrates_k_weighted_polynomials():
    k, w = synth.gl_grid(32, 16)
    kmax = 16.0
    for p in range(0, 25):
        exact = kmax ** (p + 2) / (p + 2)
        assert abs(np.sum(k ** p * w) - exact) <= 1e-12 * exact


def test_hermitian_noise_is_conjugate_symmetric():
    cfg = synth.config("fp32", n_img=3, n_tgt=4, N=32, K=8, Q=32, T=1)
    P = synth.make_problem(cfg, seed=5)
    B = P.B.numpy()
    Q = cfg.Q
    assert np.allclose(B[:, :, Q // 2:], np.conj(B[:, :, :Q // 2]), rtol=0, atol=1e-12 * np.abs(B).max())


# --------------------------------------------------------------------------
# landscape: semi-analytic pin (P2) over every pair of a tiny problem (P8)
# --------------------------------------------------------------------------
def _semi_analytic(muA, sA, cA, muB, sB, cB, gamma, delta, kmax):
    """X(gamma, delta) = sum_{i,i'} c c' (2 pi s^2)(2 pi s'^2) 2 pi
    int_0^kmax exp(-(s^2+s'^2) k^2/2) J0(k |mu_i - mu''_i'|) k dk,
    mu'' = R_gamma (mu' + delta)."""
    cg, sg = math.cos(gamma), math.sin(gamma)
    m = muB + delta[None, :]
    mpp = np.stack([cg * m[:, 0] - sg * m[:, 1], sg * m[:, 0] + cg * m[:, 1]], axis=-1)
    tot = 0.0
    for i in range(len(sA)):
        for ip in range(len(sB)):
            d = float(np.hypot(*(muA[i] - mpp[ip])))
            ss = sA[i] ** 2 + sB[ip] ** 2
            f = lambda kk: math.exp(-0.5 * ss * kk * kk) * scipy.special.j0(kk * d) * kk
            val, _ = scipy.integrate.quad(f, 0.0, kmax, epsabs=1e-16, epsrel=1e-13, limit=400)
            tot += cA[i] * cB[ip] * (2 * math.pi * sA[i] ** 2) * (2 * math.pi * sB[ip] ** 2) * 2 * math.pi * val
    return tot


def test_landscape_matches_semi_analytic_bessel_integral():
    N, K, Q = 32, 16, 64
    rng = np.random.default_rng(11)
    nA, nB, nbl = 3, 3, 4
    muA, sA, cA = synth.blob_params(rng, nA, nbl)
    muB, sB, cB = synth.blob_params(rng, nB, nbl)
    k, w = synth.gl_grid(N, K)
    delta = synth.translation_grid(9, N)
    A = synth.polar_ft(muA, sA, cA, k, Q)
    B = synth.polar_ft(muB, sB, cB, k, Q)
    U, lam = oracle.principal_vectors(oracle.kernel_C(B, w, Q))
    X = oracle.landscape(A, B, U, K, k, w, delta)
    scale = np.abs(X).max()
    for a in range(nA):
        for b in range(nB):
            for t in (1, 4, 5, 8):
                for m in (0, 7, 40):
                    ref = _semi_analytic(muA[a], sA[a], cA[a], muB[b], sB[b], cB[b],
                                         2 * math.pi * m / Q, delta[t], N / 2)
                    assert abs(X[a, b, t, m] - ref) <= 1e-11 * scale, (a, b, t, m)


# --------------------------------------------------------------------------
# full rank equals the paper's two-step route (P3)
# --------------------------------------------------------------------------
def _two_step_paper(A, B, k, w, delta, Q):
    """Section 2.4: a(k,q) = sum_j Ahat(k,psi_j) e^{-i q psi_j} dpsi;
    Step 1 Xhat(q) = 2 pi sum_r w_r conj(a(k_r,q)) b(k_r,q);
    Step 2 X(gamma_m) = sum_q e^{-i q gamma_m} Xhat(q)."""
    dpsi = 2 * math.pi / Q
    psi = dpsi * np.arange(Q)
    a = np.fft.fft(A, axis=-1) * dpsi                      # [na][K][Q]
    out = np.zeros((A.shape[0], B.shape[0], len(delta), Q), dtype=np.complex128)
    for t, d in enumerate(delta):
        ph = np.exp(-1j * k[:, None] * (d[0] * np.cos(psi)[None] + d[1] * np.sin(psi)[None]))
        b = np.fft.fft(B * ph[None], axis=-1) * dpsi       # [nb][K][Q]
        Xh = 2 * math.pi * np.einsum("r,arq,brq->abq", w, np.conj(a), b)
        out[:, :, t, :] = np.fft.fft(Xh, axis=-1)          # sum_q Xh e^{-2 pi i q m / Q}
    return out


@pytest.mark.parametrize("hermitian", [True, False])
def test_full_rank_equals_two_step_route(hermitian):
    cfg = synth.config("tiny", n_img=4, n_tgt=5, T=9) if not hermitian else \
        synth.config("fp32", N=32, K=16, Q=64, n_img=4, n_tgt=5, T=9, H=16)
    P = synth.make_problem(cfg, seed=3)
    A, B = P.A.numpy(), P.B.numpy()
    U, lam = oracle.principal_vectors(oracle.kernel_C(B, P.w, cfg.Q))
    X = oracle.landscape(A, B, U, cfg.K, P.k, P.w, P.delta)
    ref = _two_step_paper(A, B, P.k, P.w, P.delta, cfg.Q) / (2 * math.pi) ** 2
    assert _rel(X, ref) <= 1e-12


# --------------------------------------------------------------------------
# equivariance and symmetry (P4, P5)
# --------------------------------------------------------------------------
def test_grid_rotation_is_an_exact_index_shift():
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=3, n_tgt=3, T=1, H=6)
    P = synth.make_problem(cfg, seed=4)
    A = P.A.numpy()
    U, _ = oracle.principal_vectors(oracle.kernel_C(P.B, P.w, cfg.Q))
    shifts = [5, 17, 40]
    B = np.stack([np.roll(A[i], shifts[i], axis=-1) for i in range(3)])  # R_{gamma_p} A
    X = oracle.landscape(A, B, U, cfg.H, P.k, P.w, P.delta)
    Xaa = oracle.landscape(A, A, U, cfg.H, P.k, P.w, P.delta)
    for i, p in enumerate(shifts):
        assert _rel(X[i, i, 0], np.roll(Xaa[i, i, 0], -p)) <= 1e-14
        score, m, t = oracle.best(X[i:i + 1, i:i + 1])
        assert int(m[0, 0]) == (-p) % cfg.Q


def test_translation_composes_exactly():
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=2, n_tgt=2, T=9, H=7)
    P = synth.make_problem(cfg, seed=6)
    A = P.A.numpy()
    U, _ = oracle.principal_vectors(oracle.kernel_C(P.B, P.w, cfg.Q))
    d0 = np.array([0.013, -0.021])
    TA = A * oracle.phase(P.k, d0[None], cfg.Q)[0][None]        # FT of A(x - d0)
    X1 = oracle.landscape(A, TA, U, cfg.H, P.k, P.w, P.delta)
    X2 = oracle.landscape(A, A, U, cfg.H, P.k, P.w, P.delta + d0[None])
    assert _rel(X1, X2) <= 1e-13


def test_hermitian_inputs_give_real_landscape_and_swap_symmetry():
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=3, n_tgt=4, T=1, H=5)
    P = synth.make_problem(cfg, seed=8)
    A, B = P.A.numpy(), P.B.numpy()
    U, _ = oracle.principal_vectors(oracle.kernel_C(B, P.w, cfg.Q))
    X = oracle.landscape(A, B, U, cfg.H, P.k, P.w, P.delta)
    assert np.max(np.abs(X.imag)) <= 1e-14 * np.max(np.abs(X))
    Y = oracle.landscape(B, A, U, cfg.H, P.k, P.w, P.delta)     # X(gamma;A,B) = conj X(-gamma;B,A)
    Yr = np.conj(np.roll(Y[..., ::-1], 1, axis=-1))
    assert _rel(X, np.transpose(Yr, (1, 0, 2, 3))) <= 1e-14


# --------------------------------------------------------------------------
# kernel C (sections 3.3 - 3.4)
# --------------------------------------------------------------------------
def test_kernel_C_matches_q_sum_form():
    cfg = synth.config("tiny", n_img=2, n_tgt=6)
    P = synth.make_problem(cfg, seed=2)
    B = P.B.numpy()
    Q = cfg.Q
    e = oracle.eta(P.w, Q)
    bq = np.fft.fft(B * e[None, :, None], axis=-1) / math.sqrt(Q)
    bq[:, :, 0] = 0.0
    ref = np.einsum("brq,bsq->rs", np.conj(bq), bq).real / B.shape[0]
    C = oracle.kernel_C(B, P.w, Q)
    assert _rel(C, ref) <= 1e-13
    assert np.allclose(C, C.T, rtol=0, atol=0)
    assert np.linalg.eigvalsh(C).min() >= -1e-12 * np.abs(C).max()


def test_kernel_C_is_the_rotation_averaged_objective():
    """eq. for C(u;B) with on-grid gamma, gamma': the double sum over
    rotations of sum_j |[u^T R_g B] - [u^T R_g' B]|^2 equals 2 Q^2 u^T C u."""
    cfg = synth.config("fp32", N=32, K=8, Q=16, n_img=1, n_tgt=1, T=1)
    P = synth.make_problem(cfg, seed=9)
    B = P.B.numpy()[0]
    Q = cfg.Q
    e = oracle.eta(P.w, Q)
    C = oracle.kernel_C(P.B, P.w, Q)
    rng = np.random.default_rng(0)
    for _ in range(3):
        u = rng.standard_normal(cfg.K)
        u /= np.linalg.norm(u)
        tot = 0.0
        for m in range(Q):
            ym = (u * e) @ np.roll(B, m, axis=-1)
            for mp in range(Q):
                ymp = (u * e) @ np.roll(B, mp, axis=-1)
                tot += np.sum(np.abs(ym - ymp) ** 2)
        assert abs(tot - 2 * Q * Q * (u @ C @ u)) <= 1e-11 * tot


def _gauss_hermite_2d(sigma, n):
    """Nodes and weights (summing to 1) of an n x n Gauss-Hermite rule for
    the isotropic Gaussian of standard deviation sigma on R^2."""
    x, wt = np.polynomial.hermite.hermgauss(n)
    d1 = math.sqrt(2.0) * sigma * x
    w1 = wt / math.sqrt(math.pi)
    D = np.array([(a, b) for a in d1 for b in d1])
    W = np.outer(w1, w1).reshape(-1)
    return D, W


def test_translated_kernel_is_the_translation_and_rotation_averaged_objective():
    """Section 5: the sum over pairs of poses (grid rotations g, g'; Gaussian
    translations d, d') of sum_j |[u^T T_d R_g B](psi_j) - [u^T T_d' R_g' B](psi_j)|^2
    is 2 Q^2 u^T C u.  Brute force: every pose pair, translations by a 10 x 10
    Gauss-Hermite rule (exact to ~1e-15 here: k sigma <= 1)."""
    cfg = synth.config("fp32", N=32, K=8, Q=16, n_img=1, n_tgt=1, T=1)
    P = synth.make_problem(cfg, seed=9)
    B = P.B.numpy()[0]
    Q, K = cfg.Q, cfg.K
    sigma = 1.0 / float(np.max(P.k))
    e = oracle.eta(P.w, Q)
    D, W = _gauss_hermite_2d(sigma, 10)
    psi = 2 * math.pi * np.arange(Q) / Q
    C = oracle.kernel_C_translated(P.B, P.w, Q, P.k, sigma)
    rng = np.random.default_rng(0)
    for _ in range(3):
        u = rng.standard_normal(K)
        u /= np.linalg.norm(u)
        # y[(m, i)][j] = sum_r u_r eta_r exp(-i k_r d_i.n(psi_j)) B[r, j - m]
        ys, ws = [], []
        for m in range(Q):
            Bm = np.roll(B, m, axis=-1)
            for d, wd in zip(D, W):
                ph = np.exp(-1j * P.k[:, None] * (d[0] * np.cos(psi) + d[1] * np.sin(psi))[None, :])
                ys.append((u * e) @ (ph * Bm))
                ws.append(wd)
        Y, Wv = np.array(ys), np.array(ws)
        tot = 0.0
        for i in range(0, len(Y), 200):   # every pair of poses, weighted
            dif = Y[i:i + 200, None, :] - Y[None, :, :]
            tot += float(np.einsum("a,b,abj->", Wv[i:i + 200], Wv, np.abs(dif) ** 2))
        assert abs(tot - 2 * Q * Q * (u @ C @ u)) <= 1e-11 * tot, (tot, 2 * Q * Q * (u @ C @ u))


def test_translated_kernel_factors_and_limits():
    k = np.linspace(0.05, 40.0, 97)
    for sigma in (0.0, 0.013, 0.1, 0.7):
        Ep, Em = oracle.translation_factors(k, sigma)
        # I_{+-1/2} are elementary: E- reduces to exp(-sigma^2 k^2 / 2), E+ to exp(-sigma^2 (k - k')^2 / 2)
        ref = np.exp(-0.5 * (sigma * k) ** 2)
        big = ref > 1e-6
        assert np.allclose(Em[big], ref[big], rtol=1e-9, atol=0)
        assert np.all(np.abs(Em - ref) <= 1e-12)
        assert np.allclose(Ep, np.exp(-0.5 * sigma ** 2 * (k[:, None] - k[None, :]) ** 2), rtol=1e-12, atol=0)
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=1, n_tgt=9, T=1)
    P = synth.make_problem(cfg, seed=12)
    C0 = oracle.kernel_C(P.B, P.w, cfg.Q)
    assert _rel(oracle.kernel_C_translated(P.B, P.w, cfg.Q, P.k, 0.0), C0) <= 1e-14
    for sigma in (0.02, 0.2):
        C = oracle.kernel_C_translated(P.B, P.w, cfg.Q, P.k, sigma)
        assert np.allclose(C, C.T, rtol=0, atol=0)
        # a variance over poses: positive semidefinite
        assert np.linalg.eigvalsh(C).min() >= -1e-12 * np.abs(C).max()
        # a grid rotation of every target leaves it unchanged
        Cr = oracle.kernel_C_translated(np.roll(P.B.numpy(), 5, axis=-1), P.w, cfg.Q, P.k, sigma)
        assert _rel(Cr, C) <= 1e-13


def test_principal_vectors_are_sorted_orthonormal_eigenvectors():
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=1, n_tgt=12, T=1)
    P = synth.make_problem(cfg, seed=10)
    C = oracle.kernel_C(P.B, P.w, cfg.Q)
    U, lam = oracle.principal_vectors(C)
    assert np.all(np.diff(lam) <= 0)
    assert np.allclose(U.T @ U, np.eye(cfg.K), atol=1e-13)
    assert np.allclose(C @ U, U * lam[None, :], atol=1e-12 * np.abs(C).max())


# --------------------------------------------------------------------------
# truncation (P6)
# --------------------------------------------------------------------------
def test_truncation_identity_and_bound():
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=5, n_tgt=6, T=1, H=4)
    P = synth.make_problem(cfg, seed=12)
    A, B = P.A.numpy(), P.B.numpy()
    Q, K, H = cfg.Q, cfg.K, cfg.H
    C = oracle.kernel_C(B, P.w, Q)
    U, lam = oracle.principal_vectors(C)
    e = oracle.eta(P.w, Q)
    bq = np.fft.fft(B * e[None, :, None], axis=-1) / math.sqrt(Q)
    aq = np.fft.fft(A * e[None, :, None], axis=-1) / math.sqrt(Q)
    Pp = np.eye(K) - U[:, :H] @ U[:, :H].T
    pb = np.einsum("rs,bsq->brq", Pp, bq)[:, :, 1:]
    lhs = np.sum(np.abs(pb) ** 2)
    assert abs(lhs - B.shape[0] * lam[H:].sum()) <= 1e-12 * B.shape[0] * np.trace(C)
    XH = oracle.landscape(A, B, U, H, P.k, P.w, P.delta)[:, :, 0]
    XK = oracle.landscape(A, B, U, K, P.k, P.w, P.delta)[:, :, 0]
    dX = XK - XH
    dX = dX - dX.mean(axis=-1, keepdims=True)
    na = np.sqrt(np.sum(np.abs(aq[:, :, 1:]) ** 2, axis=(1, 2)))
    nb = np.sqrt(np.sum(np.abs(pb) ** 2, axis=(1, 2)))
    bound = na[:, None] * nb[None, :]
    assert np.all(np.abs(dX).max(axis=-1) <= bound * (1 + 1e-12))


# --------------------------------------------------------------------------
# decisions
# --------------------------------------------------------------------------
def test_best_tie_rule_and_nan():
    X = np.zeros((1, 3, 2, 4))
    X[0, 0, 1, 2] = 5.0
    X[0, 0, 0, 3] = 5.0            # tie: smaller t*Q+m wins -> (t=0, m=3)
    X[0, 1, 1, 0] = -1.0
    X[0, 1] -= 2.0
    X[0, 1, 1, 0] = 1.0
    X[0, 2, 0, 1] = np.nan
    s, m, t = oracle.best(X)
    assert (s[0, 0], m[0, 0], t[0, 0]) == (5.0, 3, 0)
    assert (s[0, 1], m[0, 1], t[0, 1]) == (1.0, 0, 1)
    assert np.isnan(s[0, 2]) and m[0, 2] == -1 and t[0, 2] == -1


def test_best_and_lse_treat_infinities_as_nan():
    X = np.zeros((2, 3, 2, 4))
    X[0, 0, 1, 2] = np.inf         # would otherwise win outright
    X[0, 1, 0, 0] = -np.inf        # would otherwise never win
    X[1, 2, 1, 3] = 7.0
    s, m, t = oracle.best(X)
    for b in (0, 1):
        assert np.isnan(s[0, b]) and m[0, b] == -1 and t[0, b] == -1
    assert (s[0, 2], m[0, 2], t[0, 2]) == (0.0, 0, 0)     # all zero: first index
    assert (s[1, 2], m[1, 2], t[1, 2]) == (7.0, 3, 1)
    lp, li = oracle.lse(X, 0.5)
    assert np.isnan(lp[0, :2]).all() and np.isfinite(lp[0, 2]) and np.isnan(li[0])
    assert np.isclose(lp[0, 2], np.log(8.0), rtol=1e-15)
    assert np.isfinite(lp[1]).all() and np.isfinite(li[1])


def test_lse_matches_scipy():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3, 4, 2, 8)) * 10
    lp, li = oracle.lse(X, 0.7)
    ref_lp = scipy.special.logsumexp(0.7 * X.reshape(3, 4, -1), axis=-1)
    assert np.allclose(lp, ref_lp, rtol=1e-14, atol=0)
    assert np.allclose(li, scipy.special.logsumexp(ref_lp, axis=-1), rtol=1e-14, atol=0)


# --------------------------------------------------------------------------
# gradient vs FP64 central differences (P7)
# --------------------------------------------------------------------------
def test_lse_gradient_matches_central_differences():
    cfg = synth.config("diff_fd", n_img=4, n_tgt=3, T=9, H=5)
    P = synth.make_problem(cfg, seed=13)
    A, B = P.A.numpy(), P.B.numpy()
    U, _ = oracle.principal_vectors(oracle.kernel_C(B, P.w, cfg.Q))
    s = 1.0 / np.abs(oracle.landscape(A, B, U, cfg.H, P.k, P.w, P.delta)).max() * 3.0
    g = np.array([1.0, -0.5, 2.0, 0.25])
    gB, gU = oracle.lse_grad(A, B, U, cfg.H, P.k, P.w, P.delta, s, g)
    f = lambda BB, UU: oracle.lse_loss(A, BB, UU, cfg.H, P.k, P.w, P.delta, s, g)
    rng = np.random.default_rng(0)
    scaleB = np.abs(B).max()
    for _ in range(6):
        b, r, j = rng.integers(3), rng.integers(cfg.K), rng.integers(cfg.Q)
        for unit, comp in ((1.0, gB[b, r, j].real), (1j, gB[b, r, j].imag)):
            # step sized so that rounding of L (about 1e-16 |L| / h) and the
            # O(h^2) truncation both stay near 1e-10 of max|g|
            hstep = 1e-3 * scaleB
            Bp, Bm = B.copy(), B.copy()
            Bp[b, r, j] += unit * hstep
            Bm[b, r, j] -= unit * hstep
            fd = (f(Bp, U) - f(Bm, U)) / (2 * hstep)
            assert abs(fd - comp) <= 1e-8 * np.abs(gB).max()
    for _ in range(6):
        r, h = rng.integers(cfg.K), rng.integers(cfg.H)
        Up, Um = U.copy(), U.copy()
        Up[r, h] += 1e-4
        Um[r, h] -= 1e-4
        fd = (f(B, Up) - f(B, Um)) / 2e-4
        assert abs(fd - gU[r, h]) <= 1e-8 * np.abs(gU).max()


# --------------------------------------------------------------------------
# rotations off the grid (section 2.2)
# --------------------------------------------------------------------------
def test_offgrid_landscape_on_the_grid_is_the_landscape():
    cfg = synth.config("fp32", N=32, K=16, Q=48, n_img=2, n_tgt=3, T=4, H=6)
    P = synth.make_problem(cfg, seed=21)
    U, _ = oracle.principal_vectors(oracle.kernel_C(P.B, P.w, cfg.Q))
    Ar = oracle.principal_rings(P.A, U, cfg.H, P.w, cfg.Q)
    Br = oracle.principal_rings(P.B, U, cfg.H, P.w, cfg.Q, k=P.k, delta=P.delta)
    X = oracle.landscape_rings(Ar, Br)
    g = 2 * math.pi * np.arange(cfg.Q) / cfg.Q
    for a, b, t in [(0, 0, 0), (1, 2, 3), (0, 1, 2)]:
        Xo = oracle.landscape_offgrid(Ar[a], Br[b, t], g)
        assert _rel(Xo, X[a, b, t]) <= 1e-13


def test_offgrid_landscape_peaks_at_the_true_rotation():
    """A target ring that is the image ring rotated by gamma0 (exactly, as a
    band-limited trigonometric polynomial): rotating it back, X(-gamma0) =
    sum |Ar|^2, the Cauchy-Schwarz maximum, and X is smaller at every other
    angle tried."""
    rng = np.random.default_rng(4)
    Q, H = 32, 5
    psi = 2 * math.pi * np.arange(Q) / Q
    # rings with |q| < Q/2 and no Nyquist term
    qs = np.r_[np.arange(0, Q // 2), np.arange(-Q // 2 + 1, 0)]
    coef = rng.standard_normal((H, Q - 1)) + 1j * rng.standard_normal((H, Q - 1))
    ring = lambda g: (coef[:, :, None] * np.exp(1j * qs[None, :, None] * (psi[None, None, :] - g))).sum(1)
    g0 = 2 * math.pi * 7.37 / Q
    Ar, Br = ring(0.0), ring(g0)
    assert _rel(oracle.rotate_ring(Ar, g0), Br) <= 1e-13
    gs = -g0 + np.linspace(-0.3, 0.3, 61)
    X = oracle.landscape_offgrid(Ar, Br, gs)
    peak = np.sum(np.abs(Ar) ** 2)
    assert abs(X[30] - peak) <= 1e-12 * peak
    assert np.all(X.real[np.arange(61) != 30] < peak * (1 - 1e-6))


def test_offgrid_landscape_shift_and_reality():
    """Rotating the target by a grid angle shifts the off-grid landscape by
    that angle; Hermitian rings give a real landscape at every angle."""
    cfg = synth.config("fp32", N=32, K=16, Q=64, n_img=1, n_tgt=1, T=1, H=8)
    P = synth.make_problem(cfg, seed=22)
    U, _ = oracle.principal_vectors(oracle.kernel_C(P.B, P.w, cfg.Q))
    Ar = oracle.principal_rings(P.A, U, cfg.H, P.w, cfg.Q)[0]
    Br = oracle.principal_rings(P.B, U, cfg.H, P.w, cfg.Q)[0]
    gs = np.array([0.013, 0.9, 2.71, 5.5])
    X = oracle.landscape_offgrid(Ar, Br, gs)
    Xs = oracle.landscape_offgrid(Ar, np.roll(Br, 3, axis=-1), gs - 2 * math.pi * 3 / cfg.Q)
    assert _rel(Xs, X) <= 1e-12
    assert np.abs(X.imag).max() <= 1e-12 * np.abs(X).max()
    # real rings with a strong q = Q/2 term: the band-limited rotation keeps them
    # real (the Nyquist term enters as a cosine), so X is real at any angle
    rng = np.random.default_rng(23)
    Ar = rng.standard_normal((3, 16))
    Br = rng.standard_normal((3, 16)) + 5.0 * (-1.0) ** np.arange(16)[None, :]
    Xr = oracle.landscape_offgrid(Ar, Br, np.array([0.05, 0.77, 3.3]))
    assert np.abs(Xr.imag).max() <= 1e-12 * np.abs(Xr).max()
    assert np.abs(oracle.rotate_ring(Br, 0.4).imag).max() <= 1e-12 * np.abs(Br).max()


# --------------------------------------------------------------------------
# landscape quality measures (section 3.5) and marching candidates (section 5)
# --------------------------------------------------------------------------
def test_landscape_metrics_against_library_routines():
    import scipy.stats
    rng = np.random.default_rng(31)
    R = rng.standard_normal((7, 4, 32))
    E = R + 0.3 * rng.standard_normal(R.shape)
    rel, corr, f = oracle.landscape_metrics(E, R)
    assert abs(rel - np.linalg.norm(E - R) / np.linalg.norm(R)) <= 1e-14
    assert abs(corr - np.corrcoef(E.ravel(), R.ravel())[0, 1]) <= 1e-13
    for p in range(7):
        i = np.argmax(E[p].ravel())
        want = scipy.stats.percentileofscore(R[p].ravel(), R[p].ravel()[i], kind="weak") / 100.0
        assert abs(f[p] - want) <= 1e-15
    # exact landscapes: no error, correlation 1, every optimum at the top
    rel, corr, f = oracle.landscape_metrics(R, R)
    assert rel == 0.0 and abs(corr - 1.0) <= 1e-14 and np.all(f == 1.0)
    # an affine image of the truth: correlated perfectly, same optima
    rel, corr, f = oracle.landscape_metrics(2.5 * R - 1.0, R)
    assert abs(corr - 1.0) <= 1e-14 and np.all(f == 1.0) and rel > 1.0
    # a reversed landscape picks the worst alignment: f = 1 / len
    rel, corr, f = oracle.landscape_metrics(-R, R)
    assert abs(corr + 1.0) <= 1e-14 and np.allclose(f, 1.0 / 128)
    E[3, 1, 5] = np.nan
    assert np.isnan(oracle.landscape_metrics(E, R)[2][3])


def test_top_targets_order_ties_and_nan():
    S = np.array([[0.5, 2.0, 2.0, np.nan, -1.0],
                  [np.nan, np.nan, 1.0, np.nan, np.nan]])
    c = oracle.top_targets(S, 4)
    assert c.tolist() == [[1, 2, 0, 4], [2, -1, -1, -1]]
    rng = np.random.default_rng(2)
    S = rng.standard_normal((5, 40))
    c = oracle.top_targets(S, 7)
    assert np.array_equal(c, np.argsort(-S, axis=1, kind="stable")[:, :7])
