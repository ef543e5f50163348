"""Pins of the volume oracle (paper section 4) to what the mathematics fixes,
not to itself.

* The closed-form shell coefficients of blob volumes (the input generator)
  against a sphere quadrature of the plane-wave sum.
* Wigner-d: textbook values (d^l(0) = I, d^l_00 = P_l(cos beta), the l = 1
  matrix, d^l(pi)), orthogonality and composition; the rotation formula of
  section 4.2 against a physical rotation of the blob centres.
* The radial kernel C and the diagonal of the degree kernel D against the
  SO(3) average of their defining objectives (sections 4.6, 4.8), evaluated by
  rotating the blob centres over an SO(3) quadrature; the degree kernel's
  invariance under rotations about the z axis.
* The landscape of section 4.4 against the physical inner product
  <A, R_tau B> (sphere quadrature with rotated centres, no harmonics, no
  Wigner-d, no transform); the compressed steps of section 4.9 at full rank
  against section 4.4; recovery of a grid rotation; the argmax rules.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import volume as ov
from synth import volumes as sv


def _sphere_grid(nth, nph):
    x, wx = np.polynomial.legendre.leggauss(nth)
    th = np.arccos(x)
    ph = 2 * math.pi * np.arange(nph) / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(wx, np.full(nph, 2 * math.pi / nph))
    om = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    return TH, PH, W, om


def _plane_waves(mu, s, c, k, om):
    """F(k omega) of one blob volume on the sphere grid omega."""
    out = np.zeros(om.shape[:-1], dtype=np.complex128)
    for m, si, ci in zip(mu, s, c):
        out += ci * (2 * math.pi * si * si) ** 1.5 * math.exp(-0.5 * (si * k) ** 2) * np.exp(-1j * k * (om @ m))
    return out


def test_shell_coefficients_match_sphere_quadrature():
    rng = np.random.default_rng(11)
    mu, s, c = sv.blob_params_3d(rng, 2, 5, 0.5)
    k = np.array([0.7, 2.3, 4.1])
    L = 8
    A = sv.sh_coeffs(mu, s, c, k, L)
    TH, PH, W, om = _sphere_grid(48, 96)
    worst = 0.0
    for v in range(2):
        for r in range(len(k)):
            F = _plane_waves(mu[v], s[v], c[v], k[r], om)
            for l in range(L + 1):
                for m in range(-l, l + 1):
                    num = np.sum(W * F * np.conj(sp.sph_harm_y(l, m, TH, PH)))
                    worst = max(worst, abs(num - A[v, r, ov.sh_index(l, m)]))
    assert worst <= 1e-12 * np.abs(A).max(), worst
    # a real volume's coefficients: conj(F_l^m) = (-1)^(l+m) F_l^-m
    for l in range(L + 1):
        for m in range(-l, l + 1):
            assert np.allclose(np.conj(A[..., ov.sh_index(l, m)]), (-1) ** (l + m) * A[..., ov.sh_index(l, -m)],
                               rtol=0, atol=1e-14 * np.abs(A).max())


def test_wigner_d_textbook_values():
    for l in range(0, 9):
        assert np.allclose(ov.wigner_d(l, 0.0), np.eye(2 * l + 1), atol=1e-13)
    for beta in (0.3, 1.9, -2.6):
        x = math.cos(beta)
        for l in range(0, 13):
            assert abs(ov.wigner_d(l, beta)[l, l] - sp.eval_legendre(l, x)) < 1e-12
        s2 = math.sin(beta) / math.sqrt(2)
        d1 = np.array([[(1 + x) / 2, s2, (1 - x) / 2],            # rows m1 = -1, 0, 1
                       [-s2, x, s2],
                       [(1 - x) / 2, -s2, (1 + x) / 2]])
        assert np.allclose(ov.wigner_d(1, beta), d1, atol=1e-14)
    # d^l_{m1 m2}(pi) = (-1)^(l - m2) delta_{m1, -m2}
    for l in range(0, 7):
        ms = np.arange(-l, l + 1)
        want = np.zeros((2 * l + 1, 2 * l + 1))
        for i, m2 in enumerate(ms):
            want[l - m2, i] = (-1) ** (l - m2)
        assert np.allclose(ov.wigner_d(l, math.pi), want, atol=1e-12)
    # orthogonal, and a one-parameter group in beta
    for l in (3, 10, 24):
        a, b = 0.7, 1.3
        d = ov.wigner_d(l, a)
        assert np.allclose(d @ d.T, np.eye(2 * l + 1), atol=1e-12)
        assert np.allclose(d @ ov.wigner_d(l, b), ov.wigner_d(l, a + b), atol=1e-12)


def test_rotation_formula_matches_rotated_blobs():
    rng = np.random.default_rng(12)
    mu, s, c = sv.blob_params_3d(rng, 1, 6, 0.5)
    k = np.array([1.1, 3.4])
    L = 10
    A = sv.sh_coeffs(mu, s, c, k, L)[0]
    for (al, be, ga) in [(0.7, 1.1, -0.4), (2.9, 2.2, 1.3), (-1.0, 0.2, 3.0)]:
        R = sv.rotation_matrix(al, be, ga)
        B_phys = sv.sh_coeffs((R @ mu[0].T).T[None], s, c, k, L)[0]
        B_form = ov.rotate_coeffs(A, L, al, be, ga)
        assert np.abs(B_form - B_phys).max() <= 1e-13 * np.abs(B_phys).max()


def _so3_rotations(L):
    """A product quadrature on SO(3) (alpha, gamma uniform; cos beta
    Gauss-Legendre) that integrates every Wigner D^l entry, l <= L, exactly
    (probability measure)."""
    na = 2 * L + 2
    x, wx = np.polynomial.legendre.leggauss(L + 2)
    out = []
    for ia in range(na):
        for ib, xb in enumerate(x):
            for ig in range(na):
                R = sv.rotation_matrix(2 * math.pi * ia / na, math.acos(xb), 2 * math.pi * ig / na)
                out.append((R, wx[ib] / 2 / na / na))
    return out


def _rotated_coeffs(mu, s, c, k, L, rots):
    return np.stack([sv.sh_coeffs((R @ mu[0].T).T[None], s, c, k, L)[0] for R, _ in rots])


def test_radial_kernel_is_the_so3_average_of_its_objective():
    rng = np.random.default_rng(13)
    L, K = 4, 4
    mu, s, c = sv.blob_params_3d(rng, 1, 5, 0.5)
    k, w = sv.shell_grid(4.0, K)
    rots = _so3_rotations(L)
    F = _rotated_coeffs(mu, s, c, k, L, rots)            # [tau][K][lm]
    wt = np.array([x for _, x in rots])
    eta = np.sqrt(w)
    Cdef = np.zeros((K, K), dtype=np.complex128)
    for i in range(len(rots)):                            # the double integral, literally
        D = F[i][None] - F                                # [tau'][K][lm]
        Cdef += wt[i] * np.einsum("t,tri,tsi->rs", wt, D.conj(), D)
    Cdef *= eta[:, None] * eta[None, :]
    C = ov.vol_kernel_C(sv.sh_coeffs(mu, s, c, k, L), w, L)
    assert np.abs(Cdef.imag).max() <= 1e-13 * np.abs(Cdef).max()
    assert np.allclose(Cdef.real, 2 * C, rtol=0, atol=1e-12 * np.abs(C).max())
    # target averaging: two targets give the mean of their kernels
    mu2, s2, c2 = sv.blob_params_3d(rng, 2, 5, 0.5)
    B2 = sv.sh_coeffs(mu2, s2, c2, k, L)
    assert np.allclose(ov.vol_kernel_C(B2, w, L),
                       0.5 * (ov.vol_kernel_C(B2[:1], w, L) + ov.vol_kernel_C(B2[1:], w, L)), atol=1e-14)


def test_degree_kernel_diagonal_is_the_so3_average_and_z_invariant():
    rng = np.random.default_rng(14)
    L, K = 4, 3
    mu, s, c = sv.blob_params_3d(rng, 1, 5, 0.5)
    k, w = sv.shell_grid(4.0, K)
    B = sv.sh_coeffs(mu, s, c, k, L)
    D = ov.vol_kernel_D(B, w, L)
    assert np.all(D[0] == 0) and np.all(D[:, 0] == 0)
    rots = _so3_rotations(L)
    F = _rotated_coeffs(mu, s, c, k, L, rots)
    wt = np.array([x for _, x in rots])
    for l in range(L + 1):       # the objective at v = e_l, as a double integral
        sl = slice(l * l, (l + 1) * (l + 1))
        acc = 0.0
        for i in range(len(rots)):
            diff = F[i][None, :, sl] - F[:, :, sl]
            acc += wt[i] * np.einsum("t,r,tri->", wt, w, np.abs(diff) ** 2)
        assert abs(acc - 2 * D[l, l]) <= 1e-12 * np.abs(D).max(), (l, acc, D[l, l])
    # rotations about z keep every entry (the same order m of both degrees
    # takes the same phase)
    for al in (0.4, 2.5):
        Rz = sv.rotation_matrix(al, 0.0, 0.0)
        Bz = sv.sh_coeffs((Rz @ mu[0].T).T[None], s, c, k, L)
        assert np.allclose(ov.vol_kernel_D(Bz, w, L), D, rtol=0, atol=1e-12 * np.abs(D).max())
    # ... rotations about y do not (the off-diagonal entries are not averaged)
    Ry = sv.rotation_matrix(0.0, 1.0, 0.0)
    By = sv.sh_coeffs((Ry @ mu[0].T).T[None], s, c, k, L)
    Dy = ov.vol_kernel_D(By, w, L)
    assert np.allclose(np.diag(Dy), np.diag(D), rtol=0, atol=1e-12 * np.abs(D).max())
    assert np.abs(Dy - D).max() > 1e-6 * np.abs(D).max()


def test_landscape_matches_physical_inner_product():
    rng = np.random.default_rng(15)
    L, K = 16, 5
    mu, s, c = sv.blob_params_3d(rng, 2, 4, 0.4)
    k, w = sv.shell_grid(3.0, K)
    A = sv.sh_coeffs(mu[:1], s[:1], c[:1], k, L)[0]
    B = sv.sh_coeffs(mu[1:], s[1:], c[1:], k, L)[0]
    M = 2 * L + 1
    betas = [0.5, 2.0, 2 * math.pi * 30 / M]
    X = ov.landscape_direct(A, B, w, L, betas)
    TH, PH, W, om = _sphere_grid(40, 80)
    worst = 0.0
    for ib, beta in enumerate(betas):
        for (m1, m2) in [(0, 0), (3, 17), (30, 5), (12, 12)]:
            R = sv.rotation_matrix(2 * math.pi * m1 / M, beta, 2 * math.pi * m2 / M)
            acc = 0.0
            for r in range(K):
                FA = _plane_waves(mu[0], s[0], c[0], k[r], om)
                FB = _plane_waves((R @ mu[1].T).T, s[1], c[1], k[r], om)
                acc += w[r] * np.sum(W * np.conj(FA) * FB)
            worst = max(worst, abs(acc - X[ib, m1, m2]))
    assert worst <= 1e-11 * np.abs(X).max(), worst
    # real volumes give a real landscape
    assert np.abs(X.imag).max() <= 1e-13 * np.abs(X).max()


def _random_orthogonal(rng, n):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q


def test_compressed_steps_at_full_rank_equal_the_direct_sum():
    rng = np.random.default_rng(16)
    L, K = 6, 5
    mu, s, c = sv.blob_params_3d(rng, 3, 5, 0.5)
    k, w = sv.shell_grid(5.0, K)
    V3 = sv.sh_coeffs(mu, s, c, k, L)
    betas = sv.beta_grid(7)
    for U, V in [(np.linalg.eigh(ov.vol_kernel_C(V3[2:], w, L))[1], np.linalg.eigh(ov.vol_kernel_D(V3[2:], w, L))[1]),
                 (_random_orthogonal(rng, K), _random_orthogonal(rng, L + 1))]:
        X = ov.landscape_all(V3[:2], V3[2:], w, U, K, V, L + 1, L, betas)
        for a in range(2):
            Xd = ov.landscape_direct(V3[a], V3[2], w, L, betas)
            assert np.abs(X[a, 0] - Xd).max() <= 1e-12 * np.abs(Xd).max()
    # dropping a rank changes the landscape (the steps do use H)
    U = np.linalg.eigh(ov.vol_kernel_C(V3[2:], w, L))[1][:, ::-1]
    V = np.linalg.eigh(ov.vol_kernel_D(V3[2:], w, L))[1][:, ::-1]
    X1 = ov.landscape_all(V3[:1], V3[2:], w, U, K - 2, V, L - 1, L, betas)
    Xd = ov.landscape_direct(V3[0], V3[2], w, L, betas)
    assert np.abs(X1[0, 0] - Xd).max() > 1e-6 * np.abs(Xd).max()


def test_landscape_recovers_a_grid_rotation():
    rng = np.random.default_rng(17)
    L, K = 8, 6
    M = 2 * L + 1
    mu, s, c = sv.blob_params_3d(rng, 1, 8, 0.5)
    k, w = sv.shell_grid(6.0, K)
    A = sv.sh_coeffs(mu, s, c, k, L)[0]
    p, q, t = 5, 4, 11          # alpha0, beta0, gamma0 on the grid 2 pi j / M
    R0 = sv.rotation_matrix(2 * math.pi * p / M, 2 * math.pi * q / M, 2 * math.pi * t / M)
    B = sv.sh_coeffs((R0 @ mu[0].T).T[None], s, c, k, L)[0]
    X = ov.landscape_direct(A, B, w, L, sv.beta_grid(M))
    score, idx = ov.best(X[None])
    # the inverse rotation: (gamma, beta, alpha) = (-alpha0, -beta0, -gamma0)
    assert tuple(idx[0]) == ((M - q) % M, (M - t) % M, (M - p) % M)
    assert abs(score[0] - np.einsum("r,ri->", w, np.abs(A) ** 2)) <= 1e-12 * score[0]


def test_best_rules():
    X = np.zeros((2, 3, 5, 5), dtype=np.complex128)
    X[0, 1, 2, 3] = 2.0
    X[0, 2, 0, 0] = 2.0          # a tie: the smaller flattened index wins
    X[1, 0, 0, 1] = np.nan
    score, idx = ov.best(X)
    assert score[0] == 2.0 and tuple(idx[0]) == (1, 2, 3)
    assert np.isnan(score[1]) and tuple(idx[1]) == (-1, -1, -1)
