"""FP64 CPU oracle for rotational volume alignment with principal volumes
(paper section 4).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it; it shares no code with the HIP library.

Inputs are spherical-harmonic coefficients on K shells, complex [n][K][(L+1)^2],
l-major (index l^2 + l + m), orthonormal harmonics with the Condon-Shortley
phase; w_r weights the shells for k^2 dk.

* ``wigner_d``        -- d^l(beta) = exp(-i beta J_y) in the basis |l m>,
                         m = -l..l (section 4.2: the matrix that carries a
                         rotation's interior angle); computed from the
                         eigen-decomposition of J_y.
* ``rotate_coeffs``   -- the rotated volume's coefficients (section 4.2):
                         B_l^{m1} = sum_m2 e^{-i m1 alpha} d^l_{m1 m2}(beta) e^{-i m2 gamma} A_l^{m2}.
* ``vol_kernel_C``    -- the radial kernel of section 4.6 averaged over the
                         targets: C_rr' = eta_r eta_r' Re sum_{l>=1,m} conj(B_l^m(k_r)) B_l^m(k_r'),
                         eta_r = sqrt(w_r).
* ``vol_kernel_D``    -- the degree kernel of section 4.8 averaged over the
                         targets: D_ll' = Re sum_r w_r sum_m conj(B_l^m(k_r)) B_l'^m(k_r)
                         for l, l' >= 1, zero in row and column l = 0.
* ``principal_shells`` -- [u_h^T A]_l^m = sum_r U[r,h] eta_r A_l^m(k_r) (section 4.5).
* ``landscape_direct`` -- the three steps of section 4.4 over all shells and
                         degrees: X[b-angle][m1'][m2'] for tau = (gamma_m2', beta, alpha_m1'),
                         alpha, gamma on the grid 2 pi m / M, M = 2L + 1.
* ``landscape``       -- the steps 1, 1b, 2 and 3 of section 4.9 with H_C
                         principal shells and H_D principal degrees.
* ``best``            -- argmax over (beta index, m1', m2') of Re X.
"""
from __future__ import annotations

import numpy as np


def sh_index(l: int, m: int) -> int:
    return l * l + l + m


def n_orders(L: int) -> int:
    return 2 * L + 1


def wigner_d(l: int, beta: float) -> np.ndarray:
    """Real (2l+1) x (2l+1) matrix d^l_{m1 m2}(beta) = <l m1| exp(-i beta J_y) |l m2>,
    rows and columns m = -l..l.  J_y = (J_+ - J_-)/(2i) with
    J_+ |l m> = sqrt(l(l+1) - m(m+1)) |l m+1>; exp by diagonalising the
    Hermitian J_y (eigenvalues -l..l)."""
    n = 2 * l + 1
    ms = np.arange(-l, l + 1)
    Jp = np.zeros((n, n), dtype=np.complex128)
    for i in range(n - 1):
        Jp[i + 1, i] = np.sqrt(l * (l + 1) - ms[i] * (ms[i] + 1))
    Jy = (Jp - Jp.conj().T) / 2j
    ev, W = np.linalg.eigh(Jy)
    ev = np.round(ev)   # exactly the integers -l..l
    D = (W * np.exp(-1j * beta * ev)[None, :]) @ W.conj().T
    return D.real


def rotate_coeffs(A, L: int, alpha: float, beta: float, gamma: float) -> np.ndarray:
    """Coefficients of R_tau A for tau = (gamma, beta, alpha); A [..][(L+1)^2]."""
    A = np.asarray(A, dtype=np.complex128)
    out = np.zeros_like(A)
    for l in range(L + 1):
        ms = np.arange(-l, l + 1)
        D = np.exp(-1j * ms[:, None] * alpha) * wigner_d(l, beta) * np.exp(-1j * ms[None, :] * gamma)
        sl = slice(l * l, (l + 1) * (l + 1))
        out[..., sl] = A[..., sl] @ D.T
    return out


def vol_kernel_C(B, w, L: int) -> np.ndarray:
    """K x K radial kernel, l = 0 excluded, averaged over the targets."""
    B = np.asarray(B, dtype=np.complex128)
    eta = np.sqrt(np.asarray(w, dtype=np.float64))
    n_tgt, K, _ = B.shape
    C = np.zeros((K, K))
    for b in range(n_tgt):
        X = B[b][:, 1:]                       # every l >= 1, all m
        C += (X.conj() @ X.T).real
    C /= n_tgt
    C *= eta[:, None] * eta[None, :]
    return 0.5 * (C + C.T)


def vol_kernel_D(B, w, L: int) -> np.ndarray:
    """(L+1) x (L+1) degree kernel; row and column l = 0 are zero."""
    B = np.asarray(B, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    n_tgt = B.shape[0]
    D = np.zeros((L + 1, L + 1))
    for l in range(1, L + 1):
        for lp in range(1, L + 1):
            mm = min(l, lp)
            acc = 0.0
            for m in range(-mm, mm + 1):
                x = B[:, :, sh_index(l, m)]
                y = B[:, :, sh_index(lp, m)]
                acc += np.sum(w[None, :] * (x.conj() * y)).real
            D[l, lp] = acc / n_tgt
    return 0.5 * (D + D.T)


def principal_shells(X, U, H: int, w) -> np.ndarray:
    """[n][H][(L+1)^2]: sum_r U[r, h] eta_r X[n][r][lm]."""
    X = np.asarray(X, dtype=np.complex128)
    eta = np.sqrt(np.asarray(w, dtype=np.float64))
    UH = np.asarray(U, dtype=np.float64)[:, :H] * eta[:, None]
    return np.einsum("rh,nri->nhi", UH, X)


def _embed(M: int, l: int, block: np.ndarray, out: np.ndarray):
    """Add an order block (m1, m2 in -l..l) into a periodic M x M array."""
    idx = np.arange(-l, l + 1) % M
    out[np.ix_(idx, idx)] += block


def _step3(Xhat) -> np.ndarray:
    """X(alpha_m1', gamma_m2') = sum_{m1,m2} e^{-2 pi i m1 m1'/M} e^{-2 pi i m2 m2'/M} Xhat[m1][m2]
    (orders stored at index m mod M): the forward 2-D DFT."""
    return np.fft.fft2(Xhat, axes=(-2, -1))


def landscape_direct(A, B, w, L: int, betas) -> np.ndarray:
    """X[ib][m1'][m2'] for one pair, every shell and degree (section 4.4):
    step 1 Xt_l(m1, m2) = sum_r w_r conj(A_l^m1(k_r)) B_l^m2(k_r);
    step 2 Xhat(m1, m2; beta) = sum_l d^l_{m1 m2}(beta) Xt_l(m1, m2);
    step 3 the 2-D transform over the orders."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    M = n_orders(L)
    Xt = []
    for l in range(L + 1):
        sl = slice(l * l, (l + 1) * (l + 1))
        Xt.append(np.einsum("r,ri,rj->ij", w, A[:, sl].conj(), B[:, sl]))
    out = np.empty((len(betas), M, M), dtype=np.complex128)
    for ib, beta in enumerate(betas):
        Xhat = np.zeros((M, M), dtype=np.complex128)
        for l in range(L + 1):
            _embed(M, l, wigner_d(l, beta) * Xt[l], Xhat)
        out[ib] = _step3(Xhat)
    return out


def principal_degree_wigner(V, HD: int, L: int, beta: float) -> np.ndarray:
    """[v_j^T d](beta) on the periodic M x M order grid, j < HD: [HD][M][M]."""
    M = n_orders(L)
    out = np.zeros((HD, M, M))
    for l in range(L + 1):
        d = wigner_d(l, beta)
        for j in range(HD):
            _embed(M, l, V[l, j] * d, out[j])
    return out


def landscape(As, Bs, V, HD: int, L: int, betas, vd=None) -> np.ndarray:
    """X[ib][m1'][m2'] for one pair from principal shells As, Bs [H_C][(L+1)^2]
    (section 4.9):
    step 1  Xt_l(m1, m2) = sum_h conj(As[h]_l^m1) Bs[h]_l^m2;
    step 1b Y_j(m1, m2)  = sum_l V[l, j] Xt_l(m1, m2), j < HD;
    step 2  Xhat(m1, m2; beta) = sum_j [v_j^T d]_{m1 m2}(beta) Y_j(m1, m2);
    step 3  the 2-D transform over the orders.
    ``vd`` may hold principal_degree_wigner for each beta (reused across pairs)."""
    As = np.asarray(As, dtype=np.complex128)
    Bs = np.asarray(Bs, dtype=np.complex128)
    V = np.asarray(V, dtype=np.float64)
    M = n_orders(L)
    Y = np.zeros((HD, M, M), dtype=np.complex128)
    for l in range(L + 1):
        sl = slice(l * l, (l + 1) * (l + 1))
        Xt = As[:, sl].conj().T @ Bs[:, sl]          # step 1: (2l+1) x (2l+1)
        for j in range(HD):                           # step 1b
            _embed(M, l, V[l, j] * Xt, Y[j])
    out = np.empty((len(betas), M, M), dtype=np.complex128)
    for ib, beta in enumerate(betas):
        t = vd[ib] if vd is not None else principal_degree_wigner(V, HD, L, beta)
        Xhat = np.einsum("jab,jab->ab", t, Y)        # step 2
        out[ib] = _step3(Xhat)                        # step 3
    return out


def landscape_all(A, B, w, U, HC: int, V, HD: int, L: int, betas, pairs=None) -> np.ndarray:
    """X[a][b][ib][m1'][m2'] (or [pair][...] for a list of (a, b) pairs)."""
    As = principal_shells(A, U, HC, w)
    Bs = principal_shells(B, U, HC, w)
    vd = [principal_degree_wigner(V, HD, L, b) for b in betas]
    if pairs is None:
        out = np.empty((As.shape[0], Bs.shape[0], len(betas), n_orders(L), n_orders(L)), dtype=np.complex128)
        for a in range(As.shape[0]):
            for b in range(Bs.shape[0]):
                out[a, b] = landscape(As[a], Bs[b], V, HD, L, betas, vd)
        return out
    return np.stack([landscape(As[a], Bs[b], V, HD, L, betas, vd) for a, b in pairs])


def best(X):
    """Per pair: (score, ib, m1', m2') of max Re X over the flattened
    (ib, m1', m2') index, smallest index on ties; NaN anywhere gives
    (NaN, -1, -1, -1).  X [..][n_beta][M][M]."""
    X = np.asarray(X)
    lead = X.shape[:-3]
    nb, M = X.shape[-3], X.shape[-1]
    R = X.real.reshape(-1, nb * M * M)
    score = np.full(R.shape[0], np.nan)
    idx = np.full((R.shape[0], 3), -1, dtype=np.int64)
    for p in range(R.shape[0]):
        if np.isnan(R[p]).any():
            continue
        i = int(np.argmax(R[p]))
        score[p] = R[p, i]
        idx[p] = (i // (M * M), (i // M) % M, i % M)
    return score.reshape(lead), idx.reshape(lead + (3,))
