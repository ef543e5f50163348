"""FP64 CPU oracle for radial-SVD rotational image alignment.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (no kernels, headers, tables or helpers) and never
imports it; the library never imports this.

What it computes (A. Rangan, "Radial-recombination for rigid rotational
alignment of images and volumes", arXiv 2202.07235):

* ``kernel_C``         -- the target-averaged kernel C of section 3.4 (eqs.
                          for the single-target kernel and its Plancherel
                          simplification, q = 0 excluded), with the ring
                          weights sqrt(w_r) of the kernel's defining integral;
                          evaluated in psi-space by the 1-D Plancherel
                          identity, no FFT.
* ``kernel_C_translated`` -- the kernel of the translation- and rotation-averaged
                          objective of the discussion (section 5), for an
                          isotropic Gaussian prior on the translations: the
                          closed form with the factors E+ and E- (modified
                          Bessel functions of order -1/2 and +1/2).
* ``principal_vectors`` -- U = eigenvectors of C by descending eigenvalue
                          (section 3.3: the maximisers of the Rayleigh quotient).
* ``principal_rings``  -- [u_h^T Ahat](psi_j) = sum_r U[r,h] eta_r Ahat(k_r, psi_j),
                          eta_r = sqrt(w_r dpsi) (section 3.2), with the
                          translation phase exp(-i k.delta) of the Fourier
                          shift theorem for targets.
* ``landscape``        -- X[a,b,t,m] = sum_h sum_j conj(Ar_h[a](psi_j)) Br_h^t[b](psi_{j-m}),
                          the direct psi-space form of the two-step evaluation
                          (section 2.4 / section 3.3 steps 1-2).  At H = K it
                          is the full polar quadrature of <Ahat, R_gamma T_delta Bhat>
                          (prefactor (2 pi)^-2 dropped, as the paper does).
* ``landscape_offgrid`` -- X at rotations gamma off the polar grid: the target
                          ring rotated by the phase exp(-i q gamma) on its
                          Fourier-Bessel coefficients (section 2.2, rotation by
                          any gamma), band-limited to |q| <= Q/2, then the
                          direct psi-space sum.
* ``landscape_metrics`` -- the quality measures of section 3.5: relative
                          error in the Frobenius norm and correlation over the
                          whole array, and per pair the true percentile f of
                          the approximate alignment.
* ``top_targets``      -- the candidates of principal-mode marching (section 5):
                          the k best-scoring targets of each image.
* ``best`` / ``lse``   -- maximum-likelihood alignment argmax_gamma X (section
                          2.7) and the soft-alignment log-sum-exp score.
* ``lse_grad``         -- gradient of sum_a g_a lse_img[a] with respect to the
                          target polar samples and U (chain rule written as
                          direct psi-space sums).

Every floating-point quantity is FP64.  The direct sums run in plain C
(``direct.c``, OpenMP over pairs).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
CFLAGS = ["-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c99"]
_lib = None


def _host_tag() -> str:
    """Short tag of the host CPU (model and feature flags): -march=native code
    is built per host, so a library built on one machine is never loaded on
    another whose CPU lacks an instruction it uses."""
    import hashlib
    import platform
    info = platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith(("model name", "flags")):
                    info += line
                if line.startswith("flags"):
                    break
    except OSError:
        pass
    return hashlib.sha1(info.encode()).hexdigest()[:10]


_SO = os.path.join(_HERE, "_build", f"liboracle_direct_{_host_tag()}.so")


def build(force: bool = False) -> str:
    """Compile direct.c with gcc (CFLAGS: -O3 -march=native -fopenmp) for this host."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    src = os.path.join(_HERE, "direct.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc"] + CFLAGS + ["-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
        lib.oracle_landscape_pairs.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, dp, dp, dp]
        lib.oracle_grad_tgt_rings.argtypes = [ctypes.c_int] * 5 + [dp, dp, dp]
        lib.oracle_grad_img_rings.argtypes = [ctypes.c_int] * 5 + [dp, dp, dp]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return _load().oracle_num_threads()


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(a) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


# --------------------------------------------------------------------------
# grid-derived factors
# --------------------------------------------------------------------------
def eta(w, Q: int) -> np.ndarray:
    """eta_r = sqrt(w_r dpsi), dpsi = 2 pi / Q (section 2.6, ring rescaling)."""
    return np.sqrt(np.asarray(w, dtype=np.float64) * (2.0 * math.pi / Q))


def phase(k, delta, Q: int) -> np.ndarray:
    """phi_t[r, j] = exp(-i k_r (dx cos psi_j + dy sin psi_j)): the Fourier
    transform of B(x - delta) is exp(-i k.delta) Bhat(k) (section 2.1)."""
    k = np.asarray(k, dtype=np.float64)
    d = np.asarray(delta, dtype=np.float64).reshape(-1, 2)
    psi = 2.0 * math.pi * np.arange(Q) / Q
    arg = k[None, :, None] * (d[:, 0, None, None] * np.cos(psi)[None, None, :]
                              + d[:, 1, None, None] * np.sin(psi)[None, None, :])
    return np.exp(-1j * arg)                           # [T][K][Q]


# --------------------------------------------------------------------------
# kernel C and its principal vectors (sections 3.3 - 3.4)
# --------------------------------------------------------------------------
def kernel_C(B, w, Q: int) -> np.ndarray:
    """C[r,r'] = (1/N_B) sum_b sum_{q != 0} Re conj(bq[b,r,q]) bq[b,r',q] with
    bq the unitary angular DFT of eta_r Bhat[b,r,:].  By the 1-D Plancherel
    identity the q-sum over all q is the psi-sum, and the q = 0 term is the
    squared ring mean, so C needs no FFT:
      C = eta_r eta_r' Re[ sum_j conj(B_r) B_r'  -  (1/Q) conj(sum_j B_r)(sum_j B_r') ] / N_B.
    The paper's constant (2 pi)^3 / (4 sigma_hat^2) is dropped: it scales the
    eigenvalues and leaves the principal vectors unchanged."""
    B = _c128(B)
    nb, K, _ = B.shape
    e = eta(w, Q)
    Bm = B.transpose(1, 0, 2).reshape(K, nb * Q)
    G = np.conj(Bm) @ Bm.T                            # sum_{b,j} conj(B_r) B_r'
    s = B.sum(axis=2)                                 # [nb][K]
    G0 = np.conj(s).T @ s                             # sum_b conj(sum_j B_r)(sum_j B_r')
    C = (G - G0 / Q).real * np.outer(e, e) / nb
    return 0.5 * (C + C.T)


def translation_factors(k, sigma_delta: float):
    """The factors of the translation-averaged kernel (section 5, the closed
    form for an isotropic Gaussian translation prior of standard deviation
    sigma_delta), as the paper writes them:
      E+(k_r, k_r') = exp(-sigma^2 (k_r^2 + k_r'^2) / 2) * exp(k_r k_r' sigma^2),
      E-(k_r)       = kt sqrt(pi/2) exp(-kt^2) (I_{-1/2}(kt^2) - I_{+1/2}(kt^2)),  kt = k_r sigma / 2,
    with I_nu the modified Bessel function of the first kind.  The two
    exponentials of E+ are taken as one (no overflow for large k sigma), and
    exp(-x) I_nu(x) is scipy's exponentially scaled ``ive``.  E-(0) = 1 (the
    limit kt -> 0).  Returns (E+ [K][K], E- [K])."""
    import scipy.special
    k = np.asarray(k, dtype=np.float64)
    s2 = float(sigma_delta) ** 2
    Ep = np.exp(-0.5 * s2 * (k[:, None] ** 2 + k[None, :] ** 2) + s2 * np.outer(k, k))
    kt = k * float(sigma_delta) / 2.0
    x = kt * kt
    Em = np.ones_like(k)
    nz = kt > 0
    Em[nz] = kt[nz] * math.sqrt(math.pi / 2.0) * (scipy.special.ive(-0.5, x[nz]) - scipy.special.ive(0.5, x[nz]))
    return Ep, Em


def kernel_C_translated(B, w, Q: int, k, sigma_delta: float) -> np.ndarray:
    """Target-averaged kernel of the translation- and rotation-averaged
    objective (section 5): for each target, the sum over pairs of poses
    (rotation on the grid, translation from an isotropic Gaussian of standard
    deviation sigma_delta) of sum_j |[u^T T_d R_g B](psi_j) - [u^T T_d' R_g' B](psi_j)|^2
    is quadratic in u.  Its kernel has the closed form of the paper's
    equation for the translated template cost, with the sums over the
    volume's spherical-harmonic coefficients read, for a set of image
    targets, as each target's sums over the angular frequencies q:
      C = eta_r eta_r' Re[ E+(k_r, k_r') sum_q conj(bq_r) bq_r'  -  E-(k_r) E-(k_r') conj(bq0_r) bq0_r' ] / N_B,
    bq the unitary angular DFT of the ring (bq0 its q = 0 term).  By the 1-D
    Plancherel identity the q-sum is the psi-sum and bq0 = (ring sum) / sqrt(Q),
    as in kernel_C.  sigma_delta = 0 gives kernel_C (E+ = E- = 1)."""
    B = _c128(B)
    nb, K, _ = B.shape
    e = eta(w, Q)
    Ep, Em = translation_factors(k, sigma_delta)
    Bm = B.transpose(1, 0, 2).reshape(K, nb * Q)
    G = np.conj(Bm) @ Bm.T                            # sum_{b,j} conj(B_r) B_r'
    s = B.sum(axis=2)                                 # [nb][K]
    G0 = np.conj(s).T @ s                             # sum_b conj(sum_j B_r)(sum_j B_r')
    C = (Ep * G - np.outer(Em, Em) * G0 / Q).real * np.outer(e, e) / nb
    return 0.5 * (C + C.T)


def principal_vectors(C):
    """Eigenvectors of the symmetric kernel by descending eigenvalue
    (Rayleigh-quotient maximisers, section 3.3).  Each column's sign is fixed
    so that its entry of largest magnitude is positive."""
    lam, V = np.linalg.eigh(np.asarray(C, dtype=np.float64))
    order = np.argsort(-lam, kind="stable")
    lam, V = lam[order], V[:, order]
    piv = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[piv, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return V * sgn[None, :], lam


# --------------------------------------------------------------------------
# principal rings and the landscape
# --------------------------------------------------------------------------
def principal_rings(X, U, H: int, w, Q: int, k=None, delta=None) -> np.ndarray:
    """[u_h^T Xhat](psi_j) = sum_r U[r,h] eta_r phi_t[r,j] Xhat[n,r,j]
    (section 3.2).  Without ``delta``: [n][H][Q]; with: [n][T][H][Q]."""
    X = _c128(X)
    UH = np.asarray(U, dtype=np.float64)[:, :H] * eta(w, Q)[:, None]   # [K][H]
    if delta is None:
        return np.ascontiguousarray(np.einsum("rh,nrj->nhj", UH, X))
    ph = phase(k, delta, Q)                                               # [T][K][Q]
    return np.ascontiguousarray(np.einsum("rh,trj,nrj->nthj", UH, ph, X))


def landscape_rings(Ar, Br, pairs=None) -> np.ndarray:
    """Direct O(H Q^2) psi-space sum.  Ar [n_img][H][Q]; Br [n_tgt][T][H][Q].
    Returns X [n_img][n_tgt][T][Q], or [npairs][T][Q] for a pair list."""
    Ar, Br = _c128(Ar), _c128(Br)
    na, H, Q = Ar.shape
    nb, T = Br.shape[:2]
    if pairs is None:
        ia, ib = np.meshgrid(np.arange(na), np.arange(nb), indexing="ij")
        ia, ib = ia.ravel(), ib.ravel()
    else:
        ia = np.asarray([p[0] for p in pairs])
        ib = np.asarray([p[1] for p in pairs])
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ib = np.ascontiguousarray(ib, dtype=np.int32)
    X = np.zeros((len(ia), T, Q), dtype=np.complex128)
    ipt = ctypes.POINTER(ctypes.c_int)
    _load().oracle_landscape_pairs(len(ia), ia.ctypes.data_as(ipt), ib.ctypes.data_as(ipt),
                                   T, H, Q, _dp(Ar), _dp(Br), _dp(X))
    if pairs is None:
        return X.reshape(na, nb, T, Q)
    return X


def landscape(A, B, U, H: int, k, w, delta, pairs=None) -> np.ndarray:
    """X_H[a,b,t,m] for images A [n_img][K][Q] and targets B [n_tgt][K][Q]."""
    Q = A.shape[-1]
    Ar = principal_rings(A, U, H, w, Q)
    Br = principal_rings(B, U, H, w, Q, k=k, delta=delta)
    return landscape_rings(Ar, Br, pairs)


# --------------------------------------------------------------------------
# decisions (section 2.7) and the soft-alignment score
# --------------------------------------------------------------------------
def rotate_ring(R, gamma):
    """A ring of Q samples rotated by any angle gamma (section 2.2): its
    Fourier-Bessel coefficients (the DFT over psi, divided by Q) times
    exp(-i q gamma), summed back at the grid angles.  The band is |q| <= Q/2
    with the q = Q/2 term split evenly between +Q/2 and -Q/2 (its cosine), so
    that grid rotations shift the samples exactly.  R [..., Q]."""
    R = _c128(R)
    Q = R.shape[-1]
    c = np.fft.fft(R, axis=-1) / Q
    q = np.arange(Q)
    qs = np.where(q < Q // 2, q, q - Q).astype(np.float64)    # symmetric representatives
    psi = 2.0 * math.pi * np.arange(Q) / Q
    E = np.exp(1j * qs[:, None] * (psi[None, :] - gamma))       # [q][j]
    if Q % 2 == 0:
        E[Q // 2] = np.cos((Q // 2) * (psi - gamma))
    return c @ E


def landscape_offgrid(Ar, Br, gammas) -> np.ndarray:
    """X(gamma) = sum_h sum_j conj(Ar[h](psi_j)) [R_gamma Br[h]](psi_j) for the
    principal rings of one image (Ar [H][Q]) and one translated target (Br
    [H][Q]) at any rotations gamma (rotate_ring; the direct psi-space sum of
    ``landscape`` at gamma = 2 pi m / Q)."""
    Ar, Br = _c128(Ar), _c128(Br)
    out = np.empty(len(gammas), dtype=np.complex128)
    for i, g in enumerate(gammas):
        out[i] = np.sum(np.conj(Ar) * rotate_ring(Br, float(g)))
    return out


def landscape_metrics(X_est, X_ref):
    """Section 3.5, on the real parts of two landscapes of the same shape
    [n_pairs][...]: the relative error in the Frobenius norm over the whole
    array, the correlation over the whole array, and per pair the fraction f
    of the true inner products X_ref that are <= X_ref at the approximate
    optimum argmax X_est (the first maximum; NaN if a value is not finite).
    Returns (rel_fro, corr, f [n_pairs])."""
    E = np.asarray(X_est).real.astype(np.float64)
    Rr = np.asarray(X_ref).real.astype(np.float64)
    n = E.shape[0]
    E2, R2 = E.reshape(n, -1), Rr.reshape(n, -1)
    rel = math.sqrt(float(np.sum((E2 - R2) ** 2)) / float(np.sum(R2 ** 2)))
    e, r = E2.ravel(), R2.ravel()
    de, dr = e - e.mean(), r - r.mean()
    corr = float(np.sum(de * dr) / math.sqrt(float(np.sum(de * de)) * float(np.sum(dr * dr))))
    f = np.empty(n)
    for p in range(n):
        if not (np.isfinite(E2[p]).all() and np.isfinite(R2[p]).all()):
            f[p] = np.nan
            continue
        i = int(np.argmax(E2[p]))          # first maximum
        f[p] = np.count_nonzero(R2[p] <= R2[p, i]) / R2.shape[1]
    return rel, corr, f


def top_targets(score, k: int):
    """The k best targets of each image (candidates of principal-mode
    marching, section 5): targets by decreasing score, ties to the smaller
    target, NaN never taken; -1 pads the slots beyond the finite scores."""
    S = np.asarray(score, dtype=np.float64)
    out = -np.ones((S.shape[0], k), dtype=np.int64)
    for a in range(S.shape[0]):
        ok = [b for b in range(S.shape[1]) if not math.isnan(S[a, b])]
        ok.sort(key=lambda b: (-S[a, b], b))
        out[a, :min(k, len(ok))] = ok[:k]
    return out


def best(X):
    """argmax over (t, m) of Re X per pair; ties go to the smallest t*Q + m.
    A pair whose landscape holds a value that is not finite (NaN or an
    infinity) gets score NaN and indices -1.
    Returns (score, m, t) with the leading pair axes of X."""
    R = np.asarray(X).real
    lead = R.shape[:-2]
    T, Q = R.shape[-2:]
    flat = R.reshape(-1, T * Q)
    idx = np.argmax(flat, axis=1)
    score = flat[np.arange(flat.shape[0]), idx]
    bad = ~np.isfinite(flat).all(axis=1)
    score = np.where(bad, np.nan, score)
    idx = np.where(bad, -1, idx)
    m = np.where(bad, -1, idx % Q)
    t = np.where(bad, -1, idx // Q)
    return score.reshape(lead), m.reshape(lead), t.reshape(lead)


def _logsumexp(x, axis):
    mx = np.max(x, axis=axis, keepdims=True)
    return (mx + np.log(np.sum(np.exp(x - mx), axis=axis, keepdims=True))).squeeze(axis)


def lse(X, inv_sigma2: float):
    """lse_pair[a,b] = log sum_{t,m} exp(inv_sigma2 Re X); lse_img[a] =
    log sum_b exp(lse_pair[a,b]).  Soft version of the maximum-likelihood
    alignment: the Gaussian log-likelihood of section 2.6 is, up to
    gamma-independent terms, X / sigma^2.
    A pair whose landscape holds a value that is not finite gets NaN, and so
    does every image with such a pair."""
    R = np.asarray(X).real
    na, nb, T, Q = R.shape
    R = R.reshape(na, nb, T * Q)
    bad = ~np.isfinite(R).all(axis=2)
    lp = _logsumexp(np.where(bad[..., None], 0.0, R) * inv_sigma2, axis=2)
    lp = np.where(bad, np.nan, lp)
    li = np.where(bad.any(axis=1), np.nan, _logsumexp(np.where(bad, 0.0, lp), axis=1))
    return lp, li


def lse_loss(A, B, U, H, k, w, delta, inv_sigma2, g):
    X = landscape(A, B, U, H, k, w, delta)
    _, li = lse(X, inv_sigma2)
    return float(np.dot(np.asarray(g, dtype=np.float64), li))


def lse_grad(A, B, U, H: int, k, w, delta, inv_sigma2: float, g):
    """Gradient of L = sum_a g[a] lse_img[a] with respect to the target polar
    samples Bhat (complex convention dL/dRe + i dL/dIm) and to U[:, :H]
    (U treated as a free matrix; the eigendecomposition is not differentiated).

    P[a,b,t,m] = g[a] inv_sigma2 exp(inv_sigma2 Re X - lse_img[a]) = dL/dRe X.
    Ring gradients are the direct sums of ``direct.c``; the chain rule through
    the recombination and the translation phase is the adjoint of each map."""
    A, B = _c128(A), _c128(B)
    Q = A.shape[-1]
    U = np.asarray(U, dtype=np.float64)
    Ar = principal_rings(A, U, H, w, Q)                       # [na][H][Q]
    Br = principal_rings(B, U, H, w, Q, k=k, delta=delta)     # [nb][T][H][Q]
    X = landscape_rings(Ar, Br)
    _, li = lse(X, inv_sigma2)
    g = np.asarray(g, dtype=np.float64)
    P = g[:, None, None, None] * inv_sigma2 * np.exp(inv_sigma2 * X.real - li[:, None, None, None])
    P = np.ascontiguousarray(P, dtype=np.float64)
    na, nb, T = X.shape[:3]
    gBr = np.zeros_like(Br)
    gAr = np.zeros_like(Ar)
    lib = _load()
    lib.oracle_grad_tgt_rings(na, nb, T, H, Q, _dp(P), _dp(Ar), _dp(gBr))
    lib.oracle_grad_img_rings(na, nb, T, H, Q, _dp(P), _dp(Br), _dp(gAr))
    e = eta(w, Q)
    ph = phase(k, delta, Q)                                   # [T][K][Q]
    UH = U[:, :H]
    # Br[b,t,h,j] = sum_r UH[r,h] e_r ph[t,r,j] B[b,r,j]  (complex-linear in B)
    gB = np.einsum("rh,r,trj,bthj->brj", UH, e, np.conj(ph), gBr)
    # real U: dL/dU[r,h] = Re sum conj(g_ring) * d(ring)/dU[r,h]
    gU = np.einsum("bthj,r,trj,brj->rh", np.conj(gBr), e, ph, B).real
    gU += np.einsum("ahj,r,arj->rh", np.conj(gAr), e, A).real
    return gB, gU
