"""Seeded synthetic volumes for rotational volume alignment (paper section 4).

Like the rest of ``synth`` this module only *makes inputs*: spherical shells
of radii k_r with quadrature weights for ``k^2 dk``, volumes made of Gaussian
blobs, and their spherical-harmonic coefficients on each shell, computed in
closed form.  It holds none of the alignment arithmetic (no kernels, no
Wigner-d tables, no landscape).

Conventions.  Fourier transform ``F(k) = \\int f(x) exp(-i k.x) dx`` on R^3; a
blob ``c exp(-|x - mu|^2 / (2 s^2))`` has ``F(k) = c (2 pi s^2)^{3/2}
exp(-s^2 |k|^2 / 2) exp(-i k.mu)``.  Spherical harmonics are the orthonormal
ones with the Condon-Shortley phase (scipy's ``sph_harm_y``), so the
plane-wave expansion gives the shell coefficients

    F_l^m(k) = sum_blobs c (2 pi s^2)^{3/2} exp(-s^2 k^2 / 2) 4 pi (-i)^l j_l(k |mu|) conj(Y_l^m(mu / |mu|)).

Coefficients are stored l-major, index ``l^2 + l + m`` for ``-l <= m <= l``.
A real volume has ``conj(F_l^m) = (-1)^(l+m) F_l^(-m)``.

Rotations: ``R(alpha, beta, gamma) = R_z(alpha) R_y(beta) R_z(gamma)``
(right-handed, counter-clockwise); the rotated volume ``f(R^-1 x)`` is the
same blobs with centres ``R mu``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.special as sp

__all__ = ["shell_grid", "n_coeffs", "rotation_matrix", "random_rotations", "blob_params_3d",
           "sh_coeffs", "real_sh_noise", "VolConfig", "VOL_CONFIGS", "vol_config", "VolProblem",
           "make_volume_problem", "beta_grid"]


def shell_grid(k_max: float, K: int):
    """Radii k_r and weights w_r with sum_r g(k_r) w_r ~ \\int_0^k_max g(k) k^2 dk
    (Gauss-Legendre nodes on [0, k_max], weights times k^2)."""
    x, wx = np.polynomial.legendre.leggauss(K)
    k = (x + 1.0) * (k_max / 2.0)
    w = wx * (k_max / 2.0) * k * k
    return k.astype(np.float64), w.astype(np.float64)


def n_coeffs(L: int) -> int:
    return (L + 1) * (L + 1)


def beta_grid(n: int) -> np.ndarray:
    """n interior angles 2 pi j / n, j = 0..n-1 (the same uniform periodic grid
    as the two azimuthal angles; values above pi stand for negative angles)."""
    return 2.0 * math.pi * np.arange(n) / n


def rotation_matrix(alpha: float, beta: float, gamma: float) -> np.ndarray:
    def rz(a):
        return np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])

    def ry(b):
        return np.array([[math.cos(b), 0.0, math.sin(b)], [0.0, 1.0, 0.0], [-math.sin(b), 0.0, math.cos(b)]])

    return rz(alpha) @ ry(beta) @ rz(gamma)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n rotations uniform on SO(3) (normalised Gaussian quaternions)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], axis=1)


def blob_params_3d(rng: np.random.Generator, n: int, n_blobs: int, radius: float = 0.5):
    """Centres uniform in the ball of the given radius, widths U[0.02, 0.08],
    amplitudes N(0, 1)."""
    d = rng.standard_normal((n, n_blobs, 3))
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    r = radius * rng.random((n, n_blobs)) ** (1.0 / 3.0)
    mu = d * r[..., None]
    s = rng.uniform(0.02, 0.08, size=(n, n_blobs))
    c = rng.standard_normal((n, n_blobs))
    return mu, s, c


def _lm_tables(L: int):
    ls = np.concatenate([np.full(2 * l + 1, l) for l in range(L + 1)])
    ms = np.concatenate([np.arange(-l, l + 1) for l in range(L + 1)])
    return ls, ms


def sh_coeffs(mu, s, c, k, L: int) -> np.ndarray:
    """Closed-form shell coefficients of blob volumes: complex128 [n][K][(L+1)^2]."""
    mu = np.asarray(mu, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    n, nb = s.shape
    K = k.shape[0]
    ls, ms = _lm_tables(L)
    out = np.empty((n, K, n_coeffs(L)), dtype=np.complex128)
    il = (-1j) ** np.arange(L + 1)
    for v in range(n):
        rr = np.linalg.norm(mu[v], axis=-1)                              # [nb]
        th = np.arccos(np.clip(np.where(rr > 0, mu[v, :, 2] / np.where(rr > 0, rr, 1.0), 1.0), -1.0, 1.0))
        ph = np.arctan2(mu[v, :, 1], mu[v, :, 0])
        Y = sp.sph_harm_y(ls[None, :], ms[None, :], th[:, None], ph[:, None])   # [nb][lm]
        amp = c[v][:, None] * (2.0 * math.pi * s[v][:, None] ** 2) ** 1.5 \
            * np.exp(-0.5 * (s[v][:, None] * k[None, :]) ** 2)           # [nb][K]
        j = sp.spherical_jn(np.arange(L + 1)[None, None, :], (k[None, :, None] * rr[:, None, None]))  # [nb][K][L+1]
        radial = amp[..., None] * 4.0 * math.pi * il[None, None, :] * j  # [nb][K][L+1]
        out[v] = np.einsum("bki,bi->ki", radial[:, :, ls], np.conj(Y))
    return out


def real_sh_noise(rng: np.random.Generator, n: int, w, L: int, var: np.ndarray) -> np.ndarray:
    """Noise of a real volume in shell coefficients: E|n_l^m(k_r)|^2 = var / w_r
    and conj(n_l^m) = (-1)^(l+m) n_l^(-m)."""
    w = np.asarray(w, dtype=np.float64)
    K = w.shape[0]
    out = np.zeros((n, K, n_coeffs(L)), dtype=np.complex128)
    sd = np.sqrt(np.asarray(var, dtype=np.float64)[:, None] / w[None, :])   # [n][K]
    for l in range(L + 1):
        base = l * l + l
        x = rng.standard_normal((n, K)) * sd
        out[:, :, base] = x if l % 2 == 0 else 1j * x
        for m in range(1, l + 1):
            z = (rng.standard_normal((n, K)) + 1j * rng.standard_normal((n, K))) * sd / math.sqrt(2.0)
            out[:, :, base + m] = z
            out[:, :, base - m] = (-1) ** (l + m) * np.conj(z)
    return out


@dataclass
class VolConfig:
    name: str
    K: int             # shells
    L: int             # largest degree; M = 2 L + 1 orders
    k_max: float
    n_vol: int         # volumes to align (noisy rotated copies)
    n_tgt: int         # targets (clean)
    n_blobs: int
    radius: float
    snr: float | None  # None: no noise
    n_beta: int        # interior angles (uniform grid of beta_grid)
    H_C: int           # radial rank
    H_D: int           # degree rank


VOL_CONFIGS = {
    # small cases the oracle finishes in seconds
    "vtiny": VolConfig("vtiny", K=6, L=6, k_max=6.0, n_vol=4, n_tgt=2, n_blobs=6, radius=0.5, snr=None,
                       n_beta=13, H_C=6, H_D=7),
    "vsmall": VolConfig("vsmall", K=16, L=16, k_max=16.0, n_vol=6, n_tgt=2, n_blobs=12, radius=0.5, snr=1.0,
                        n_beta=33, H_C=8, H_D=8),
    # the paper's volume example: many volumes to one target (shapes of the
    # TRPV1 study stood in for by blob volumes: 48 shells, degrees to 48)
    "volume": VolConfig("volume", K=48, L=48, k_max=48.0, n_vol=96, n_tgt=1, n_blobs=32, radius=0.5, snr=0.5,
                        n_beta=97, H_C=16, H_D=16),
}


def vol_config(name: str, **over) -> VolConfig:
    d = dict(VOL_CONFIGS[name].__dict__)
    d.update(over)
    return VolConfig(**d)


@dataclass
class VolProblem:
    cfg: VolConfig
    k: np.ndarray          # [K]
    w: np.ndarray          # [K]
    beta: np.ndarray       # [n_beta]
    A: np.ndarray          # [n_vol][K][(L+1)^2] complex128 (noisy rotated copies)
    B: np.ndarray          # [n_tgt][K][(L+1)^2] complex128 (clean targets)
    truth: dict            # source target and rotation matrix of each copy


def make_volume_problem(cfg: VolConfig, seed: int) -> VolProblem:
    rng = np.random.default_rng(seed)
    k, w = shell_grid(cfg.k_max, cfg.K)
    mu, s, c = blob_params_3d(rng, cfg.n_tgt, cfg.n_blobs, cfg.radius)
    src = rng.integers(0, cfg.n_tgt, size=cfg.n_vol)
    rot = random_rotations(rng, cfg.n_vol)
    mu_c = np.einsum("vij,vbj->vbi", rot, mu[src])
    B = sh_coeffs(mu, s, c, k, cfg.L)
    A = sh_coeffs(mu_c, s[src], c[src], k, cfg.L)
    if cfg.snr is not None:
        norm2 = np.einsum("k,vki->v", w, np.abs(A) ** 2)
        var = norm2 / (cfg.K * n_coeffs(cfg.L) * cfg.snr)
        A = A + real_sh_noise(rng, cfg.n_vol, w, cfg.L, var)
    return VolProblem(cfg, k, w, beta_grid(cfg.n_beta), A, B, {"src": src, "rot": rot})
