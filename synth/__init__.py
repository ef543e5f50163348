"""Seeded synthetic inputs for radial-SVD rotational alignment.

This module only *makes inputs*: the polar quadrature grid, Gaussian-blob
images whose Fourier transform is known in closed form, transformed and noisy
copies of them, and the translation grid.  It holds none of the alignment
method's arithmetic (no ring recombination, no angular FFT, no kernel C, no
landscape), so both the FP64 oracle and the HIP path can consume it without
sharing any of the method.

Conventions (paper section 2.1): the Fourier transform is
``Ahat(k) = \\int A(x) exp(-i k.x) dx``; polar samples ``Ahat(k_r, psi_j)`` with
``psi_j = 2 pi j / Q``.  A Gaussian blob ``c exp(-|x-mu|^2 / (2 s^2))`` has
``Ahat(k) = c 2 pi s^2 exp(-s^2 |k|^2 / 2) exp(-i k.mu)``.

Radial nodes (section 2.3): the paper uses a Gauss-Jacobi rule for ``k dk``;
here Gauss-Legendre nodes on ``[0, k_max]`` with weights multiplied by ``k``
(``sum_r g(k_r) w_r ~ \\int_0^{k_max} g(k) k dk``), ``k_max = N/2``.

Noise (section 2.5): Hermitian noise (the transform of real-space noise) with
per-node variance ``sigma_hat^2 / (w_r dpsi)``; ``sigma_hat^2`` is set per copy
from the requested SNR as ``||B||_w^2 / (K Q SNR)`` with
``||B||_w^2 = sum_{r,j} w_r dpsi |Bhat(k_r, psi_j)|^2``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

__all__ = [
    "gl_grid", "translation_grid", "blob_params", "polar_ft", "Problem",
    "make_problem", "CONFIGS", "config", "batch_configs",
]


# --------------------------------------------------------------------------
# grid
# --------------------------------------------------------------------------
def gl_grid(N: int, K: int):
    """Radial nodes k_r and weights w_r for \\int_0^{N/2} g(k) k dk."""
    k_max = N / 2.0
    x, wx = np.polynomial.legendre.leggauss(K)
    k = (x + 1.0) * (k_max / 2.0)
    w = wx * (k_max / 2.0) * k
    return k.astype(np.float64), w.astype(np.float64)


def translation_grid(T: int, N: int):
    """T in {1, 9, 25}: a centred sqrt(T) x sqrt(T) grid with 1 pixel spacing
    (pixel = 2/N on the [-1,1]^2 image).  Row t = iy*n + ix."""
    n = int(round(math.sqrt(T)))
    if n * n != T:
        raise ValueError("T must be a perfect square")
    px = 2.0 / N
    c = (n - 1) / 2.0
    d = np.zeros((T, 2), dtype=np.float64)
    for iy in range(n):
        for ix in range(n):
            d[iy * n + ix] = ((ix - c) * px, (iy - c) * px)
    return d


# --------------------------------------------------------------------------
# blobs and their closed-form transform
# --------------------------------------------------------------------------
def blob_params(rng: np.random.Generator, n: int, n_blobs: int):
    """Centres uniform in the disk of radius 0.3, widths U[0.02, 0.08],
    amplitudes N(0, 1)."""
    r = 0.3 * np.sqrt(rng.random((n, n_blobs)))
    th = 2.0 * np.pi * rng.random((n, n_blobs))
    mu = np.stack([r * np.cos(th), r * np.sin(th)], axis=-1)
    s = rng.uniform(0.02, 0.08, size=(n, n_blobs))
    c = rng.standard_normal((n, n_blobs))
    return mu, s, c


def polar_ft(mu, s, c, k, Q: int, device="cpu", chunk: int = 256) -> torch.Tensor:
    """Closed-form FT of blob images on the polar grid, complex128 [n][K][Q]."""
    mu = torch.as_tensor(mu, dtype=torch.float64, device=device)
    s = torch.as_tensor(s, dtype=torch.float64, device=device)
    c = torch.as_tensor(c, dtype=torch.float64, device=device)
    k = torch.as_tensor(k, dtype=torch.float64, device=device)
    n, nb = s.shape
    K = k.shape[0]
    psi = torch.arange(Q, dtype=torch.float64, device=device) * (2.0 * math.pi / Q)
    kx = k[:, None] * torch.cos(psi)[None, :]          # [K][Q]
    ky = k[:, None] * torch.sin(psi)[None, :]
    out = torch.empty((n, K, Q), dtype=torch.complex128, device=device)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        acc = torch.zeros((i1 - i0, K, Q), dtype=torch.complex128, device=device)
        for ib in range(nb):
            si = s[i0:i1, ib][:, None, None]
            amp = c[i0:i1, ib][:, None, None] * (2.0 * math.pi) * si * si \
                * torch.exp(-0.5 * si * si * (k * k)[None, :, None])
            ph = -(kx[None] * mu[i0:i1, ib, 0][:, None, None]
                   + ky[None] * mu[i0:i1, ib, 1][:, None, None])
            acc += amp * torch.polar(torch.ones_like(ph), ph)
        out[i0:i1] = acc
    return out


def _rotate_translate(mu, gamma, delta):
    """Centres of R_gamma T_delta A: mu -> R_gamma (mu + delta) (rotation
    counter-clockwise by gamma)."""
    m = mu + delta[:, None, :]
    cg, sg = np.cos(gamma)[:, None], np.sin(gamma)[:, None]
    return np.stack([cg * m[..., 0] - sg * m[..., 1], sg * m[..., 0] + cg * m[..., 1]], axis=-1)


def _weighted_norm2(X: torch.Tensor, w, Q: int) -> torch.Tensor:
    wt = torch.as_tensor(w, dtype=torch.float64, device=X.device) * (2.0 * math.pi / Q)
    return (X.real ** 2 + X.imag ** 2).mul(wt[None, :, None]).sum(dim=(1, 2))


def hermitian_noise(gen: torch.Generator, n: int, w, Q: int, var_scale: torch.Tensor,
                    device="cpu") -> torch.Tensor:
    """Noise with E|n(k_r,psi_j)|^2 = var_scale / (w_r dpsi) and
    n(k, psi + pi) = conj(n(k, psi))."""
    K = len(w)
    dpsi = 2.0 * math.pi / Q
    w_t = torch.as_tensor(w, dtype=torch.float64, device=device)
    std = torch.sqrt(var_scale.to(device)[:, None, None] / (w_t[None, :, None] * dpsi) / 2.0)
    h = Q // 2
    re = torch.randn((n, K, h), generator=gen, dtype=torch.float64, device=device)
    im = torch.randn((n, K, h), generator=gen, dtype=torch.float64, device=device)
    half = torch.complex(re, im) * std
    return torch.cat([half, half.conj()], dim=2)


# --------------------------------------------------------------------------
# configurations of the paper's image-alignment workload (synthetic stand-ins)
# --------------------------------------------------------------------------
@dataclass
class Config:
    name: str
    N: int
    K: int
    Q: int
    n_img: int
    n_tgt: int
    T: int
    H: int
    n_blobs: int = 16
    snr: float | None = 0.5          # None: cfg-1 style iid complex noise
    grid_rotation: bool = False      # targets rotated by a grid angle (index shift)
    noisy_side: str = "tgt"          # which side holds the transformed noisy copies
    extra: dict = field(default_factory=dict)


CONFIGS = {
    "tiny": Config("tiny", N=32, K=16, Q=64, n_img=8, n_tgt=8, T=1, H=16,
                   snr=None, grid_rotation=True),
    "fp32": Config("fp32", N=128, K=64, Q=256, n_img=1024, n_tgt=1024, T=9, H=16),
    "precision": Config("precision", N=256, K=128, Q=512, n_img=4096, n_tgt=4096, T=9,
                        H=24, n_blobs=32, snr=0.1),
    "diff": Config("diff", N=128, K=64, Q=256, n_img=2048, n_tgt=256, T=9, H=16,
                   noisy_side="img"),
    "diff_fd": Config("diff_fd", N=32, K=16, Q=64, n_img=16, n_tgt=8, T=9, H=8,
                      noisy_side="img"),
}


def batch_configs(n_jobs: int = 64, seed: int = 4000, scale: float = 1.0):
    """Independent jobs of the batching workload: N uniform in {64, 96, 128,
    192, 256} with K = N/2 and Q = 2N; N_A log-uniform in [128, 2048] and N_B
    log-uniform in [64, 1024] (both multiplied by ``scale``, at least 8);
    T uniform in {1, 9, 25}; H uniform in [8, 32]."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n_jobs):
        N = int(rng.choice([64, 96, 128, 192, 256]))
        na = int(round(math.exp(rng.uniform(math.log(128), math.log(2048)))))
        nb = int(round(math.exp(rng.uniform(math.log(64), math.log(1024)))))
        T = int(rng.choice([1, 9, 25]))
        H = int(rng.integers(8, 33))
        out.append(Config(f"batch{j}", N=N, K=N // 2, Q=2 * N, n_img=max(8, int(na * scale)),
                          n_tgt=max(8, int(nb * scale)), T=T, H=H))
    return out


def config(name: str, **over) -> Config:
    base = CONFIGS[name]
    d = dict(base.__dict__)
    d.update(over)
    return Config(**d)


@dataclass
class Problem:
    cfg: Config
    k: np.ndarray          # [K] float64
    w: np.ndarray          # [K] float64
    delta: np.ndarray      # [T][2] float64
    A: torch.Tensor        # [n_img][K][Q] complex128
    B: torch.Tensor        # [n_tgt][K][Q] complex128
    truth: dict            # source index, gamma, delta0 of the noisy copies
    hermitian: bool


def make_problem(cfg: Config, seed: int, device="cpu") -> Problem:
    """Sources are clean blob images; copies are rotated (and, for
    continuous rotations, shifted by up to one pixel) noisy copies of random
    sources.  ``noisy_side`` says whether the copies are the targets (B) or the
    images (A)."""
    rng = np.random.default_rng(seed)
    k, w = gl_grid(cfg.N, cfg.K)
    delta = translation_grid(cfg.T, cfg.N)
    n_src, n_cp = (cfg.n_img, cfg.n_tgt) if cfg.noisy_side == "tgt" else (cfg.n_tgt, cfg.n_img)
    mu, s, c = blob_params(rng, n_src, cfg.n_blobs)
    src = rng.integers(0, n_src, size=n_cp)
    px = 2.0 / cfg.N
    if cfg.grid_rotation:
        shift = rng.integers(0, cfg.Q, size=n_cp)
        gamma = shift * (2.0 * np.pi / cfg.Q)
        d0 = np.zeros((n_cp, 2))
    else:
        gamma = 2.0 * np.pi * rng.random(n_cp)
        d0 = rng.uniform(-px, px, size=(n_cp, 2))
        shift = None
    S = polar_ft(mu, s, c, k, cfg.Q, device=device)
    if cfg.grid_rotation:
        idx = torch.as_tensor(src, device=device)
        C = S[idx].clone()
        for i in range(n_cp):
            C[i] = torch.roll(C[i], shifts=int(shift[i]), dims=1)   # Bhat(psi - gamma)
    else:
        mu_c = _rotate_translate(mu[src], gamma, d0)
        C = polar_ft(mu_c, s[src], c[src], k, cfg.Q, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed + 7919)
    if cfg.snr is None:
        rms = torch.sqrt((C.real ** 2 + C.imag ** 2).mean(dim=(1, 2)))
        std = (0.1 * rms / math.sqrt(2.0))[:, None, None]
        noise = torch.complex(torch.randn(C.shape, generator=gen, dtype=torch.float64, device=device),
                              torch.randn(C.shape, generator=gen, dtype=torch.float64, device=device)) * std
        hermitian = False
    else:
        var = _weighted_norm2(C, w, cfg.Q) / (cfg.K * cfg.Q * cfg.snr)
        noise = hermitian_noise(gen, n_cp, w, cfg.Q, var, device=device)
        hermitian = True
    C = C + noise
    truth = {"src": src, "gamma": gamma, "delta0": d0, "shift": shift}
    A, B = (S, C) if cfg.noisy_side == "tgt" else (C, S)
    return Problem(cfg, k, w, delta, A, B, truth, hermitian)
