"""Principal-mode marching (paper section 5) and landscape quality (section 3.5).

``march`` aligns every image at a low rank, keeps each image's best-scoring
targets, and evaluates those pairs again at a higher rank with the same
principal vectors: the low-rank pass is the cheap coarse landscape, the
high-rank pass refines the candidates.  ``landscape_metrics`` measures how
well a low-rank landscape stands in for the full one.  Both only marshal
arguments to the library (align_pairs, align_top_targets, align_pairs_list,
align_landscape_metrics); every step runs in its kernels.
"""
from __future__ import annotations

import torch

from . import Plan, align_landscape_metrics, align_top_targets


def march(A_polar, B_polar, k, w, delta, H_low: int, H_high: int, n_cand: int, precision: str = "fp32",
          products: int = 3, hermitian: bool = True, sigma_delta: float = 0.0, stream=None) -> dict:
    """Two-stage marching.  Returns the candidates cand [n_img][n_cand] (-1
    where an image has fewer finite low-rank scores), and for each candidate
    its low-rank score and its high-rank best (score, m, t), all
    [n_img][n_cand]; plus both plans."""
    low = Plan(A_polar, B_polar, k, w, delta, H_low, precision=precision, products=products,
               hermitian=hermitian, sigma_delta=sigma_delta, stream=stream)
    coarse = low.pairs("best", stream=stream)
    n_img, dev = low.n_img, low.device
    cand = torch.empty((n_img, n_cand), dtype=torch.int32, device=dev)
    align_top_targets(coarse["best_score"], n_cand, cand, stream)
    # the same principal vectors at the higher rank (no second eigensolve)
    U = low.U_lambda(stream)[0][:, :H_high].contiguous()
    high = Plan(A_polar, B_polar, k, w, delta, H_high, precision=precision, products=products,
                hermitian=hermitian, U=U, stream=stream)
    img = torch.arange(n_img, dtype=torch.int32, device=dev).repeat_interleave(n_cand)
    pairs = torch.stack([img, cand.reshape(-1)], dim=1).contiguous()
    fine = high.pairs_list(pairs, "best", stream=stream)
    low_score = torch.gather(coarse["best_score"], 1, cand.clamp(min=0).long())
    low_score = torch.where(cand >= 0, low_score, torch.full_like(low_score, float("nan")))
    return {"cand": cand, "low_score": low_score,
            "score": fine["best_score"].view(n_img, n_cand), "m": fine["best_m"].view(n_img, n_cand),
            "t": fine["best_t"].view(n_img, n_cand), "plans": (low, high)}


def landscape_metrics(X_est: torch.Tensor, X_ref: torch.Tensor, stream=None) -> dict:
    """Relative Frobenius error, correlation and mean f of X_est against X_ref
    (FULL landscapes [n_img][n_tgt][T][Q] of equal shape and dtype), and f per
    pair."""
    n = X_est.shape[0] * X_est.shape[1]
    Xe = X_est.reshape(n, -1).contiguous()
    Xr = X_ref.reshape(n, -1).contiguous()
    f = torch.empty(n, dtype=torch.float32, device=X_est.device)
    stats = torch.empty((n, 6), dtype=torch.float64, device=X_est.device)
    summary = torch.empty(3, dtype=torch.float64, device=X_est.device)
    align_landscape_metrics(Xe, Xr, f, stats, summary, stream)
    s = summary.cpu()
    return {"rel_fro": float(s[0]), "corr": float(s[1]), "mean_f": float(s[2]),
            "f": f.view(X_est.shape[0], X_est.shape[1])}
