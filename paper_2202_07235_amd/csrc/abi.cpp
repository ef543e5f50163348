// C ABI of the radsvd library: argument validation (always before the first
// launch), workspace carving, plan lifetime and error reporting.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "common.h"
#include "internal.h"
#include "volume.h"

using namespace radsvd;

namespace {

thread_local char g_err[512] = "";

radsvd_status fail(radsvd_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

radsvd_status dev_check(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(RADSVD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return RADSVD_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

radsvd_status validate_problem(const radsvd_problem *pr) {
    if (!pr) return fail(RADSVD_ERR_INVALID_ARG, "problem is NULL");
    if (pr->K < 2 || pr->K > kMaxK) return fail(RADSVD_ERR_INVALID_ARG, "K=%d outside [2, %d]", pr->K, kMaxK);
    if (pr->Q < 8 || pr->Q > kMaxQ || (pr->Q & 1) || !fft_size_ok(pr->Q))
        return fail(RADSVD_ERR_INVALID_ARG, "Q=%d must be even, 2^a 3^b, in [8, %d]", pr->Q, kMaxQ);
    const int hmax = pr->K < kMaxH ? pr->K : kMaxH;
    if (pr->H < 1 || pr->H > hmax) return fail(RADSVD_ERR_INVALID_ARG, "H=%d outside [1, %d]", pr->H, hmax);
    if (pr->T < 1 || pr->T > kMaxT) return fail(RADSVD_ERR_INVALID_ARG, "T=%d outside [1, %d]", pr->T, kMaxT);
    if (!pr->k || !pr->w) return fail(RADSVD_ERR_INVALID_ARG, "k or w is NULL");
    if (!pr->delta && pr->T != 1) return fail(RADSVD_ERR_INVALID_ARG, "delta is NULL with T=%d", pr->T);
    for (int r = 0; r < pr->K; ++r) {
        if (!(pr->k[r] > 0.0) || !isfinite(pr->k[r]))
            return fail(RADSVD_ERR_INVALID_ARG, "k[%d] must be finite and > 0", r);
        if (!(pr->w[r] > 0.0) || !isfinite(pr->w[r]))
            return fail(RADSVD_ERR_INVALID_ARG, "w[%d] must be finite and > 0", r);
    }
    if (pr->delta)
        for (int t = 0; t < 2 * pr->T; ++t)
            if (!isfinite(pr->delta[t])) return fail(RADSVD_ERR_INVALID_ARG, "delta[%d] not finite", t);
    if (pr->prec < RADSVD_FP64 || pr->prec > RADSVD_BF16X3)
        return fail(RADSVD_ERR_INVALID_ARG, "prec=%d unknown", pr->prec);
    if (pr->hermitian != 0 && pr->hermitian != 1)
        return fail(RADSVD_ERR_INVALID_ARG, "hermitian must be 0 or 1");
    if (pr->prec == RADSVD_BF16X3 && pr->products != 3 && pr->products != 6)
        return fail(RADSVD_ERR_INVALID_ARG, "products=%d must be 3 or 6 for BF16X3", pr->products);
    if (!(pr->sigma_delta >= 0.0) || !isfinite(pr->sigma_delta))
        return fail(RADSVD_ERR_INVALID_ARG, "sigma_delta must be finite and >= 0");
    return RADSVD_OK;
}

struct Layout {
    size_t off_k, off_eta, off_delta, off_phase, off_C, off_U, off_lam, off_ueta, off_rsum, off_gram, off_g0,
        off_Ag, off_Bg, off_Af, off_Bf, off_log, total;
    size_t Af_bytes, Bf_bytes;
    int nsplit, H8, nplanes_a, nplanes_b, ffmt_a, ffmt_b, na_pad, nb_pad, Qc;
    bool fast;
};

Layout make_layout(const radsvd_problem *pr, int n_img, int n_tgt) {
    Layout L{};
    const int K = pr->K, Q = pr->Q, H = pr->H, T = pr->T;
    const size_t R = (pr->prec == RADSVD_FP64) ? 8 : 4;
    const size_t CX = 2 * R;
    L.Qc = pr->hermitian ? Q / 2 + 1 : Q;
    L.fast = pr->hermitian && pr->prec != RADSVD_FP64;
    L.H8 = (H + 7) / 8 * 8;
    // bf16x3 loads two bf16 planes per side with 3 products; with 6 products
    // the images keep their three planes and the targets keep FP32 values (in
    // bf16 fragment order), split into three bf16 terms in registers
    const bool b3 = pr->prec == RADSVD_BF16X3;
    const bool split_b = b3 && pr->products != 3;
    L.ffmt_a = pr->prec == RADSVD_FP32 ? kFragF32 : kFragBF16;
    L.ffmt_b = pr->prec == RADSVD_FP32 ? kFragF32 : (split_b ? kFragF32B : kFragBF16);
    if (wide_plan(pr->prec, pr->products, pr->hermitian, Q)) {
        L.ffmt_a = kFragBF16D;
        L.ffmt_b = kFragF32P;
    }
    L.nplanes_a = b3 ? (pr->products == 3 ? 2 : 3) : 1;
    L.nplanes_b = b3 ? (pr->products == 3 ? 2 : 1) : 1;
    L.na_pad = (n_img + kFastTA - 1) / kFastTA * kFastTA;
    L.nb_pad = (n_tgt + kFastTB - 1) / kFastTB * kFastTB;
    const int tiles = (K + 63) / 64;
    int ns = 1024 / (tiles * tiles);
    if (ns > n_tgt) ns = n_tgt;
    if (ns < 1) ns = 1;
    L.nsplit = ns;
    const int KP = (K + 1) & ~1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.off_k = take(K * 8);
    L.off_eta = take(K * 8);
    L.off_delta = take((size_t)T * 2 * 8);
    L.off_phase = take((size_t)T * K * Q * CX);
    L.off_C = take((size_t)K * K * 8);
    L.off_U = take((size_t)K * K * 8);
    L.off_lam = take((size_t)K * 8);
    L.off_ueta = take((size_t)K * H * R);
    L.off_rsum = take((size_t)n_tgt * K * 16);
    (void)KP;
    L.off_gram = take((size_t)ns * K * K * 8);
    L.off_g0 = take((size_t)K * K * 8);
    L.off_log = take(eig_log_bytes(K));
    L.off_Ag = take((size_t)n_img * L.Qc * H * CX);
    L.off_Bg = take((size_t)n_tgt * T * L.Qc * H * CX);
    if (L.fast) {
        // one fragment-ordered operand block per (tile, q): 8 images or 16 targets
        const size_t blk_a = (size_t)L.nplanes_a * frag_plane_bytes(L.ffmt_a, L.H8);
        const size_t blk_b = (size_t)L.nplanes_b * frag_plane_bytes(L.ffmt_b, L.H8);
        L.Af_bytes = (size_t)(L.na_pad / kFastTA) * L.Qc * blk_a;
        L.Bf_bytes = (size_t)T * (L.nb_pad / kFastTB) * L.Qc * blk_b;
        L.off_Af = take(L.Af_bytes);
        L.off_Bf = take(L.Bf_bytes);
    }
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

const char *radsvd_last_error(void) { return g_err; }

size_t align_prepare_workspace(const radsvd_problem *prob, int n_img, int n_tgt) {
    g_err[0] = 0;
    if (validate_problem(prob) != RADSVD_OK) return 0;
    if (n_img < 1 || n_img > (1 << 20) || n_tgt < 1 || n_tgt > (1 << 20)) {
        fail(RADSVD_ERR_INVALID_ARG, "n_img=%d / n_tgt=%d outside [1, 2^20]", n_img, n_tgt);
        return 0;
    }
    return make_layout(prob, n_img, n_tgt).total;
}

radsvd_status align_prepare(const radsvd_problem *prob, int n_img, const void *A_polar, int n_tgt,
                            const void *B_polar, const double *U_in, void *ws, size_t ws_bytes,
                            void *stream, radsvd_plan **out) {
    g_err[0] = 0;
    radsvd_status st = validate_problem(prob);
    if (st != RADSVD_OK) return st;
    if (!out) return fail(RADSVD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_img < 1 || n_img > (1 << 20) || n_tgt < 1 || n_tgt > (1 << 20))
        return fail(RADSVD_ERR_INVALID_ARG, "n_img=%d / n_tgt=%d outside [1, 2^20]", n_img, n_tgt);
    if (!A_polar || !B_polar) return fail(RADSVD_ERR_INVALID_ARG, "A_polar or B_polar is NULL");
    if (!aligned(A_polar, 16) || !aligned(B_polar, 16))
        return fail(RADSVD_ERR_INVALID_ARG, "A_polar / B_polar must be 16-byte aligned");
    if (U_in && !aligned(U_in, 8)) return fail(RADSVD_ERR_INVALID_ARG, "U_in must be 8-byte aligned");
    const Layout L = make_layout(prob, n_img, n_tgt);
    if (!ws) return fail(RADSVD_ERR_WORKSPACE, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(RADSVD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(RADSVD_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);

    radsvd_plan *p = new (std::nothrow) radsvd_plan();
    if (!p) return fail(RADSVD_ERR_DEVICE, "host allocation failed");
    p->K = prob->K;
    p->Q = prob->Q;
    p->H = prob->H;
    p->T = prob->T;
    p->prec = prob->prec;
    p->herm = prob->hermitian;
    p->products = prob->prec == RADSVD_BF16X3 ? prob->products : 0;
    p->sigma_delta = prob->sigma_delta;
    p->n_img = n_img;
    p->n_tgt = n_tgt;
    p->M = prob->Q / 2;
    p->Qc = L.Qc;
    p->H8 = L.H8;
    p->nplanes_a = L.nplanes_a;
    p->nplanes_b = L.nplanes_b;
    p->ffmt_a = L.ffmt_a;
    p->ffmt_b = L.ffmt_b;
    p->na_pad = L.na_pad;
    p->nb_pad = L.nb_pad;
    p->user_U = U_in != nullptr;
    p->band = 0;
    p->waves = 0;
    p->ws = reinterpret_cast<char *>(ws);
    p->ws_bytes = ws_bytes;
    p->A_polar = A_polar;
    p->B_polar = B_polar;
    char *w = p->ws;
    p->d_k = reinterpret_cast<double *>(w + L.off_k);
    p->d_eta = reinterpret_cast<double *>(w + L.off_eta);
    p->d_delta = reinterpret_cast<double *>(w + L.off_delta);
    p->phase = w + L.off_phase;
    p->C = reinterpret_cast<double *>(w + L.off_C);
    p->U = reinterpret_cast<double *>(w + L.off_U);
    p->lam = reinterpret_cast<double *>(w + L.off_lam);
    p->Ueta = w + L.off_ueta;
    p->ringsum = reinterpret_cast<double *>(w + L.off_rsum);
    p->gram_part = reinterpret_cast<double *>(w + L.off_gram);
    p->ring_gram = reinterpret_cast<double *>(w + L.off_g0);
    p->gram_nsplit = L.nsplit;
    p->eig_log = w + L.off_log;
    p->Ag = w + L.off_Ag;
    p->Bg = w + L.off_Bg;
    p->Af = L.fast ? w + L.off_Af : nullptr;
    p->Bf = L.fast ? w + L.off_Bf : nullptr;
    p->Af_bytes = L.Af_bytes;
    p->Bf_bytes = L.Bf_bytes;

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    GridArgs g;
    memset(&g, 0, sizeof(g));
    g.K = prob->K;
    g.Q = prob->Q;
    g.T = prob->T;
    for (int r = 0; r < prob->K; ++r) {
        g.k[r] = prob->k[r];
        g.w[r] = prob->w[r];
    }
    for (int t = 0; t < prob->T; ++t) {
        g.delta[t][0] = prob->delta ? prob->delta[2 * t] : 0.0;
        g.delta[t][1] = prob->delta ? prob->delta[2 * t + 1] : 0.0;
    }
    hipError_t e = launch_setup(p, g, s);
    if (e == hipSuccess) {
        if (U_in) {
            e = launch_user_U(p, U_in, s);
            if (e == hipSuccess) e = launch_ueta(p, U_in, p->H, s);
        } else {
            e = launch_kernel_C(p, s);
            if (e == hipSuccess) e = launch_eig(p, s);
            if (e == hipSuccess) e = launch_ueta(p, p->U, p->K, s);
        }
    }
    if (e == hipSuccess) e = launch_principal_rings(p, s);
    if (e != hipSuccess) {
        delete p;
        return dev_check(e, "align_prepare launch");
    }
    *out = p;
    return RADSVD_OK;
}

radsvd_status align_pairs(const radsvd_plan *p, int flags, float inv_sigma2, float *best_score,
                          int32_t *best_m, int32_t *best_t, float *lse_pair, float *lse_img,
                          void *X_full, void *stream) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    if (flags <= 0 || (flags & ~7)) return fail(RADSVD_ERR_INVALID_ARG, "out_flags=%d invalid", flags);
    if ((flags & RADSVD_OUT_BEST) && (!best_score || !best_m || !best_t))
        return fail(RADSVD_ERR_INVALID_ARG, "BEST output pointers must be non-NULL");
    if ((flags & RADSVD_OUT_LSE) && !lse_pair)
        return fail(RADSVD_ERR_INVALID_ARG, "LSE output lse_pair must be non-NULL");
    if ((flags & RADSVD_OUT_LSE) && !(inv_sigma2 > 0.f && isfinite(inv_sigma2)))
        return fail(RADSVD_ERR_INVALID_ARG, "inv_sigma2 must be finite and > 0");
    if ((flags & RADSVD_OUT_FULL) && !X_full)
        return fail(RADSVD_ERR_INVALID_ARG, "FULL output X_full must be non-NULL");
    if ((flags & RADSVD_OUT_BEST) && (!aligned(best_score, 4) || !aligned(best_m, 4) || !aligned(best_t, 4)))
        return fail(RADSVD_ERR_INVALID_ARG, "BEST outputs must be 4-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (fast_path_supported(p, flags)) {
        e = launch_pairs_fast(p, flags, inv_sigma2, best_score, best_m, best_t, lse_pair, X_full, s);
    } else {
        e = ensure_generic_layout(p, s);
        if (e == hipSuccess)
            e = launch_pairs_generic(p, flags, inv_sigma2, best_score, best_m, best_t, lse_pair, X_full, s);
    }
    if (e == hipSuccess && (flags & RADSVD_OUT_LSE) && lse_img)
        e = launch_lse_img(p->n_img, p->n_tgt, lse_pair, lse_img, s);
    return dev_check(e, "align_pairs launch");
}

size_t align_backward_workspace(const radsvd_plan *p) {
    g_err[0] = 0;
    if (!p) {
        fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
        return 0;
    }
    return backward_bytes(p);
}

radsvd_status align_pairs_backward(const radsvd_plan *p, float inv_sigma2, const float *lse_img,
                                   const float *grad_lse_img, void *grad_B_polar, double *grad_U,
                                   void *bwd_ws, size_t bwd_bytes, void *stream) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    if (!lse_img || !grad_lse_img) return fail(RADSVD_ERR_INVALID_ARG, "lse_img / grad_lse_img NULL");
    if (!(inv_sigma2 > 0.f && isfinite(inv_sigma2)))
        return fail(RADSVD_ERR_INVALID_ARG, "inv_sigma2 must be finite and > 0");
    if (grad_B_polar && !aligned(grad_B_polar, 16))
        return fail(RADSVD_ERR_INVALID_ARG, "grad_B_polar must be 16-byte aligned");
    if (grad_U && !aligned(grad_U, 8)) return fail(RADSVD_ERR_INVALID_ARG, "grad_U must be 8-byte aligned");
    const size_t need = backward_bytes(p);
    if (need == 0) return fail(RADSVD_ERR_UNSUPPORTED, "backward not available for this plan");
    if (!bwd_ws) return fail(RADSVD_ERR_WORKSPACE, "backward workspace is NULL");
    if (!aligned(bwd_ws, 256)) return fail(RADSVD_ERR_WORKSPACE, "backward workspace must be 256-byte aligned");
    if (bwd_bytes < need)
        return fail(RADSVD_ERR_WORKSPACE, "backward workspace too small: %zu < %zu", bwd_bytes, need);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = ensure_generic_layout(p, s);
    if (e == hipSuccess) e = launch_backward(p, inv_sigma2, lse_img, grad_lse_img, grad_B_polar, grad_U, bwd_ws, s);
    return dev_check(e, "align_pairs_backward launch");
}

size_t align_batched_workspace(int n_jobs) {
    g_err[0] = 0;
    if (n_jobs < 1 || n_jobs > 4096) {
        fail(RADSVD_ERR_INVALID_ARG, "n_jobs=%d outside [1, 4096]", n_jobs);
        return 0;
    }
    return batched_bytes(n_jobs);
}

}  // extern "C"

namespace {
radsvd_status validate_batch(const radsvd_plan *const *plans, int n_jobs, const radsvd_job_out *outs) {
    if (!plans || !outs) return fail(RADSVD_ERR_INVALID_ARG, "plans / outs is NULL");
    int prec = -1;
    for (int i = 0; i < n_jobs; ++i) {
        const radsvd_plan *p = plans[i];
        if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plans[%d] is NULL", i);
        if (!outs[i].best_score || !outs[i].best_m || !outs[i].best_t)
            return fail(RADSVD_ERR_INVALID_ARG, "outs[%d] has a NULL pointer", i);
        if (prec < 0) prec = p->prec;
        if (p->prec != prec) return fail(RADSVD_ERR_INVALID_ARG, "plans differ in precision");
        if (p->prec == RADSVD_BF16X3 && p->products != plans[0]->products)
            return fail(RADSVD_ERR_INVALID_ARG, "plans differ in the bf16x3 product count");
        if (!batched_supported(p))
            return fail(RADSVD_ERR_UNSUPPORTED,
                        "plans[%d]: the batched launch needs a Hermitian FP32/BF16/bf16x3 plan with "
                        "Q in {128, 192, 256, 384, 512} (got Q=%d)", i, p->Q);
    }
    return RADSVD_OK;
}
}  // namespace

extern "C" {

radsvd_status align_pairs_batched(const radsvd_plan *const *plans, int n_jobs, const radsvd_job_out *outs,
                                  void *batch_ws, size_t batch_bytes, void *stream) {
    g_err[0] = 0;
    if (n_jobs < 1 || n_jobs > 4096) return fail(RADSVD_ERR_INVALID_ARG, "n_jobs=%d outside [1, 4096]", n_jobs);
    const radsvd_status st = validate_batch(plans, n_jobs, outs);
    if (st != RADSVD_OK) return st;
    const size_t need = batched_bytes(n_jobs);
    if (!batch_ws) return fail(RADSVD_ERR_WORKSPACE, "batch workspace is NULL");
    if (!aligned(batch_ws, 256)) return fail(RADSVD_ERR_WORKSPACE, "batch workspace must be 256-byte aligned");
    if (batch_bytes < need) return fail(RADSVD_ERR_WORKSPACE, "batch workspace too small: %zu < %zu", batch_bytes, need);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return dev_check(launch_pairs_batched(plans, n_jobs, outs, batch_ws, s), "align_pairs_batched launch");
}

static_assert(RADSVD_NOALLOC_MAX_JOBS >= 1 && RADSVD_NOALLOC_MAX_JOBS <= 4096, "no-allocation job limit");

radsvd_status align_pairs_batched_noalloc(const radsvd_plan *const *plans, int n_jobs,
                                          const radsvd_job_out *outs, void *stream) {
    g_err[0] = 0;
    if (n_jobs < 1) return fail(RADSVD_ERR_INVALID_ARG, "n_jobs=%d must be >= 1", n_jobs);
    if (n_jobs > RADSVD_NOALLOC_MAX_JOBS || batched_bytes(n_jobs) > kNoAllocScratchBytes)
        return fail(RADSVD_ERR_UNSUPPORTED, "n_jobs=%d exceeds the no-allocation limit of %d jobs", n_jobs,
                    RADSVD_NOALLOC_MAX_JOBS);
    const radsvd_status st = validate_batch(plans, n_jobs, outs);
    if (st != RADSVD_OK) return st;
    void *ws = nullptr;
    const hipError_t e = noalloc_scratch(&ws);
    if (e != hipSuccess) return dev_check(e, "align_pairs_batched_noalloc scratch address");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return dev_check(launch_pairs_batched(plans, n_jobs, outs, ws, s), "align_pairs_batched_noalloc launch");
}

radsvd_status align_get_U(const radsvd_plan *p, double *U_dev, double *lambda_dev, void *stream) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (U_dev) e = hipMemcpyAsync(U_dev, p->U, (size_t)p->K * p->K * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && lambda_dev)
        e = hipMemcpyAsync(lambda_dev, p->lam, (size_t)p->K * 8, hipMemcpyDeviceToDevice, s);
    return dev_check(e, "align_get_U copy");
}

radsvd_status align_set_tile(radsvd_plan *p, int band) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    if (!fast_band_ok(band)) return fail(RADSVD_ERR_INVALID_ARG, "band=%d not one of 0, 1, 2, 4, 8, 16", band);
    p->band = band;
    return RADSVD_OK;
}

radsvd_status align_pairs_list(const radsvd_plan *p, int flags, float inv_sigma2, int n, const int32_t *pairs,
                               float *best_score, int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full,
                               void *stream) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    if (n < 1) return fail(RADSVD_ERR_INVALID_ARG, "n=%d must be >= 1", n);
    if (!pairs || !aligned(pairs, 4)) return fail(RADSVD_ERR_INVALID_ARG, "pairs must be non-NULL and 4-byte aligned");
    if (flags <= 0 || (flags & ~7)) return fail(RADSVD_ERR_INVALID_ARG, "out_flags=%d invalid", flags);
    if ((flags & RADSVD_OUT_BEST) && (!best_score || !best_m || !best_t))
        return fail(RADSVD_ERR_INVALID_ARG, "BEST output pointers must be non-NULL");
    if ((flags & RADSVD_OUT_LSE) && (!lse_pair || !(inv_sigma2 > 0.f && isfinite(inv_sigma2))))
        return fail(RADSVD_ERR_INVALID_ARG, "LSE needs lse_pair and a finite inv_sigma2 > 0");
    if ((flags & RADSVD_OUT_FULL) && !X_full) return fail(RADSVD_ERR_INVALID_ARG, "FULL output X_full must be non-NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = ensure_generic_layout(p, s);
    if (e == hipSuccess) e = launch_pairs_list(p, flags, inv_sigma2, n, pairs, best_score, best_m, best_t, lse_pair,
                                               X_full, s);
    return dev_check(e, "align_pairs_list launch");
}

radsvd_status align_top_targets(int n_img, int n_tgt, const float *score, int k, int32_t *cand, void *stream) {
    g_err[0] = 0;
    if (n_img < 1 || n_tgt < 1) return fail(RADSVD_ERR_INVALID_ARG, "n_img=%d, n_tgt=%d must be >= 1", n_img, n_tgt);
    if (k < 1 || k > kMaxTopK) return fail(RADSVD_ERR_INVALID_ARG, "k=%d outside [1, %d]", k, kMaxTopK);
    if (!score || !cand || !aligned(score, 4) || !aligned(cand, 4))
        return fail(RADSVD_ERR_INVALID_ARG, "score and cand must be non-NULL and 4-byte aligned");
    return dev_check(launch_top_targets(n_img, n_tgt, score, k, cand, reinterpret_cast<hipStream_t>(stream)),
                     "align_top_targets launch");
}

radsvd_status align_landscape_metrics(long long n_pairs, int len, const void *X_est, const void *X_ref, int fp64,
                                      float *f, double *pair_stats, double *summary, void *stream) {
    g_err[0] = 0;
    if (n_pairs < 1 || len < 1) return fail(RADSVD_ERR_INVALID_ARG, "n_pairs and len must be >= 1");
    if (fp64 != 0 && fp64 != 1) return fail(RADSVD_ERR_INVALID_ARG, "fp64 must be 0 or 1");
    if (!X_est || !X_ref || !f || !pair_stats || !summary)
        return fail(RADSVD_ERR_INVALID_ARG, "arrays must be non-NULL");
    const size_t al = fp64 ? 16 : 8;
    if (!aligned(X_est, al) || !aligned(X_ref, al) || !aligned(f, 4) || !aligned(pair_stats, 8) || !aligned(summary, 8))
        return fail(RADSVD_ERR_INVALID_ARG, "misaligned array");
    return dev_check(launch_landscape_metrics(n_pairs, len, X_est, X_ref, fp64, f, pair_stats, summary,
                                              reinterpret_cast<hipStream_t>(stream)),
                     "align_landscape_metrics launch");
}

radsvd_status align_refine_rotation(const radsvd_plan *p, const int32_t *best_m, const int32_t *best_t, int R,
                                    float *fine_score, int32_t *fine_m, void *stream) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    if (!best_m || !best_t || !fine_score || !fine_m)
        return fail(RADSVD_ERR_INVALID_ARG, "best_m, best_t, fine_score and fine_m must be non-NULL");
    if (!aligned(best_m, 4) || !aligned(best_t, 4) || !aligned(fine_score, 4) || !aligned(fine_m, 4))
        return fail(RADSVD_ERR_INVALID_ARG, "arrays must be 4-byte aligned");
    if (R < 1 || R > kMaxRefine) return fail(RADSVD_ERR_INVALID_ARG, "R=%d outside [1, %d]", R, kMaxRefine);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = ensure_generic_layout(p, s);
    if (e == hipSuccess) e = launch_refine_rotation(p, best_m, best_t, R, fine_score, fine_m, s);
    return dev_check(e, "align_refine_rotation launch");
}

radsvd_status align_set_waves(radsvd_plan *p, int waves) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    if (waves != 0 && waves != 4 && waves != 8) return fail(RADSVD_ERR_INVALID_ARG, "waves=%d not one of 0, 4, 8", waves);
    if (!fast_waves_ok(p, waves))
        return fail(RADSVD_ERR_UNSUPPORTED, "waves=%d: not available for this plan (Q=%d, H8=%d)", waves, p->Q, p->H8);
    p->waves = waves;
    return RADSVD_OK;
}

void align_plan_destroy(radsvd_plan *p) { delete p; }

}  // extern "C"

// ---------------------------------------------------------------------------
// volume alignment (paper section 4)
// ---------------------------------------------------------------------------
namespace {

int vol_max_L(radsvd_precision prec) { return prec == RADSVD_FP64 ? kVolMaxL64 : kVolMaxL32; }

radsvd_status validate_vol(const radsvd_vol_problem *pr) {
    if (!pr) return fail(RADSVD_ERR_INVALID_ARG, "problem is NULL");
    if (pr->prec != RADSVD_FP64 && pr->prec != RADSVD_FP32)
        return fail(RADSVD_ERR_INVALID_ARG, "prec=%d: volume plans take RADSVD_FP64 or RADSVD_FP32", pr->prec);
    if (pr->K < 2 || pr->K > kVolMaxK) return fail(RADSVD_ERR_INVALID_ARG, "K=%d outside [2, %d]", pr->K, kVolMaxK);
    const int lmax = vol_max_L(pr->prec);
    if (pr->L < 1 || pr->L > lmax) return fail(RADSVD_ERR_INVALID_ARG, "L=%d outside [1, %d]", pr->L, lmax);
    if (pr->H_C < 1 || pr->H_C > pr->K) return fail(RADSVD_ERR_INVALID_ARG, "H_C=%d outside [1, %d]", pr->H_C, pr->K);
    if (pr->H_D < 1 || pr->H_D > pr->L + 1)
        return fail(RADSVD_ERR_INVALID_ARG, "H_D=%d outside [1, %d]", pr->H_D, pr->L + 1);
    if (pr->n_beta < 1 || pr->n_beta > kVolMaxBeta)
        return fail(RADSVD_ERR_INVALID_ARG, "n_beta=%d outside [1, %d]", pr->n_beta, kVolMaxBeta);
    if (!pr->w || !pr->beta) return fail(RADSVD_ERR_INVALID_ARG, "w or beta is NULL");
    for (int r = 0; r < pr->K; ++r)
        if (!(pr->w[r] > 0.0) || !isfinite(pr->w[r]))
            return fail(RADSVD_ERR_INVALID_ARG, "w[%d] must be finite and > 0", r);
    for (int i = 0; i < pr->n_beta; ++i)
        if (!isfinite(pr->beta[i])) return fail(RADSVD_ERR_INVALID_ARG, "beta[%d] not finite", i);
    if (pr->real_volumes != 0 && pr->real_volumes != 1)
        return fail(RADSVD_ERR_INVALID_ARG, "real_volumes must be 0 or 1");
    return RADSVD_OK;
}

radsvd_status validate_vol_counts(int n_vol, int n_tgt) {
    if (n_vol < 1 || n_vol > (1 << 20) || n_tgt < 1 || n_tgt > (1 << 20))
        return fail(RADSVD_ERR_INVALID_ARG, "n_vol=%d / n_tgt=%d outside [1, 2^20]", n_vol, n_tgt);
    if ((long long)n_vol * n_tgt > (1LL << 31))
        return fail(RADSVD_ERR_INVALID_ARG, "n_vol * n_tgt = %lld above 2^31", (long long)n_vol * n_tgt);
    return RADSVD_OK;
}

struct VolLayout {
    size_t off_w, off_beta, off_C, off_U, off_lamC, off_logC, off_D, off_V, off_lamD, off_logD, off_As, off_Bs,
        off_Vd, off_Xt, off_Y, off_Xh, off_pv, off_pi, total;
    int chunk;
};

VolLayout make_vol_layout(const radsvd_vol_problem *pr, int n_vol, int n_tgt) {
    VolLayout Lo{};
    const size_t R = pr->prec == RADSVD_FP64 ? 8 : 4, CX = 2 * R;
    const int K = pr->K, L1 = pr->L + 1, M = 2 * pr->L + 1, NC = L1 * L1;
    const size_t MM = (size_t)M * M;
    const long long n_pairs = (long long)n_vol * n_tgt;
    const long long L1l = L1;
    const size_t nxt = (size_t)(L1l * (2 * L1l - 1) * (2 * L1l + 1) / 3);   // sum_{l <= L} (2l+1)^2
    const size_t per_pair = ((size_t)pr->H_D * MM + nxt + (size_t)pr->n_beta * MM) * CX;
    long long chunk = (long long)(kVolChunkBytes / per_pair);
    chunk = std::max<long long>(1, std::min<long long>(chunk, kVolMaxChunk));
    chunk = std::min(chunk, n_pairs);
    Lo.chunk = (int)chunk;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    Lo.off_w = take(K * 8);
    Lo.off_beta = take((size_t)pr->n_beta * 8);
    Lo.off_C = take((size_t)K * K * 8);
    Lo.off_U = take((size_t)K * K * 8);
    Lo.off_lamC = take(K * 8);
    Lo.off_logC = take(eig_log_bytes(K));
    Lo.off_D = take((size_t)L1 * L1 * 8);
    Lo.off_V = take((size_t)L1 * L1 * 8);
    Lo.off_lamD = take(L1 * 8);
    Lo.off_logD = take(eig_log_bytes(L1));
    Lo.off_As = take((size_t)n_vol * pr->H_C * NC * CX);
    Lo.off_Bs = take((size_t)n_tgt * pr->H_C * NC * CX);
    Lo.off_Vd = take((size_t)pr->n_beta * pr->H_D * MM * R);
    Lo.off_Xt = take((size_t)chunk * nxt * CX);
    Lo.off_Y = take((size_t)chunk * pr->H_D * MM * CX);
    Lo.off_Xh = take((size_t)chunk * pr->n_beta * MM * CX);
    Lo.off_pv = take((size_t)chunk * pr->n_beta * 8);
    Lo.off_pi = take((size_t)chunk * pr->n_beta * 4);
    Lo.total = off;
    return Lo;
}

}  // namespace

extern "C" {

size_t vol_prepare_workspace(const radsvd_vol_problem *prob, int n_vol, int n_tgt) {
    g_err[0] = 0;
    if (validate_vol(prob) != RADSVD_OK || validate_vol_counts(n_vol, n_tgt) != RADSVD_OK) return 0;
    return make_vol_layout(prob, n_vol, n_tgt).total;
}

radsvd_status vol_prepare(const radsvd_vol_problem *prob, int n_vol, const void *A_sh, int n_tgt, const void *B_sh,
                          const double *U_in, const double *V_in, void *ws, size_t ws_bytes, void *stream,
                          radsvd_vol_plan **out) {
    g_err[0] = 0;
    radsvd_status st = validate_vol(prob);
    if (st != RADSVD_OK) return st;
    if (!out) return fail(RADSVD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    st = validate_vol_counts(n_vol, n_tgt);
    if (st != RADSVD_OK) return st;
    if (!A_sh || !B_sh) return fail(RADSVD_ERR_INVALID_ARG, "A_sh or B_sh is NULL");
    if (!aligned(A_sh, 16) || !aligned(B_sh, 16))
        return fail(RADSVD_ERR_INVALID_ARG, "A_sh / B_sh must be 16-byte aligned");
    if ((U_in && !aligned(U_in, 8)) || (V_in && !aligned(V_in, 8)))
        return fail(RADSVD_ERR_INVALID_ARG, "U_in / V_in must be 8-byte aligned");
    const VolLayout Lo = make_vol_layout(prob, n_vol, n_tgt);
    if (!ws) return fail(RADSVD_ERR_WORKSPACE, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(RADSVD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < Lo.total)
        return fail(RADSVD_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, Lo.total);
    radsvd_vol_plan *p = new (std::nothrow) radsvd_vol_plan();
    if (!p) return fail(RADSVD_ERR_DEVICE, "host allocation failed");
    p->K = prob->K;
    p->L = prob->L;
    p->M = 2 * prob->L + 1;
    p->NC = (prob->L + 1) * (prob->L + 1);
    p->HC = prob->H_C;
    p->HD = prob->H_D;
    p->n_beta = prob->n_beta;
    p->prec = prob->prec;
    p->n_vol = n_vol;
    p->n_tgt = n_tgt;
    p->chunk = Lo.chunk;
    p->user_U = U_in != nullptr;
    p->user_V = V_in != nullptr;
    p->real = prob->real_volumes;
    p->ws = reinterpret_cast<char *>(ws);
    p->ws_bytes = ws_bytes;
    char *w = p->ws;
    p->w = reinterpret_cast<double *>(w + Lo.off_w);
    p->beta = reinterpret_cast<double *>(w + Lo.off_beta);
    p->C = reinterpret_cast<double *>(w + Lo.off_C);
    p->U = reinterpret_cast<double *>(w + Lo.off_U);
    p->lamC = reinterpret_cast<double *>(w + Lo.off_lamC);
    p->logC = w + Lo.off_logC;
    p->D = reinterpret_cast<double *>(w + Lo.off_D);
    p->V = reinterpret_cast<double *>(w + Lo.off_V);
    p->lamD = reinterpret_cast<double *>(w + Lo.off_lamD);
    p->logD = w + Lo.off_logD;
    p->As = w + Lo.off_As;
    p->Bs = w + Lo.off_Bs;
    p->Vd = w + Lo.off_Vd;
    p->Xt = w + Lo.off_Xt;
    p->Y = w + Lo.off_Y;
    p->Xh = w + Lo.off_Xh;
    p->part_val = reinterpret_cast<double *>(w + Lo.off_pv);
    p->part_idx = reinterpret_cast<int32_t *>(w + Lo.off_pi);
    VolGrid g;
    memset(&g, 0, sizeof(g));
    g.K = prob->K;
    g.n_beta = prob->n_beta;
    for (int r = 0; r < prob->K; ++r) g.w[r] = prob->w[r];
    for (int i = 0; i < prob->n_beta; ++i) g.beta[i] = prob->beta[i];
    const hipError_t e = vol_launch_prepare(p, g, A_sh, B_sh, U_in, V_in, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        delete p;
        return dev_check(e, "vol_prepare launch");
    }
    *out = p;
    return RADSVD_OK;
}

radsvd_status vol_align(const radsvd_vol_plan *p, int flags, float *best_score, int32_t *best_idx, void *X_full,
                        void *stream) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    if (flags <= 0 || (flags & ~(RADSVD_OUT_BEST | RADSVD_OUT_FULL)))
        return fail(RADSVD_ERR_INVALID_ARG, "out_flags=%d invalid (RADSVD_OUT_BEST and/or RADSVD_OUT_FULL)", flags);
    if ((flags & RADSVD_OUT_BEST) && (!best_score || !best_idx))
        return fail(RADSVD_ERR_INVALID_ARG, "BEST output pointers must be non-NULL");
    if ((flags & RADSVD_OUT_BEST) && (!aligned(best_score, 4) || !aligned(best_idx, 4)))
        return fail(RADSVD_ERR_INVALID_ARG, "BEST outputs must be 4-byte aligned");
    if ((flags & RADSVD_OUT_FULL) && !X_full) return fail(RADSVD_ERR_INVALID_ARG, "FULL output X_full must be non-NULL");
    if ((flags & RADSVD_OUT_FULL) && !aligned(X_full, p->prec == RADSVD_FP64 ? 16 : 8))
        return fail(RADSVD_ERR_INVALID_ARG, "X_full misaligned");
    const hipError_t e = vol_launch_align(p, flags, (flags & RADSVD_OUT_BEST) ? best_score : nullptr,
                                          (flags & RADSVD_OUT_BEST) ? best_idx : nullptr, X_full,
                                          reinterpret_cast<hipStream_t>(stream));
    return dev_check(e, "vol_align launch");
}

radsvd_status vol_get_UV(const radsvd_vol_plan *p, double *U_dev, double *lamC_dev, double *V_dev, double *lamD_dev,
                         void *stream) {
    g_err[0] = 0;
    if (!p) return fail(RADSVD_ERR_INVALID_ARG, "plan is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t L1 = p->L + 1;
    hipError_t e = hipSuccess;
    if (U_dev) e = hipMemcpyAsync(U_dev, p->U, (size_t)p->K * p->K * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && lamC_dev) e = hipMemcpyAsync(lamC_dev, p->lamC, (size_t)p->K * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && V_dev) e = hipMemcpyAsync(V_dev, p->V, L1 * L1 * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && lamD_dev) e = hipMemcpyAsync(lamD_dev, p->lamD, L1 * 8, hipMemcpyDeviceToDevice, s);
    return dev_check(e, "vol_get_UV copy");
}

void vol_plan_destroy(radsvd_vol_plan *p) { delete p; }

}  // extern "C"
