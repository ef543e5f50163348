// Generic per-pair kernel: any precision, Hermitian or not, every output mode.
// One workgroup per pair (a, b); for each translation t:
//   Step 1 (paper section 3.3): S[q] = sum_h conj(At[a][q][h]) * Bt[b][t][q][h]
//          for the stored frequencies (all Q, or q in [0, Q/2] for Hermitian
//          inputs, the rest following from S[Q-q] = conj(S[q]));
//   Step 2: X[m] = sum_q S[q] exp(-2 pi i q m / Q), an in-LDS FFT;
//   epilogue: running best (ties -> smallest t*Q+m, NaN wins), running
//   log-sum-exp, or the full landscape.
// The split-precision modes reproduce the arithmetic of the matrix-core path
// (bf16 operand terms, exact bf16 x bf16 products, FP32 accumulation).
#include <math.h>

#include "common.h"
#include "internal.h"

namespace radsvd {

template <int PREC>
__device__ __forceinline__ void contract_term(const cx<float> &a, const cx<float> &b, int products,
                                              float &re, float &im) {
    // re += ar*br + ai*bi ; im += ar*bi - ai*br   (conj(a) * b)
    if (PREC == RADSVD_FP32) {
        re = fmaf(a.re, b.re, re);
        re = fmaf(a.im, b.im, re);
        im = fmaf(a.re, b.im, im);
        im = fmaf(-a.im, b.re, im);
    } else {
        uint16_t ar[3], ai[3], br[3], bi[3];
        split3_bf16(a.re, ar[0], ar[1], ar[2]);
        split3_bf16(a.im, ai[0], ai[1], ai[2]);
        split3_bf16(b.re, br[0], br[1], br[2]);
        split3_bf16(b.im, bi[0], bi[1], bi[2]);
        // (i, j) term pairs of the split products
        const int np = (PREC == RADSVD_BF16) ? 1 : products;
        const int pi_[6] = {0, 0, 1, 1, 0, 2};
        const int pj_[6] = {0, 1, 0, 1, 2, 0};
        for (int u = 0; u < np; ++u) {
            const float xr = bf16_to_f32(ar[pi_[u]]), xi = bf16_to_f32(ai[pi_[u]]);
            const float yr = bf16_to_f32(br[pj_[u]]), yi = bf16_to_f32(bi[pj_[u]]);
            re = fmaf(xr, yr, re);
            re = fmaf(xi, yi, re);
            im = fmaf(xr, yi, im);
            im = fmaf(-xi, yr, im);
        }
    }
}

struct BestAcc {
    float v;
    int idx;
};
__device__ __forceinline__ bool better(float v1, int i1, float v2, int i2) {
    const bool n1 = isnan(v1), n2 = isnan(v2);
    if (n1 != n2) return n1;
    if (!n1 && v1 != v2) return v1 > v2;
    return i1 < i2;
}

template <typename R, int PREC>
__global__ __launch_bounds__(256) void k_pairs_generic(
    const cx<R> *__restrict__ Ag, const cx<R> *__restrict__ Bg, int n_img, int n_tgt, int T, int H,
    int Q, int Qc, int herm, int products, int flags, float inv_s2, float *__restrict__ best_score,
    int32_t *__restrict__ best_m, int32_t *__restrict__ best_t, float *__restrict__ lse_pair,
    cx<R> *__restrict__ Xfull, const int32_t *__restrict__ plist) {
    extern __shared__ unsigned char smem_raw[];
    cx<R> *tw = reinterpret_cast<cx<R> *>(smem_raw);
    cx<R> *S = tw + Q;
    __shared__ float rv[4];
    __shared__ int ri[4];
    __shared__ float rs[4];
    // grid mode: pair (blockIdx.y, blockIdx.x), outputs [n_img][n_tgt]; list mode:
    // pair plist[2 i], plist[2 i + 1], outputs at list position i
    const size_t o = plist ? (size_t)blockIdx.x : (size_t)blockIdx.y * n_tgt + blockIdx.x;
    const int a = plist ? plist[2 * o] : (int)blockIdx.y, b = plist ? plist[2 * o + 1] : (int)blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (a < 0 || a >= n_img || b < 0 || b >= n_tgt) {   // a list entry outside the plan (uniform per workgroup)
        if (tid == 0) {
            if (flags & RADSVD_OUT_BEST) {
                best_score[o] = NAN;
                best_m[o] = -1;
                best_t[o] = -1;
            }
            if (flags & RADSVD_OUT_LSE) lse_pair[o] = NAN;
        }
        return;
    }
    const int lane = tid & 63, wid = tid >> 6;
    for (int i = tid; i < Q; i += nt) {
        double s, c;
        sincospi(-2.0 * (double)i / (double)Q, &s, &c);
        tw[i] = cx<R>{(R)c, (R)s};
    }
    __shared__ FftPlan spl;   // in LDS: the FFT stage loops index it at run time
    if (threadIdx.x == 0) fft_init_plan(spl, Q);
    __syncthreads();
    const FftPlan &pl = spl;
    const int M = Q / 2;
    float best_v = 0.f;
    int best_i = 0x7fffffff;
    bool have_best = false;
    float lse_m = -INFINITY, lse_s = 0.f;
    bool lse_nan = false;
    const cx<R> *Aa = Ag + (size_t)a * Qc * H;
    for (int t = 0; t < T; ++t) {
        const cx<R> *Bb = Bg + ((size_t)b * T + t) * Qc * H;
        __syncthreads();
        for (int q = tid; q < Qc; q += nt) {
            const cx<R> *x = Aa + q;   // rank h at x[h * Qc]
            const cx<R> *y = Bb + q;
            cx<R> acc;
            if (PREC == RADSVD_FP64) {
                R re = 0, im = 0;
                for (int h = 0; h < H; ++h) {
                    const cx<R> u = x[(size_t)h * Qc], v = y[(size_t)h * Qc];
                    re += u.re * v.re + u.im * v.im;
                    im += u.re * v.im - u.im * v.re;
                }
                acc = cx<R>{re, im};
            } else {
                float re = 0.f, im = 0.f;
                for (int h = 0; h < H; ++h) {
                    const cx<R> u = x[(size_t)h * Qc], v = y[(size_t)h * Qc];
                    cx<float> xf = {(float)u.re, (float)u.im};
                    cx<float> yf = {(float)v.re, (float)v.im};
                    contract_term<PREC>(xf, yf, products, re, im);
                }
                acc = cx<R>{(R)re, (R)im};
            }
            if (herm) {
                if (q == 0 || q == M) acc.im = (R)0;
                S[q] = acc;
                if (q > 0 && q < M) S[Q - q] = cconj(acc);
            } else {
                S[q] = acc;
            }
        }
        __syncthreads();
        lds_fft_dif(S, 1, Q, pl, tw);
        // epilogue
        if (flags & RADSVD_OUT_FULL) {
            cx<R> *Xo = Xfull + (o * T + t) * Q;
            for (int m = tid; m < Q; m += nt) Xo[m] = S[fft_pos(m, pl)];
        }
        if (flags & RADSVD_OUT_BEST) {
            // threads without a value must never win: -inf with the largest index
            float v = -INFINITY;
            int idx = 0x7fffffff;
            bool any = false;
            for (int m = tid; m < Q; m += nt) {
                // a non-finite value counts as NaN, which wins every comparison
                const float xs = (float)S[fft_pos(m, pl)].re;
                const float x = isfinite(xs) ? xs : NAN;
                const int id = t * Q + m;
                if (!any || better(x, id, v, idx)) {
                    v = x;
                    idx = id;
                    any = true;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const float v2 = __shfl_xor(v, o, 64);
                const int i2 = __shfl_xor(idx, o, 64);
                if (better(v2, i2, v, idx)) {
                    v = v2;
                    idx = i2;
                }
            }
            if (lane == 0) {
                rv[wid] = v;
                ri[wid] = idx;
            }
            __syncthreads();
            if (tid == 0) {
                float bv = rv[0];
                int bi = ri[0];
                for (int w = 1; w < (nt >> 6); ++w)
                    if (better(rv[w], ri[w], bv, bi)) {
                        bv = rv[w];
                        bi = ri[w];
                    }
                if (!have_best || better(bv, bi, best_v, best_i)) {
                    best_v = bv;
                    best_i = bi;
                }
                have_best = true;
            }
            __syncthreads();
        }
        if (flags & RADSVD_OUT_LSE) {
            float mx = -INFINITY;
            bool nan_seen = false;
            for (int m = tid; m < Q; m += nt) {
                const float xs = (float)S[fft_pos(m, pl)].re;
                const float x = xs * inv_s2;
                if (!isfinite(xs)) nan_seen = true;
                else mx = fmaxf(mx, x);
            }
            for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
            if (lane == 0) rv[wid] = mx;
            const int anynan = __syncthreads_or(nan_seen ? 1 : 0);
            float bmx = rv[0];
            for (int w = 1; w < (nt >> 6); ++w) bmx = fmaxf(bmx, rv[w]);
            float sum = 0.f;
            for (int m = tid; m < Q; m += nt) {
                const float xs = (float)S[fft_pos(m, pl)].re;
                if (isfinite(xs)) sum += expf(xs * inv_s2 - bmx);
            }
            for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
            __syncthreads();
            if (lane == 0) rs[wid] = sum;
            __syncthreads();
            if (tid == 0) {
                float tot = 0.f;
                for (int w = 0; w < (nt >> 6); ++w) tot += rs[w];
                if (anynan) lse_nan = true;
                const float nm = fmaxf(lse_m, bmx);
                if (nm == -INFINITY) {
                    lse_s = 0.f;
                } else {
                    lse_s = lse_s * expf(lse_m - nm) + tot * expf(bmx - nm);
                }
                lse_m = nm;
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        if (flags & RADSVD_OUT_BEST) {
            if (isnan(best_v)) {
                best_score[o] = NAN;
                best_m[o] = -1;
                best_t[o] = -1;
            } else {
                best_score[o] = best_v;
                best_m[o] = best_i % Q;
                best_t[o] = best_i / Q;
            }
        }
        if (flags & RADSVD_OUT_LSE) lse_pair[o] = lse_nan ? NAN : lse_m + logf(lse_s);
    }
}

template <typename R, int PREC>
static void launch_g(const radsvd_plan *p, int flags, float inv_s2, float *bs, int32_t *bm,
                     int32_t *bt, float *lp, void *Xf, int n_list, const int32_t *plist, hipStream_t s) {
    const size_t shmem = 2 * (size_t)p->Q * sizeof(cx<R>);
    const dim3 grid = plist ? dim3(n_list) : dim3(p->n_tgt, p->n_img);
    hipLaunchKernelGGL((k_pairs_generic<R, PREC>), grid, dim3(256), shmem, s,
                       reinterpret_cast<const cx<R> *>(p->Ag), reinterpret_cast<const cx<R> *>(p->Bg),
                       p->n_img, p->n_tgt, p->T, p->H, p->Q, p->Qc, p->herm, p->products, flags, inv_s2,
                       bs, bm, bt, lp, reinterpret_cast<cx<R> *>(Xf), plist);
}

static hipError_t launch_generic_any(const radsvd_plan *p, int flags, float inv_s2, float *best_score,
                                     int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full, int n_list,
                                     const int32_t *plist, hipStream_t s) {
    switch (p->prec) {
    case RADSVD_FP64:
        launch_g<double, RADSVD_FP64>(p, flags, inv_s2, best_score, best_m, best_t, lse_pair, X_full, n_list,
                                      plist, s);
        break;
    case RADSVD_FP32:
        launch_g<float, RADSVD_FP32>(p, flags, inv_s2, best_score, best_m, best_t, lse_pair, X_full, n_list,
                                     plist, s);
        break;
    case RADSVD_BF16:
        launch_g<float, RADSVD_BF16>(p, flags, inv_s2, best_score, best_m, best_t, lse_pair, X_full, n_list,
                                     plist, s);
        break;
    default:
        launch_g<float, RADSVD_BF16X3>(p, flags, inv_s2, best_score, best_m, best_t, lse_pair, X_full, n_list,
                                       plist, s);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_pairs_generic(const radsvd_plan *p, int flags, float inv_s2, float *best_score,
                                int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full,
                                hipStream_t s) {
    return launch_generic_any(p, flags, inv_s2, best_score, best_m, best_t, lse_pair, X_full, 0, nullptr, s);
}

hipError_t launch_pairs_list(const radsvd_plan *p, int flags, float inv_s2, int n, const int32_t *pairs,
                             float *best_score, int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full,
                             hipStream_t s) {
    return launch_generic_any(p, flags, inv_s2, best_score, best_m, best_t, lse_pair, X_full, n, pairs, s);
}

}  // namespace radsvd
