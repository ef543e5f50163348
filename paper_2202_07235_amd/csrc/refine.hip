// Rotations off the polar grid (paper section 2.2: a rotation by any gamma is
// the phase exp(-i q gamma) on the Fourier-Bessel coefficients; section 2.4:
// finer gamma by zero-padding the frequency array before the transform over
// q).  For each pair, at the translation of its best grid rotation m, the
// landscape is evaluated at gamma = 2 pi (R m + j) / (R Q), |j| < R: the
// zero-padded (length R Q) transform restricted to one grid step on either
// side of the grid maximum.  Frequencies are taken in the band |q| <= Q/2
// with the q = Q/2 term as a cosine, so that grid rotations reproduce the
// landscape exactly.
//
// One wavefront per pair.  Lane l holds S[q] = sum_h conj(At[a][h][q]) Bt[b][t][h][q]
// for q = l, l + 64, ... (generic operand layout [item][h][q], so a wave's loads
// of one rank are contiguous); each candidate rotation
// is a lane-local partial sum over those q and one cross-lane reduction.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace radsvd {

template <typename R>
__device__ __forceinline__ void sincos_2pi_frac(long long n, long long den, R &s, R &c) {
    // angle 2 pi n / den with n reduced to [0, den) first: exact argument reduction
    n %= den;
    if (n < 0) n += den;
    if constexpr (sizeof(R) == 8) {
        sincospi(2.0 * (double)n / (double)den, &s, &c);
    } else {
        sincospif(2.0f * (float)((double)n / (double)den), &s, &c);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_refine_rotation(const cx<R> *__restrict__ Ag, const cx<R> *__restrict__ Bg,
                                                         int n_img, int n_tgt, int T, int H, int Q, int Qc, int herm,
                                                         const int32_t *__restrict__ best_m,
                                                         const int32_t *__restrict__ best_t, int Rf,
                                                         float *__restrict__ fine_score, int32_t *__restrict__ fine_m) {
    constexpr int MAXQ = kMaxQ / 64;   // frequencies per lane
    const int lane = threadIdx.x & 63;
    const long long n_pairs = (long long)n_img * n_tgt;
    const int M = Q / 2;
    const long long den = (long long)Rf * Q;
    for (long long pair = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); pair < n_pairs;
         pair += (long long)gridDim.x * 4) {
        const int a = (int)(pair / n_tgt), b = (int)(pair - (long long)a * n_tgt);
        const int m = best_m[pair], t = best_t[pair];
        if (m < 0 || m >= Q || t < 0 || t >= T) {   // a pair without a best (non-finite landscape)
            if (lane == 0) {
                fine_score[pair] = NAN;
                fine_m[pair] = -1;
            }
            continue;
        }
        const cx<R> *Aa = Ag + (size_t)a * Qc * H;
        const cx<R> *Bb = Bg + ((size_t)b * T + t) * Qc * H;
        cx<R> S[MAXQ];
#pragma unroll
        for (int i = 0; i < MAXQ; ++i) {
            const int q = lane + 64 * i;
            R re = 0, im = 0;
            if (q < Qc) {
                const cx<R> *x = Aa + q;   // rank h at x[h * Qc]
                const cx<R> *y = Bb + q;
                for (int h = 0; h < H; ++h) {
                    const cx<R> u = x[(size_t)h * Qc], v = y[(size_t)h * Qc];
                    re += u.re * v.re + u.im * v.im;
                    im += u.re * v.im - u.im * v.re;
                }
            }
            S[i] = cx<R>{re, im};
        }
        float bestv = -INFINITY;
        int bestj = 0;
        bool bad = false;
        for (int j = -Rf + 1; j < Rf; ++j) {
            const long long nfine = (long long)Rf * m + j;   // gamma = 2 pi nfine / (R Q)
            R part = 0;
#pragma unroll
            for (int i = 0; i < MAXQ; ++i) {
                const int q = lane + 64 * i;
                if (q >= Qc) continue;
                R s, c;
                if (q == M) {   // the Nyquist term: its cosine (real part of S[M])
                    sincos_2pi_frac<R>((long long)M * nfine, den, s, c);
                    part += S[i].re * c;
                    continue;
                }
                // symmetric representative of q; Hermitian plans store q in [0, M]
                // and the conjugate half doubles the terms 0 < q < M
                const long long qs = (herm || q < M) ? q : (long long)q - Q;
                sincos_2pi_frac<R>(qs * nfine, den, s, c);
                const R term = S[i].re * c + S[i].im * s;   // Re(exp(-i qs gamma) S[q])
                part += (herm && q > 0) ? 2 * term : term;
            }
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
            const float v = (float)part;
            if (!isfinite(v)) bad = true;
            if (v > bestv) {   // strict: ties keep the smaller j
                bestv = v;
                bestj = j;
            }
        }
        if (lane == 0) {
            if (bad) {
                fine_score[pair] = NAN;
                fine_m[pair] = -1;
            } else {
                long long f = ((long long)Rf * m + bestj) % den;
                if (f < 0) f += den;
                fine_score[pair] = bestv;
                fine_m[pair] = (int32_t)f;
            }
        }
    }
}

hipError_t launch_refine_rotation(const radsvd_plan *p, const int32_t *best_m, const int32_t *best_t, int Rf,
                                  float *fine_score, int32_t *fine_m, hipStream_t s) {
    const long long n_pairs = (long long)p->n_img * p->n_tgt;
    const int blocks = (int)std::min<long long>((n_pairs + 3) / 4, 1 << 20);
    if (p->prec == RADSVD_FP64)
        hipLaunchKernelGGL(k_refine_rotation<double>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const cx<double> *>(p->Ag), reinterpret_cast<const cx<double> *>(p->Bg),
                           p->n_img, p->n_tgt, p->T, p->H, p->Q, p->Qc, p->herm, best_m, best_t, Rf, fine_score,
                           fine_m);
    else
        hipLaunchKernelGGL(k_refine_rotation<float>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const cx<float> *>(p->Ag), reinterpret_cast<const cx<float> *>(p->Bg),
                           p->n_img, p->n_tgt, p->T, p->H, p->Q, p->Qc, p->herm, best_m, best_t, Rf, fine_score,
                           fine_m);
    return hipGetLastError();
}

}  // namespace radsvd
