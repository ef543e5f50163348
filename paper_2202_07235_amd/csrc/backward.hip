// Backward pass of the soft-alignment loss L = sum_a g[a] lse_img[a], with
// lse_img[a] = log sum_b exp(lse_pair[a][b]) and lse_pair[a][b] =
// log sum_{t,m} exp(s Re X[a][b][t][m]) (s = inv_sigma2): the Gaussian
// log-likelihood of paper section 2.6 marginalised over the alignments.
//
// With P[a,b,t,m] = dL/dRe X = g[a] s exp(s Re X - lse_img[a]) and the unitary
// angular coefficients at, bt of the principal rings (X[m] = sum_q W^{qm}
// sum_h conj(at[h,q]) bt[h,q], W = exp(-2 pi i / Q)):
//   Phat[q]        = sum_m P[m] exp(+2 pi i q m / Q)
//   g_bt[b,t,h,q]  = sum_a at[a,h,q] Phat[a,b,t,q]
//   g_at[a,h,q]    = sum_{b,t} conj(Phat[a,b,t,q]) bt[b,t,h,q]
// back to psi-space by the adjoint (inverse) unitary transform, then through
// the recombination Br_h^t = sum_r U[r,h] eta_r phi_t[r,.] Bhat[r,.]:
//   dL/dBhat[b,r,j] = eta_r sum_t conj(phi_t[r,j]) sum_h U[r,h] g_Br[b,t,h,j]
//   dL/dU[r,h]      = sum Re(conj(g_Ar[a,h,j]) eta_r Ahat[a,r,j])
//                   + sum Re(conj(g_Br[b,t,h,j]) eta_r phi_t[r,j] Bhat[b,r,j])
// (complex gradients: dL/dRe + i dL/dIm; U is a free real matrix).
//
// For Hermitian inputs only q in [0, Q/2] is stored; the other half follows
// from Phat[Q-q] = conj Phat[q] and at, bt, g_at, g_bt[Q-q] = (-1)^q conj(.[q]).
// Every step runs in FP64; images are processed in chunks so that the Phat
// buffer stays within a fixed budget.  All reductions have a fixed order.
// The forward's lse_img (FP32) only serves as the exponent shift c_a: the
// kernel forms Pt = exp(s Re X - c_a) and the per-pair sums of Pt, and the
// exact normalisation g[a] s exp(c_a - lse_img[a]) = g[a] s / sum_{b,t,m} Pt
// is applied as a per-image factor kappa[a] in the contractions.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace radsvd {

namespace {

constexpr size_t kPhatBudget = size_t(4) << 30;   // bytes of Phat per image chunk

struct BwdLayout {
    int chunk;   // images per chunk
    size_t off_phat, off_sum, off_kappa, off_gBt, off_gAt, off_gApart, off_gBpsi, off_gApsi, off_ph64, off_part,
        total;
};

// tiles of the per-frequency contractions (k_bwd_gBt, k_bwd_gAt)
constexpr int kGbCB = 2, kGbAT = 8, kGaCB = 4, kGaAT = 8;

// spans of columns of the g_at contraction: enough workgroups to fill the chip,
// each span at least 256 columns (so the partials stay below Phat / 8)
int gat_max_split(size_t NBT) { return (int)std::max<size_t>(1, std::min<size_t>(8, NBT / 256)); }

int gat_span(int ca, int Qs, int NBT) {
    const int nwg = ((ca + 64 * kGaCB - 1) / (64 * kGaCB)) * Qs;   // the g_at kernel's images per workgroup
    const int ns = std::max(1, std::min(gat_max_split(NBT), (4096 + nwg - 1) / nwg));
    return ((NBT + ns - 1) / ns + 15) / 16 * 16;
}

BwdLayout bwd_layout(const radsvd_plan *p) {
    const size_t Qs = p->Qc, T = p->T, H = p->H, K = p->K, Q = p->Q;
    const size_t na = p->n_img, nb = p->n_tgt, NBT = nb * T;
    BwdLayout L{};
    const size_t per_img = Qs * NBT * sizeof(cx<double>);
    size_t ch = kPhatBudget / per_img;
    if (ch < 1) ch = 1;
    if (ch > na) ch = na;
    if (ch > 65535) ch = 65535;
    L.chunk = (int)ch;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = align_up(off + b, 256);
        return o;
    };
    L.off_phat = take(ch * per_img);                        // [chunk][Qs][NBT]
    L.off_sum = take(ch * NBT * sizeof(double));            // [chunk][nb] or [chunk][NBT]
    L.off_kappa = take(ch * sizeof(double));                // [chunk]
    L.off_gBt = take(NBT * Qs * H * sizeof(cx<double>));    // [NBT][Qs][H]
    L.off_gAt = take(na * Qs * H * sizeof(cx<double>));     // [na][Qs][H]
    L.off_gApart = take(gat_max_split(NBT) * ch * Qs * H * sizeof(cx<double>));   // [split][chunk][Qs][H]
    L.off_gBpsi = take(NBT * H * Q * sizeof(cx<double>));   // [NBT][H][Q]
    L.off_gApsi = take(na * H * Q * sizeof(cx<double>));    // [na][H][Q]
    L.off_ph64 = take(T * K * Q * sizeof(cx<double>));      // [T][K][Q]
    L.off_part = take((na + nb) * K * H * sizeof(double));  // [na + nb][K][H]
    L.total = off;
    return L;
}

template <typename R>
__device__ __forceinline__ cx<double> up(const cx<R> &v) {
    return cx<double>{(double)v.re, (double)v.im};
}

// re + i im += sum_h conj(x[h st]) y[h st] over the ranks of one frequency
// (generic layout [item][h][q]: rank stride st = Qs); the loads of eight ranks
// are issued together so that a row costs H/8 memory round trips
template <typename R>
__device__ __forceinline__ void conj_dot(const cx<R> *__restrict__ x, const cx<R> *__restrict__ y, int H, int st,
                                         double &re, double &im) {
    int h = 0;
    for (; h + 8 <= H; h += 8) {
        cx<R> xv[8], yv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            xv[k] = x[(size_t)(h + k) * st];
            yv[k] = y[(size_t)(h + k) * st];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const cx<double> u = up(xv[k]), v = up(yv[k]);
            re += u.re * v.re + u.im * v.im;
            im += u.re * v.im - u.im * v.re;
        }
    }
    for (; h < H; ++h) {
        const cx<double> u = up(x[(size_t)h * st]), v = up(y[(size_t)h * st]);
        re += u.re * v.re + u.im * v.im;
        im += u.re * v.im - u.im * v.re;
    }
}

__device__ __forceinline__ void fill_twiddles(cx<double> *tw, int Q) {
    for (int i = threadIdx.x; i < Q; i += blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)i / (double)Q, &s, &c);
        tw[i] = cx<double>{c, s};
    }
}

// phi_t[r][j] = exp(-i k_r (dx cos psi_j + dy sin psi_j)) in FP64
__global__ void k_bwd_phase(const double *d_k, const double *d_delta, int K, int Q, int T, cx<double> *ph) {
    const int total = T * K * Q;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int j = i % Q, r = (i / Q) % K, t = i / (Q * K);
        double s, c;
        sincospi(2.0 * (double)j / (double)Q, &s, &c);
        const double arg = d_k[r] * (d_delta[2 * t] * c + d_delta[2 * t + 1] * s);
        double ps, pc;
        sincos(arg, &ps, &pc);
        ph[i] = cx<double>{pc, -ps};
    }
}

// sum over the 64 lanes of a wave; every lane gets the same value (fixed order)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// One workgroup per (image a0 + blockIdx.y, nbw consecutive targets); for each
// target, translations in groups of TG: the landscape X (contraction + FFT,
// FP64), Pt = exp(s Re X - c_a), the transform of Pt at the stored q, and the
// pair's sum of Pt over (t, m).
//
// Hermitian inputs: X_t and Pt_t are real, so two translations share one
// complex transform each way.  With spectra S_e, S_o extended by
// S[Q-q] = conj S[q] (real at q = 0 and Q/2), Z = S_e + i S_o transforms to
// X_e + i X_o; with Y = Pt_e + i Pt_o and its transform Yh,
// F_e[q] = (Yh[q] + conj Yh[Q-q]) / 2 and F_o[q] = (Yh[q] - conj Yh[Q-q]) / 2i.
template <typename R>
__global__ __launch_bounds__(256) void k_bwd_phat(const cx<R> *__restrict__ Ag, const cx<R> *__restrict__ Bg,
                                                  int a0, int n_tgt, int nbw, int T, int TG, int H, int Q, int Qs,
                                                  int herm, double s2, const float *__restrict__ lse_img,
                                                  cx<double> *__restrict__ Phat, double *__restrict__ psum) {
    __shared__ double red[16];
    __shared__ FftPlan spl;
    extern __shared__ unsigned char smem_raw[];
    const int NR = herm ? (TG + 1) / 2 : TG;   // transform rows per group
    cx<double> *tw = reinterpret_cast<cx<double> *>(smem_raw);
    cx<double> *X = tw + Q;                     // [NR][Q]
    cx<double> *Pb = X + (size_t)NR * Q;        // [NR][Q]
    const int al = blockIdx.y, a = a0 + al;
    const int b_begin = blockIdx.x * nbw, b_end = min(n_tgt, b_begin + nbw);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int M = Q / 2;
    const size_t NBT = (size_t)n_tgt * T;
    fill_twiddles(tw, Q);
    if (tid == 0) fft_init_plan(spl, Q);
    __syncthreads();
    const FftPlan &pl = spl;
    const double ca = (double)lse_img[a];
    const cx<R> *Aq = Ag + (size_t)a * Qs * H;
    for (int b = b_begin; b < b_end; ++b) {
        double mysum = 0.0;
        for (int t0 = 0; t0 < T; t0 += TG) {
            const int tg = min(TG, T - t0);
            const int nr = herm ? (tg + 1) / 2 : tg;
            const cx<R> *Bt = Bg + ((size_t)b * T + t0) * Qs * H;
            __syncthreads();   // X, Pb of the previous group are consumed
            if (herm) {
                for (int i = tid; i < nr * Qs; i += nt) {
                    const int rr = i / Qs, q = i - rr * Qs;
                    double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;
                    conj_dot(Aq + q, Bt + (size_t)(2 * rr) * H * Qs + q, H, Qs, er, ei);
                    if (2 * rr + 1 < tg) conj_dot(Aq + q, Bt + (size_t)(2 * rr + 1) * H * Qs + q, H, Qs, orr, oi);
                    if (q == 0 || q == M) ei = oi = 0.0;   // the real endpoints of a Hermitian spectrum
                    cx<double> *Z = X + (size_t)rr * Q;
                    Z[q] = cx<double>{er - oi, ei + orr};
                    if (q > 0 && q < M) Z[Q - q] = cx<double>{er + oi, orr - ei};
                }
            } else {
                for (int i = tid; i < tg * Qs; i += nt) {
                    const int tt = i / Qs, q = i - tt * Qs;
                    double re = 0.0, im = 0.0;
                    conj_dot(Aq + q, Bt + (size_t)tt * H * Qs + q, H, Qs, re, im);
                    X[(size_t)tt * Q + q] = cx<double>{re, im};
                }
            }
            __syncthreads();
            lds_fft_dif(X, nr, Q, pl, tw);   // X[row][pos(m)] = sum_q Z[q] W^{qm}
            for (int i = tid; i < nr * Q; i += nt) {
                const int rr = i / Q, m = i - rr * Q;
                const cx<double> x = X[(size_t)rr * Q + fft_pos(m, pl)];
                const double pe = exp(s2 * x.re - ca);
                double po = 0.0;
                if (herm && 2 * rr + 1 < tg) po = exp(s2 * x.im - ca);
                mysum += pe + po;
                Pb[(size_t)rr * Q + m] = cx<double>{pe, po};
            }
            __syncthreads();
            lds_fft_dif(Pb, nr, Q, pl, tw);   // sum_m Y[m] W^{qm}; Phat = conj of the unpacked transform
            cx<double> *out = Phat + (size_t)al * Qs * NBT + (size_t)b * T + t0;
            for (int i = tid; i < tg * Qs; i += nt) {
                const int q = i / tg, tt = i - q * tg;
                cx<double> F;
                if (herm) {
                    const cx<double> *Y = Pb + (size_t)(tt >> 1) * Q;
                    const cx<double> y = Y[fft_pos(q, pl)], z = Y[fft_pos(q == 0 ? 0 : Q - q, pl)];
                    if ((tt & 1) == 0) F = cx<double>{0.5 * (y.re + z.re), 0.5 * (y.im - z.im)};
                    else F = cx<double>{0.5 * (y.im + z.im), 0.5 * (z.re - y.re)};
                } else {
                    F = Pb[(size_t)tt * Q + fft_pos(q, pl)];
                }
                out[(size_t)q * NBT + tt] = cx<double>{F.re, -F.im};
            }
        }
        const double v = wave_sum(mysum);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            double sacc = 0.0;
            for (int w = 0; w < (nt >> 6); ++w) sacc += red[w];
            psum[(size_t)al * n_tgt + b] = sacc;
        }
    }
}


// ---- the P-hat step for Hermitian inputs and Q a power of two (64 .. 512) ----
//
// One wavefront per row of two landscape columns c0 = 2 r, c1 = 2 r + 1 of one
// image (columns are (target, translation) pairs): Z = S_e + i S_o (the two
// columns' spectra, extended by S[Q-q] = conj S[q]) is transformed to
// X_e + i X_o, Pt = exp(s X - c_a) is formed for both, Y = Pt_e + i Pt_o is
// transformed back, and the two columns' Phat are unpacked from it (the same
// algebra as k_bwd_phat).  The transforms run in the wave's own LDS rows with
// no workgroup barrier: a decimation-in-frequency FFT (one radix-2 stage first
// when log2 Q is odd, then radix-4 stages), whose output order is the
// digit reversal below.  Each column's sum of Pt goes to psum[image][column].

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// position of frequency k in the output of wave_fft_dif<Q>
template <int Q>
__device__ __forceinline__ int wfft_pos(int k) {
    constexpr int LOG = __builtin_ctz(Q);
    constexpr int ND = LOG / 2;   // radix-4 digits
    const int r2 = (LOG & 1) ? (k & 1) : 0;
    int x = (LOG & 1) ? (k >> 1) : k, rev = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        rev = (rev << 2) | (x & 3);
        x >>= 2;
    }
    return (LOG & 1) ? r2 * (Q / 2) + rev : rev;
}
// inverse of wfft_pos
template <int Q>
__device__ __forceinline__ int wfft_freq(int p) {
    constexpr int LOG = __builtin_ctz(Q);
    constexpr int ND = LOG / 2;
    const int blk = (LOG & 1) ? p / (Q / 2) : 0;
    int x = (LOG & 1) ? p % (Q / 2) : p, rev = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        rev = (rev << 2) | (x & 3);
        x >>= 2;
    }
    return (LOG & 1) ? 2 * rev + blk : rev;
}

// in place: buf[wfft_pos<Q>(k)] = sum_j buf[j] W_Q^{jk}, W_Q = exp(-2 pi i / Q); tw[k] = W_Q^k
template <int Q>
__device__ __forceinline__ void wave_fft_dif(cx<double> *buf, const cx<double> *tw, int lane) {
    constexpr int LOG = __builtin_ctz(Q);
    int L = Q;
    if constexpr (LOG & 1) {
        for (int i = lane; i < Q / 2; i += 64) {
            const cx<double> a = buf[i], b = buf[i + Q / 2];
            buf[i] = cadd(a, b);
            buf[i + Q / 2] = cmul(csub(a, b), tw[i]);
        }
        L = Q / 2;
        wave_sync();
    }
    for (; L >= 4; L /= 4) {
        const int qL = L / 4, stride = Q / L;
        for (int u = lane; u < Q / 4; u += 64) {
            const int blk = u / qL, i = u - blk * qL, base = blk * L + i;
            const cx<double> x0 = buf[base], x1 = buf[base + qL], x2 = buf[base + 2 * qL], x3 = buf[base + 3 * qL];
            const cx<double> t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3);
            const cx<double> d = csub(x1, x3), t3 = {d.im, -d.re};   // -i (x1 - x3)
            buf[base] = cadd(t0, t2);
            buf[base + qL] = cmul(cadd(t1, t3), tw[i * stride]);
            buf[base + 2 * qL] = cmul(csub(t0, t2), tw[2 * i * stride]);
            buf[base + 3 * qL] = cmul(csub(t1, t3), tw[3 * i * stride]);
        }
        wave_sync();
    }
}

template <typename R, int Q>
__global__ __launch_bounds__(256) void k_bwd_phat_wave(const cx<R> *__restrict__ Ag, const cx<R> *__restrict__ Bg,
                                                       int a0, int NBT, int rows_per_wg, int H, double s2,
                                                       const float *__restrict__ lse_img,
                                                       cx<double> *__restrict__ Phat, double *__restrict__ psum) {
    constexpr int M = Q / 2, Qs = M + 1;
    constexpr int KQ = (Qs + 63) / 64;   // spectrum entries per lane
    __shared__ cx<double> tw[Q];
    __shared__ cx<double> wbuf[4][2][Q];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < Q; i += blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * (double)i / (double)Q, &sn, &cs);
        tw[i] = cx<double>{cs, sn};
    }
    __syncthreads();
    const int al = blockIdx.y, a = a0 + al;
    const double ca = (double)lse_img[a];
    const cx<R> *Aq = Ag + (size_t)a * Qs * H;
    cx<double> *b1 = wbuf[w][0], *b2 = wbuf[w][1];
    const int n_rows = (NBT + 1) / 2;
    const int r_begin = blockIdx.x * rows_per_wg, r_end = min(n_rows, r_begin + rows_per_wg);
    for (int r = r_begin + w; r < r_end; r += 4) {
        const int c0 = 2 * r, c1 = 2 * r + 1;
        const bool two = c1 < NBT;
        // spectra of the two columns at q = lane + 64 k, q <= M
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            const int q = lane + 64 * k;
            if (q > M) continue;
            double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;
            conj_dot(Aq + q, Bg + (size_t)c0 * H * Qs + q, H, Qs, er, ei);
            if (two) conj_dot(Aq + q, Bg + (size_t)c1 * H * Qs + q, H, Qs, orr, oi);
            if (q == 0 || q == M) ei = oi = 0.0;   // the real endpoints of a Hermitian spectrum
            b1[q] = cx<double>{er - oi, ei + orr};
            if (q > 0 && q < M) b1[Q - q] = cx<double>{er + oi, orr - ei};
        }
        wave_sync();
        wave_fft_dif<Q>(b1, tw, lane);   // b1[pos(m)] = X_e[m] + i X_o[m]
        double se = 0.0, so = 0.0;
        for (int p = lane; p < Q; p += 64) {
            const cx<double> x = b1[p];
            const double pe = exp(s2 * x.re - ca);
            const double po = two ? exp(s2 * x.im - ca) : 0.0;
            se += pe;
            so += po;
            b2[wfft_freq<Q>(p)] = cx<double>{pe, po};   // natural order for the second transform
        }
        wave_sync();
        wave_fft_dif<Q>(b2, tw, lane);   // b2[pos(q)] = sum_m Y[m] W^{qm}
        cx<double> *out = Phat + (size_t)al * Qs * NBT;
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            const int q = lane + 64 * k;
            if (q > M) continue;
            const cx<double> y = b2[wfft_pos<Q>(q)], z = b2[wfft_pos<Q>(q == 0 ? 0 : Q - q)];
            // Phat = conj of each column's transform
            out[(size_t)q * NBT + c0] = cx<double>{0.5 * (y.re + z.re), -0.5 * (y.im - z.im)};
            if (two) out[(size_t)q * NBT + c1] = cx<double>{0.5 * (y.im + z.im), -0.5 * (z.re - y.re)};
        }
        se = wave_sum(se);
        so = wave_sum(so);
        if (lane == 0) {
            psum[(size_t)al * NBT + c0] = se;
            if (two) psum[(size_t)al * NBT + c1] = so;
        }
        wave_sync();   // b1, b2 are rewritten by the next row
    }
}

// kappa[a] = g[a] s / sum_{b,t,m} Pt  (= g[a] s exp(c_a - lse_img[a]), exact lse)
// (psum: per image, n_cols partial sums; one workgroup per image, each thread
// a contiguous range, the ranges added in thread order: a fixed order)
__global__ __launch_bounds__(256) void k_bwd_kappa(const double *__restrict__ psum, const float *__restrict__ glse,
                                                   int a0, int n_cols, double s2, double *__restrict__ kappa) {
    __shared__ double part[256];
    const int al = blockIdx.x, tid = threadIdx.x;
    const int per = (n_cols + 255) / 256, c0 = min(n_cols, per * tid), c1 = min(n_cols, c0 + per);
    double acc = 0.0;
    for (int c = c0; c < c1; ++c) acc += psum[(size_t)al * n_cols + c];
    part[tid] = acc;
    __syncthreads();
    if (tid == 0) {
        double sacc = 0.0;
        for (int x = 0; x < 256; ++x) sacc += part[x];
        kappa[al] = (double)glse[a0 + al] * s2 / sacc;
    }
}

// Register blocking of the two per-frequency contractions: a thread keeps CB
// columns (g_bt) or images (g_at) times HPT ranks h = wave + 4 i, so each rank
// value it reads from LDS (the same address across the wave) serves CB
// products and each Phat value HPT of them.  Tiles of AT images (g_bt) or
// columns (g_at) are fetched into registers while the previous tile is used.
// Every output is a sum over the chunk's images (g_bt) or the span's columns
// (g_at) taken in index order.  g_bt runs with CB = 2: its workgroups each
// reduce over the whole chunk, and with CB = 4 their count (NBT / 256 times
// Qs) no longer filled the chip evenly (1.51 ms against 1.33 per call at the
// differentiation workload; CB = 2 with tiles of 8 images took the backward
// from 22.6 to 22.3 ms); g_at with CB = 4 took 1.07 ms against 1.32.

// g_bt[bt][q][h] (+)= sum_{a in chunk} at[a][q][h] kappa[a] Phat[a][q][bt]; one
// workgroup per (TILE columns bt, q)
template <typename R, int HPT, int CB, int AT>
__global__ __launch_bounds__(256) void k_bwd_gBt(const cx<R> *__restrict__ Ag, const cx<double> *__restrict__ Phat,
                                                 const double *__restrict__ kappa, int a0, int na_chunk, int NBT,
                                                 int Qs, int H, int accumulate, cx<double> *__restrict__ gBt) {
    constexpr int TILE = 64 * CB;
    __shared__ cx<double> sP[AT][TILE];
    __shared__ cx<double> sA[AT][kMaxH];
    const int q = blockIdx.y, bt0 = blockIdx.x * TILE;
    const int tid = threadIdx.x, bl = tid & 63, hg = tid >> 6;
    cx<double> acc[CB][HPT];
#pragma unroll
    for (int k = 0; k < CB; ++k)
#pragma unroll
        for (int i = 0; i < HPT; ++i) acc[k][i] = cx<double>{0.0, 0.0};
    constexpr int NP = AT * TILE / 256;   // Phat values per thread and tile
    constexpr int NA = (AT * kMaxH + 255) / 256;   // rank values per thread and tile
    cx<double> rp[NP], ra[NA];
    auto fetch = [&](int c0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int e = tid + 256 * j, aa = e / TILE, bb = e % TILE;
            cx<double> v = {0.0, 0.0};
            if (c0 + aa < na_chunk && bt0 + bb < NBT)
                v = cscale(Phat[((size_t)(c0 + aa) * Qs + q) * NBT + bt0 + bb], kappa[c0 + aa]);
            rp[j] = v;
        }
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const int e = tid + 256 * j, aa = e / H, h = e - aa * H;
            ra[j] = cx<double>{0.0, 0.0};
            if (e < AT * H && c0 + aa < na_chunk) ra[j] = up(Ag[((size_t)(a0 + c0 + aa) * H + h) * Qs + q]);
        }
    };
    fetch(0);
    for (int c0 = 0; c0 < na_chunk; c0 += AT) {
        __syncthreads();   // the previous tile is consumed
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int e = tid + 256 * j;
            sP[e / TILE][e % TILE] = rp[j];
        }
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const int e = tid + 256 * j;
            if (e < AT * H) sA[e / H][e % H] = ra[j];
        }
        __syncthreads();
        if (c0 + AT < na_chunk) fetch(c0 + AT);
#pragma unroll 2
        for (int aa = 0; aa < AT; ++aa) {
            cx<double> pv[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) pv[k] = sP[aa][bl + 64 * k];
#pragma unroll
            for (int i = 0; i < HPT; ++i) {
                const int h = hg + 4 * i;
                if (h < H) {
                    const cx<double> av = sA[aa][h];
#pragma unroll
                    for (int k = 0; k < CB; ++k) acc[k][i] = cadd(acc[k][i], cmul(av, pv[k]));
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < CB; ++k) {
        const int bt = bt0 + bl + 64 * k;
        if (bt >= NBT) continue;
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            const int h = hg + 4 * i;
            if (h < H) {
                cx<double> *o = gBt + ((size_t)bt * Qs + q) * H + h;
                *o = accumulate ? cadd(*o, acc[k][i]) : acc[k][i];
            }
        }
    }
}

// Partial g_at over one span of columns: part[sp][al][q][h] =
// sum_{bt in span sp} conj(Phat[al][q][bt]) bt[bt][q][h]; one workgroup per
// (TILE images, q, span)
template <typename R, int HPT, int CB, int AT>
__global__ __launch_bounds__(256) void k_bwd_gAt(const cx<R> *__restrict__ Bg, const cx<double> *__restrict__ Phat,
                                                 int na_chunk, int NBT, int Qs, int H, int span,
                                                 cx<double> *__restrict__ part) {
    constexpr int TILE = 64 * CB;
    __shared__ cx<double> sP[TILE][AT + 1];
    __shared__ cx<double> sB[AT][kMaxH];
    const int q = blockIdx.y, al0 = blockIdx.x * TILE, sp = blockIdx.z;
    const int c_begin = sp * span, c_end = min(NBT, c_begin + span);
    const int tid = threadIdx.x, al = tid & 63, hg = tid >> 6;
    cx<double> acc[CB][HPT];
#pragma unroll
    for (int k = 0; k < CB; ++k)
#pragma unroll
        for (int i = 0; i < HPT; ++i) acc[k][i] = cx<double>{0.0, 0.0};
    constexpr int NP = AT * TILE / 256;
    constexpr int NB = (AT * kMaxH + 255) / 256;   // rank values per thread and tile
    cx<double> rp[NP], rb[NB];
    auto fetch = [&](int c0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int e = tid + 256 * j, aa = e / AT, bb = e % AT;
            double vr = 0.0, vi = 0.0;
            if (al0 + aa < na_chunk && c0 + bb < c_end) {
                const cx<double> *src = Phat + ((size_t)(al0 + aa) * Qs + q) * NBT + c0 + bb;
                vr = src->re;
                vi = src->im;
            }
            rp[j] = cx<double>{vr, vi};
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int e = tid + 256 * j, bb = e / H, h = e - bb * H;
            rb[j] = cx<double>{0.0, 0.0};
            if (e < AT * H && c0 + bb < c_end) rb[j] = up(Bg[((size_t)(c0 + bb) * H + h) * Qs + q]);
        }
    };
    fetch(c_begin);
    for (int c0 = c_begin; c0 < c_end; c0 += AT) {
        __syncthreads();   // the previous tile is consumed
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int e = tid + 256 * j;
            sP[e / AT][e % AT] = rp[j];
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int e = tid + 256 * j;
            if (e < AT * H) sB[e / H][e % H] = rb[j];
        }
        __syncthreads();
        if (c0 + AT < c_end) fetch(c0 + AT);
#pragma unroll 2
        for (int bb = 0; bb < AT; ++bb) {
            cx<double> pv[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) pv[k] = cconj(sP[al + 64 * k][bb]);
#pragma unroll
            for (int i = 0; i < HPT; ++i) {
                const int h = hg + 4 * i;
                if (h < H) {
                    const cx<double> bv = sB[bb][h];
#pragma unroll
                    for (int k = 0; k < CB; ++k) acc[k][i] = cadd(acc[k][i], cmul(pv[k], bv));
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < CB; ++k) {
        const int a = al0 + al + 64 * k;
        if (a >= na_chunk) continue;
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            const int h = hg + 4 * i;
            if (h < H) part[(((size_t)sp * na_chunk + a) * Qs + q) * H + h] = acc[k][i];
        }
    }
}

// g_at[a0 + al][q][h] = kappa[al] sum_sp part[sp][al][q][h] (spans in order)
__global__ void k_bwd_gAt_reduce(const cx<double> *__restrict__ part, const double *__restrict__ kappa, int a0,
                                 int na_chunk, int QH, int nsplit, cx<double> *__restrict__ gAt) {
    const size_t total = (size_t)na_chunk * QH;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        cx<double> v = part[i];
        for (int sp = 1; sp < nsplit; ++sp) v = cadd(v, part[(size_t)sp * total + i]);
        gAt[(size_t)a0 * QH + i] = cscale(v, kappa[i / QH]);
    }
}

// psi-space ring gradients: G[n][q][h] (stored q) -> Gpsi[n][h][j] =
// Q^{-1/2} sum_q exp(+2 pi i q j / Q) G[q], the full spectrum rebuilt from the
// Hermitian half when herm.  One workgroup per row n; HC rank rows per pass.
__global__ __launch_bounds__(256) void k_bwd_inv_rings(const cx<double> *__restrict__ G, int H, int Q, int Qs,
                                                       int herm, int HC, cx<double> *__restrict__ Gpsi) {
    extern __shared__ unsigned char smem_raw[];
    cx<double> *tw = reinterpret_cast<cx<double> *>(smem_raw);
    cx<double> *buf = tw + Q;
    const int n = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int M = Q / 2;
    fill_twiddles(tw, Q);
    __shared__ FftPlan spl;   // in LDS: the FFT stage loops index it at run time
    if (threadIdx.x == 0) fft_init_plan(spl, Q);
    __syncthreads();
    const FftPlan &pl = spl;
    const double sc = 1.0 / sqrt((double)Q);
    const cx<double> *Gn = G + (size_t)n * Qs * H;
    for (int h0 = 0; h0 < H; h0 += HC) {
        const int hc = min(HC, H - h0);
        __syncthreads();
        for (int i = tid; i < hc * Q; i += nt) {
            const int hh = i / Q, q = i - hh * Q;
            cx<double> v;
            if (!herm || q <= M) {
                v = Gn[(size_t)q * H + h0 + hh];
            } else {
                const int qq = Q - q;
                const cx<double> u = Gn[(size_t)qq * H + h0 + hh];
                v = (qq & 1) ? cx<double>{-u.re, u.im} : cx<double>{u.re, -u.im};   // (-1)^qq conj(u)
            }
            buf[hh * Q + q] = cconj(v);
        }
        __syncthreads();
        lds_fft_dif(buf, hc, Q, pl, tw);
        for (int i = tid; i < hc * Q; i += nt) {
            const int hh = i / Q, j = i - hh * Q;
            const cx<double> v = buf[hh * Q + fft_pos(j, pl)];
            Gpsi[((size_t)n * H + h0 + hh) * Q + j] = cx<double>{v.re * sc, -v.im * sc};
        }
    }
}

// dL/dBhat[b][r][j] = eta_r sum_t conj(phi_t[r][j]) sum_h U[r][h] g_Br[b][t][h][j]
template <typename R>
__global__ __launch_bounds__(256) void k_bwd_gBhat(const cx<double> *__restrict__ gBpsi, const double *__restrict__ U,
                                                   const double *__restrict__ eta, const cx<double> *__restrict__ ph,
                                                   int K, int H, int Q, int T, cx<R> *__restrict__ gB) {
    const int b = blockIdx.x, r = blockIdx.y;
    const double er = eta[r];
    for (int j = threadIdx.x; j < Q; j += blockDim.x) {
        cx<double> acc = {0.0, 0.0};
        for (int t = 0; t < T; ++t) {
            const cx<double> *g = gBpsi + ((size_t)b * T + t) * H * Q + j;
            cx<double> s = {0.0, 0.0};
            for (int h = 0; h < H; ++h) {
                const double u = U[(size_t)r * K + h];
                const cx<double> v = g[(size_t)h * Q];
                s.re += u * v.re;
                s.im += u * v.im;
            }
            acc = cadd(acc, cmul(cconj(ph[((size_t)t * K + r) * Q + j]), s));
        }
        gB[((size_t)b * K + r) * Q + j] = cx<R>{(R)(er * acc.re), (R)(er * acc.im)};
    }
}

// part[n][r][h] = sum_t sum_j Re(conj(Gpsi[n][t][h][j]) eta_r phi_t[r][j] X[n][r][j])
// (phi = 1 when ph is null).  One workgroup per item n; j in chunks of 16.
template <typename R>
__global__ __launch_bounds__(256) void k_bwd_gU_part(const cx<double> *__restrict__ Gpsi, const cx<R> *__restrict__ Xp,
                                                     const double *__restrict__ eta, const cx<double> *__restrict__ ph,
                                                     int K, int H, int Q, int T, double *__restrict__ part) {
    __shared__ cx<double> sY[kMaxK][17];
    __shared__ cx<double> sG[kMaxH][17];
    const int n = blockIdx.x, tid = threadIdx.x;
    const int nout = K * H;
    double acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    for (int t = 0; t < T; ++t) {
        for (int j0 = 0; j0 < Q; j0 += 16) {
            __syncthreads();
            for (int e = tid; e < K * 16; e += 256) {
                const int r = e >> 4, jj = e & 15, j = j0 + jj;
                cx<double> y = {0.0, 0.0};
                if (j < Q) {
                    y = up(Xp[((size_t)n * K + r) * Q + j]);
                    if (ph) y = cmul(ph[((size_t)t * K + r) * Q + j], y);
                    y = cscale(y, eta[r]);
                }
                sY[r][jj] = y;
            }
            for (int e = tid; e < H * 16; e += 256) {
                const int h = e >> 4, jj = e & 15, j = j0 + jj;
                sG[h][jj] = (j < Q) ? Gpsi[(((size_t)n * T + t) * H + h) * Q + j] : cx<double>{0.0, 0.0};
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int o = tid + 256 * i;
                if (o < nout) {
                    const int r = o / H, h = o - r * H;
                    double s = 0.0;
                    for (int jj = 0; jj < 16; ++jj) s += sG[h][jj].re * sY[r][jj].re + sG[h][jj].im * sY[r][jj].im;
                    acc[i] += s;
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int o = tid + 256 * i;
        if (o < nout) part[(size_t)n * nout + o] = acc[i];
    }
}

// gU[r][h] = sum_n part[n][r][h]: one workgroup per 64 outputs, its four waves
// take contiguous quarters of the items and add them in wave order (fixed)
__global__ __launch_bounds__(256) void k_bwd_gU_reduce(const double *__restrict__ part, int n_items, int K, int H,
                                                       double *__restrict__ gU) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + lane;
    const int per = (n_items + 3) / 4, n0 = min(n_items, per * w), n1 = min(n_items, n0 + per);
    double s = 0.0;
    if (o < K * H)
        for (int n = n0; n < n1; ++n) s += part[(size_t)n * K * H + o];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && o < K * H) gU[o] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

template <typename R>
hipError_t run_backward(const radsvd_plan *p, float inv_s2, const float *lse_img, const float *glse, void *gB_out,
                        double *gU_out, void *ws, hipStream_t s) {
    const BwdLayout L = bwd_layout(p);
    char *w = reinterpret_cast<char *>(ws);
    cx<double> *Phat = reinterpret_cast<cx<double> *>(w + L.off_phat);
    double *psum = reinterpret_cast<double *>(w + L.off_sum);
    double *kappa = reinterpret_cast<double *>(w + L.off_kappa);
    cx<double> *gBt = reinterpret_cast<cx<double> *>(w + L.off_gBt);
    cx<double> *gAt = reinterpret_cast<cx<double> *>(w + L.off_gAt);
    cx<double> *gApart = reinterpret_cast<cx<double> *>(w + L.off_gApart);
    cx<double> *gBpsi = reinterpret_cast<cx<double> *>(w + L.off_gBpsi);
    cx<double> *gApsi = reinterpret_cast<cx<double> *>(w + L.off_gApsi);
    cx<double> *ph = reinterpret_cast<cx<double> *>(w + L.off_ph64);
    double *part = reinterpret_cast<double *>(w + L.off_part);
    const cx<R> *Ag = reinterpret_cast<const cx<R> *>(p->Ag);
    const cx<R> *Bg = reinterpret_cast<const cx<R> *>(p->Bg);
    const int K = p->K, Q = p->Q, H = p->H, T = p->T, Qs = p->Qc, na = p->n_img, nb = p->n_tgt;
    const int NBT = nb * T;
    const bool want_U = gU_out != nullptr;

    hipLaunchKernelGGL(k_bwd_phase, dim3((T * K * Q + 255) / 256 < 4096 ? (T * K * Q + 255) / 256 : 4096), dim3(256),
                       0, s, p->d_k, p->d_delta, K, Q, T, ph);
    // translations per group: twiddles and the two row sets within ~40 KB of LDS
    // (four workgroups per CU); a Hermitian row holds two translations
    const int rows = max(1, (int)(((size_t)40 * 1024 / ((size_t)Q * sizeof(cx<double>)) - 1) / 2));
    const int TG = max(1, min(T, p->herm ? 2 * rows : rows));
    const int NR = p->herm ? (TG + 1) / 2 : TG;
    const size_t sh_phat = (size_t)(1 + 2 * NR) * Q * sizeof(cx<double>);
    {
        hipError_t e = hipFuncSetAttribute((const void *)k_bwd_phat<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sh_phat);
        if (e != hipSuccess) return e;
    }
    // the wave-per-row P-hat kernel: Hermitian inputs, Q a power of two
    const bool wave_path = p->herm && Q >= 64 && Q <= 512 && (Q & (Q - 1)) == 0;
    for (int a0 = 0; a0 < na; a0 += L.chunk) {
        const int ca = min(L.chunk, na - a0);
        int n_cols;
        if (wave_path) {
            const int n_rows = (NBT + 1) / 2, rpw = 16;
            const dim3 grid((n_rows + rpw - 1) / rpw, ca);
            switch (Q) {
            case 64: hipLaunchKernelGGL((k_bwd_phat_wave<R, 64>), grid, dim3(256), 0, s, Ag, Bg, a0, NBT, rpw, H,
                                        (double)inv_s2, lse_img, Phat, psum); break;
            case 128: hipLaunchKernelGGL((k_bwd_phat_wave<R, 128>), grid, dim3(256), 0, s, Ag, Bg, a0, NBT, rpw, H,
                                         (double)inv_s2, lse_img, Phat, psum); break;
            case 256: hipLaunchKernelGGL((k_bwd_phat_wave<R, 256>), grid, dim3(256), 0, s, Ag, Bg, a0, NBT, rpw, H,
                                         (double)inv_s2, lse_img, Phat, psum); break;
            default: hipLaunchKernelGGL((k_bwd_phat_wave<R, 512>), grid, dim3(256), 0, s, Ag, Bg, a0, NBT, rpw, H,
                                        (double)inv_s2, lse_img, Phat, psum); break;
            }
            n_cols = NBT;
        } else {
            // targets per workgroup: amortise the set-up while keeping ~4k workgroups
            const int nbw = max(1, min(16, (int)(((size_t)ca * nb) / 4096)));
            hipLaunchKernelGGL(k_bwd_phat<R>, dim3((nb + nbw - 1) / nbw, ca), dim3(256), sh_phat, s, Ag, Bg, a0, nb,
                               nbw, T, TG, H, Q, Qs, p->herm, (double)inv_s2, lse_img, Phat, psum);
            n_cols = nb;
        }
        hipLaunchKernelGGL(k_bwd_kappa, dim3(ca), dim3(256), 0, s, psum, glse, a0, n_cols, (double)inv_s2, kappa);
        const dim3 gb((NBT + 64 * kGbCB - 1) / (64 * kGbCB), Qs);
        if (H <= 16)
            hipLaunchKernelGGL((k_bwd_gBt<R, 4, kGbCB, kGbAT>), gb, dim3(256), 0, s, Ag, Phat, kappa, a0, ca, NBT, Qs,
                               H, a0 > 0 ? 1 : 0, gBt);
        else
            hipLaunchKernelGGL((k_bwd_gBt<R, 8, kGbCB, kGbAT>), gb, dim3(256), 0, s, Ag, Phat, kappa, a0, ca, NBT, Qs,
                               H, a0 > 0 ? 1 : 0, gBt);
        if (want_U) {
            const int span = gat_span(ca, Qs, NBT), nsplit = (NBT + span - 1) / span;
            const dim3 ga((ca + 64 * kGaCB - 1) / (64 * kGaCB), Qs, nsplit);
            if (H <= 16)
                hipLaunchKernelGGL((k_bwd_gAt<R, 4, kGaCB, kGaAT>), ga, dim3(256), 0, s, Bg, Phat, ca, NBT, Qs, H,
                                   span, gApart);
            else
                hipLaunchKernelGGL((k_bwd_gAt<R, 8, kGaCB, kGaAT>), ga, dim3(256), 0, s, Bg, Phat, ca, NBT, Qs, H,
                                   span, gApart);
            const size_t tot = (size_t)ca * Qs * H;
            const int nblk = (int)std::min<size_t>(4096, (tot + 255) / 256);
            hipLaunchKernelGGL(k_bwd_gAt_reduce, dim3(nblk), dim3(256), 0, s, gApart, kappa, a0, ca, Qs * H, nsplit,
                               gAt);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int HC = max(1, min(H, (int)((size_t)60 * 1024 / ((size_t)Q * sizeof(cx<double>))) - 1));
    const size_t sh_inv = (size_t)(1 + HC) * Q * sizeof(cx<double>);
    hipLaunchKernelGGL(k_bwd_inv_rings, dim3(NBT), dim3(256), sh_inv, s, gBt, H, Q, Qs, p->herm, HC, gBpsi);
    if (gB_out)
        hipLaunchKernelGGL(k_bwd_gBhat<R>, dim3(nb, K), dim3(256), 0, s, gBpsi, p->U, p->d_eta, ph, K, H, Q, T,
                           reinterpret_cast<cx<R> *>(gB_out));
    if (want_U) {
        hipLaunchKernelGGL(k_bwd_inv_rings, dim3(na), dim3(256), sh_inv, s, gAt, H, Q, Qs, p->herm, HC, gApsi);
        hipLaunchKernelGGL(k_bwd_gU_part<R>, dim3(na), dim3(256), 0, s, gApsi,
                           reinterpret_cast<const cx<R> *>(p->A_polar), p->d_eta, (const cx<double> *)nullptr, K, H,
                           Q, 1, part);
        hipLaunchKernelGGL(k_bwd_gU_part<R>, dim3(nb), dim3(256), 0, s, gBpsi,
                           reinterpret_cast<const cx<R> *>(p->B_polar), p->d_eta, ph, K, H, Q, T,
                           part + (size_t)na * K * H);
        hipLaunchKernelGGL(k_bwd_gU_reduce, dim3((K * H + 63) / 64), dim3(256), 0, s, part, na + nb, K, H, gU_out);
    }
    return hipGetLastError();
}

}  // namespace

size_t backward_bytes(const radsvd_plan *p) { return bwd_layout(p).total; }

hipError_t launch_backward(const radsvd_plan *p, float inv_s2, const float *lse_img, const float *glse, void *gB,
                           double *gU, void *ws, hipStream_t s) {
    if (p->prec == RADSVD_FP64) return run_backward<double>(p, inv_s2, lse_img, glse, gB, gU, ws, s);
    return run_backward<float>(p, inv_s2, lse_img, glse, gB, gU, ws, s);
}

}  // namespace radsvd
