// Rotational volume alignment with principal volumes (paper section 4).
//
// Precompute (section 4.9, items 1-7 of its operation count):
//   k_vol_C       radial kernel C_rr' = sqrt(w_r w_r') Re sum_{l>=1,m} conj(B_l^m(k_r)) B_l^m(k_r')
//                 averaged over the targets (section 4.6);
//   k_vol_D       degree kernel D_ll' = Re sum_r w_r sum_m conj(B_l^m(k_r)) B_l'^m(k_r),
//                 l, l' >= 1, averaged over the targets (section 4.8);
//   (Jacobi)      their eigenvectors, descending (the FP64 solver of C for images);
//   k_vol_shells  principal shells [u_h^T A]_l^m = sum_r U[r][h] sqrt(w_r) A_l^m(k_r) (section 4.5);
//   k_vol_wigner  [v_j^T d]_{m1 m2}(beta) = sum_l V[l][j] d^l_{m1 m2}(beta) on the periodic
//                 M x M order grid, with d^l by its three-term recurrence in l from
//                 the closed form at l = max(|m1|, |m2|) (section 4.7), in FP64, one
//                 recurrence for up to 16 ranks.
// Per pair (section 4.9, steps 1, 1b, 2, 3):
//   k_vol_xt      step 1, Xt_l(m1, m2) = sum_h conj(As[h]_l^m1) Bs[h]_l^m2, one workgroup
//                 per (degree, pair) with the degree's blocks staged in LDS;
//   k_vol_step1b  Y_j(m1, m2) = sum_l V[l][j] Xt_l(m1, m2);
//   k_vol_step2   Xhat(beta) = sum_j [v_j^T d](beta) Y_j for a block of pairs and every
//                 angle, 8 pairs x 8 angles per thread;
//   k_vol_land*   one workgroup per (pair, beta): Xhat into LDS, then the 2-D
//                 transform over the orders (M = 2L + 1 is odd: a direct DFT
//                 against an LDS twiddle table, as two dense complex matrix
//                 products on the matrix cores, FP32 or FP64 as the plan), then
//                 the best Re X of the angle and the FULL write;
//   k_vol_best    per pair, the best over the angles.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "internal.h"
#include "volume.h"

namespace radsvd {

namespace {

__device__ __forceinline__ void vol_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum over a 256-thread workgroup, the same value in every thread; fixed order
__device__ double vol_block_sum(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

__global__ void k_vol_setup(VolGrid g, double *w, double *beta) {
    for (int i = threadIdx.x; i < g.K; i += blockDim.x) w[i] = g.w[i];
    for (int i = threadIdx.x; i < g.n_beta; i += blockDim.x) beta[i] = g.beta[i];
}

template <typename R>
__global__ __launch_bounds__(256) void k_vol_C(const cx<R> *__restrict__ B, int n_tgt, int K, int NC,
                                               const double *__restrict__ w, double *__restrict__ C) {
    __shared__ double red[4];
    const int r = blockIdx.x, rp = blockIdx.y;
    if (rp < r) return;   // uniform in the workgroup
    const long long per = NC - 1;   // every (l, m) with l >= 1
    const long long n = (long long)n_tgt * per;
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) {
        const long long b = i / per;
        const int c = 1 + (int)(i - b * per);
        const cx<R> x = B[((size_t)b * K + r) * NC + c], y = B[((size_t)b * K + rp) * NC + c];
        acc += (double)x.re * (double)y.re + (double)x.im * (double)y.im;
    }
    const double s = vol_block_sum(acc, red) * (sqrt(w[r]) * sqrt(w[rp])) / (double)n_tgt;
    if (threadIdx.x == 0) {
        C[(size_t)r * K + rp] = s;
        C[(size_t)rp * K + r] = s;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_vol_D(const cx<R> *__restrict__ B, int n_tgt, int K, int NC, int L,
                                               const double *__restrict__ w, double *__restrict__ D) {
    __shared__ double red[4];
    const int l = blockIdx.x, lp = blockIdx.y;   // l <= lp: the orders |m| <= l
    if (lp < l) return;
    double s = 0.0;
    if (l >= 1) {
        const int nm = 2 * l + 1;
        const long long n = (long long)n_tgt * K * nm;
        double acc = 0.0;
        for (long long i = threadIdx.x; i < n; i += 256) {
            const long long br = i / nm;
            const int m = (int)(i - br * nm) - l;
            const int r = (int)(br % K);
            const cx<R> *row = B + (size_t)br * NC;   // [b][r]
            const cx<R> x = row[l * l + l + m], y = row[lp * lp + lp + m];
            acc += w[r] * ((double)x.re * (double)y.re + (double)x.im * (double)y.im);
        }
        s = vol_block_sum(acc, red) / (double)n_tgt;
    }
    if (threadIdx.x == 0) {
        D[(size_t)l * (L + 1) + lp] = s;
        D[(size_t)lp * (L + 1) + l] = s;
    }
}

// caller-supplied principal vectors [n][H] into the [n][n] column layout
__global__ void k_vol_user_mat(const double *__restrict__ Uin, int n, int H, double *__restrict__ U,
                               double *__restrict__ lam) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * n; i += gridDim.x * blockDim.x) {
        const int r = i / n, c = i - r * n;
        U[i] = c < H ? Uin[(size_t)r * H + c] : 0.0;
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        lam[i] = __builtin_nan("");
}

// principal shells, thread per (volume, coefficient) and block of up to
// kShellHB ranks: each volume value is read once per rank block; the weights
// U[r][h] sqrt(w_r) are staged in LDS (dynamic, K kShellHB doubles)
constexpr int kShellHB = 16;
template <typename R>
__global__ __launch_bounds__(256) void k_vol_shells(const cx<R> *__restrict__ X, int n, int K, int NC,
                                                    const double *__restrict__ U, int H,
                                                    const double *__restrict__ w, cx<R> *__restrict__ out) {
    extern __shared__ double sUw[];   // [K][kShellHB]
    const int h0 = blockIdx.y * kShellHB;
    for (int k = threadIdx.x; k < K * kShellHB; k += 256) {
        const int r = k / kShellHB, hh = k - r * kShellHB;
        sUw[k] = h0 + hh < H ? U[(size_t)r * K + h0 + hh] * sqrt(w[r]) : 0.0;
    }
    __syncthreads();
    const int nbx = (NC + 255) / 256;
    const long long v = blockIdx.x / nbx;
    const int i = (int)(blockIdx.x - v * nbx) * 256 + threadIdx.x;
    if (i >= NC) return;
    double re[kShellHB], im[kShellHB];
#pragma unroll
    for (int hh = 0; hh < kShellHB; ++hh) re[hh] = im[hh] = 0.0;
    for (int r = 0; r < K; ++r) {
        const cx<R> x = X[((size_t)v * K + r) * NC + i];
        const double xr = (double)x.re, xi = (double)x.im;
#pragma unroll
        for (int hh = 0; hh < kShellHB; ++hh) {
            const double u = sUw[r * kShellHB + hh];
            re[hh] += u * xr;
            im[hh] += u * xi;
        }
    }
#pragma unroll
    for (int hh = 0; hh < kShellHB; ++hh)
        if (h0 + hh < H) out[((size_t)v * H + h0 + hh) * NC + i] = cx<R>{(R)re[hh], (R)im[hh]};
}

// d^l_{ab}(beta) at l = max(|a|, |b|), from c = cos(beta/2), s = sin(beta/2):
// the one surviving term of the finite sum for d^l
__device__ double wigner_seed(int l, int a, int b, double c, double s) {
    int e, pc, ps;
    double sgn = 1.0;
    if (a == l) {
        e = b;
        pc = l + b;
        ps = l - b;
        if ((l - b) & 1) sgn = -1.0;
    } else if (a == -l) {
        e = b;
        pc = l - b;
        ps = l + b;
    } else if (b == l) {
        e = a;
        pc = l + a;
        ps = l - a;
    } else {   // b == -l
        e = a;
        pc = l - a;
        ps = l + a;
        if ((a + l) & 1) sgn = -1.0;
    }
    // sqrt(binomial(2l, l + e)) = prod_{i=1}^{l-|e|} sqrt((l + |e| + i) / i)
    const int ae = e < 0 ? -e : e;
    double v = sgn;
    for (int i = 1; i <= l - ae; ++i) v *= sqrt((double)(l + ae + i) / (double)i);
    for (int i = 0; i < pc; ++i) v *= c;
    for (int i = 0; i < ps; ++i) v *= s;
    return v;
}

constexpr int kWigJB = 16;   // degree ranks accumulated per recurrence

// thread per (beta, m1, m2) and block of up to kWigJB ranks: one recurrence
// in l, accumulated into each rank's table.  The workgroup stages the first
// HD columns of V in LDS (dynamic, (L + 1) HD doubles); the root
// sqrt((l^2 - a^2)(l^2 - b^2)) of one step is carried into the next.
template <typename R>
__global__ __launch_bounds__(256) void k_vol_wigner(const double *__restrict__ beta, int n_beta, int L, int M,
                                                    const double *__restrict__ V, int HD, int real,
                                                    R *__restrict__ Vd) {
    extern __shared__ double sVw[];   // [L + 1][HD]
    const int L1 = L + 1;
    for (int k = threadIdx.x; k < L1 * HD; k += 256) {
        const int l = k / HD, j = k - l * HD;
        sVw[k] = V[(size_t)l * L1 + j];
    }
    __syncthreads();
    const long long MM = (long long)M * M;
    const int njb = (HD + kWigJB - 1) / kWigJB;
    const long long total = (long long)n_beta * njb * MM;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const long long el = i % MM;   // im1 M + im2
    const long long t = i / MM;
    const int jb = (int)(t % njb) * kWigJB;
    const int ib = (int)(t / njb);
    const int im1 = (int)(el / M), im2 = (int)(el - (long long)im1 * M);
    if (real && im1 > L) return;   // orders m1 < 0 are not read for real volumes
    const int a = im1 <= L ? im1 : im1 - M, b = im2 <= L ? im2 : im2 - M;
    const int l0 = std::max(a < 0 ? -a : a, b < 0 ? -b : b);
    double sb, cb;
    sincos(0.5 * beta[ib], &sb, &cb);
    const double x = cos(beta[ib]);
    double acc[kWigJB];
#pragma unroll
    for (int jj = 0; jj < kWigJB; ++jj) acc[jj] = 0.0;
    auto add = [&](int l, double d) {
        const double *v = sVw + l * HD + jb;
#pragma unroll
        for (int jj = 0; jj < kWigJB; ++jj)
            if (jb + jj < HD) acc[jj] += v[jj] * d;
    };
    double dprev = 0.0, d = wigner_seed(l0, a, b, cb, sb);
    add(l0, d);
    int l = l0;
    if (l0 == 0) {   // d^1_00 = cos(beta); the recurrence below needs l >= 1
        dprev = d;
        d = x;
        l = 1;
        add(1, d);
    }
    const double ab = (double)a * b, a2 = (double)a * a, b2 = (double)b * b;
    double rt = 0.0;   // sqrt((l^2 - a^2)(l^2 - b^2)) at the current l
    if (l < L) {
        const double fl = l;
        rt = sqrt((fl * fl - a2) * (fl * fl - b2));
    }
    for (; l < L; ++l) {
        const double fl = l, fl1 = l + 1;
        const double rt1 = sqrt((fl1 * fl1 - a2) * (fl1 * fl1 - b2));
        const double num = (2.0 * fl + 1.0) * (fl * fl1 * x - ab) * d - fl1 * rt * dprev;
        const double den = fl * rt1;
        dprev = d;
        d = num / den;
        rt = rt1;
        add(l + 1, d);
    }
    R *out = Vd + ((size_t)ib * HD + jb) * MM + el;
#pragma unroll
    for (int jj = 0; jj < kWigJB; ++jj)
        if (jb + jj < HD) out[(size_t)jj * MM] = (R)acc[jj];
}

// offset of degree l in the per-pair step-1 array: sum_{l' < l} (2l' + 1)^2
__host__ __device__ __forceinline__ long long xt_off(int l) { return (long long)l * (2 * l - 1) * (2 * l + 1) / 3; }

constexpr int kXtH = 16;    // ranks staged in LDS per round
constexpr int kXtOut = 8;   // outputs per thread per pass

// step 1, one workgroup per (degree l, pair): Xt_l = As_l^H Bs_l, a
// (2l+1) x (2l+1) product over the H_C principal shells, with the shells'
// degree-l blocks staged through LDS kXtH ranks at a time; real volumes need
// only the rows m1 >= 0 (step 1b reads no others), the rest is left unwritten
template <typename R>
__global__ __launch_bounds__(256) void k_vol_xt(const cx<R> *__restrict__ As, const cx<R> *__restrict__ Bs,
                                                int n_tgt, long long p0, int NC, int HC, long long NXT, int real,
                                                cx<R> *__restrict__ Xt) {
    __shared__ cx<R> sa[kXtH][2 * kVolMaxL32 + 1], sb[kXtH][2 * kVolMaxL32 + 1];
    const int l = blockIdx.x;
    const long long p = blockIdx.y;
    const long long pg = p0 + p;
    const long long a = pg / n_tgt, b = pg - a * n_tgt;
    const int n = 2 * l + 1, base = l * l;
    const int r0 = real ? l : 0, nn = (n - r0) * n;   // outputs: rows m1 + l >= r0
    const cx<R> *Aa = As + (size_t)a * HC * NC + base;
    const cx<R> *Bb = Bs + (size_t)b * HC * NC + base;
    cx<R> *out = Xt + (size_t)p * NXT + xt_off(l) + (size_t)r0 * n;
    for (int o0 = 0; o0 < nn; o0 += 256 * kXtOut) {
        R re[kXtOut], im[kXtOut];
#pragma unroll
        for (int c = 0; c < kXtOut; ++c) re[c] = im[c] = 0;
        for (int h0 = 0; h0 < HC; h0 += kXtH) {
            const int hn = std::min(kXtH, HC - h0);
            __syncthreads();
            for (int i = threadIdx.x; i < hn * n; i += 256) {
                const int h = i / n, m = i - h * n;
                sa[h][m] = Aa[(size_t)(h0 + h) * NC + m];
                sb[h][m] = Bb[(size_t)(h0 + h) * NC + m];
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < kXtOut; ++c) {
                const int o = o0 + c * 256 + threadIdx.x;
                if (o < nn) {
                    const int m1 = r0 + o / n, m2 = o % n;
                    for (int h = 0; h < hn; ++h) {
                        const cx<R> u = sa[h][m1], v = sb[h][m2];
                        re[c] += u.re * v.re + u.im * v.im;   // conj(u) v
                        im[c] += u.re * v.im - u.im * v.re;
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kXtOut; ++c) {
            const int o = o0 + c * 256 + threadIdx.x;
            if (o < nn) out[o] = cx<R>{re[c], im[c]};
        }
    }
}

constexpr int kStep1JB = 16;   // degree ranks accumulated per pass

// step 1b, thread per (pair, m1, m2): Y_j(m1, m2) = sum_{l >= max(|m1|,|m2|)} V[l][j] Xt_l(m1, m2);
// every Xt entry is read once
template <typename R>
__global__ __launch_bounds__(256) void k_vol_step1b(const cx<R> *__restrict__ Xt, int L, int M, int HD, long long NXT,
                                                    const double *__restrict__ V, int nrow, cx<R> *__restrict__ Y) {
    __shared__ R sV[(kVolMaxL32 + 1) * (kVolMaxL32 + 1)];   // [l][j], j < HD
    const int L1 = L + 1;
    for (int i = threadIdx.x; i < L1 * HD; i += 256) {
        const int l = i / HD, j = i - l * HD;
        sV[i] = (R)V[(size_t)l * L1 + j];
    }
    __syncthreads();
    const int MM = M * M;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nrow * M) return;   // nrow = M, or L + 1 for real volumes (orders m1 >= 0)
    const long long p = blockIdx.y;
    const int im1 = i / M, im2 = i - im1 * M;
    const int m1 = im1 <= L ? im1 : im1 - M, m2 = im2 <= L ? im2 : im2 - M;
    const int l0 = std::max(m1 < 0 ? -m1 : m1, m2 < 0 ? -m2 : m2);
    const cx<R> *Xp = Xt + (size_t)p * NXT;
    cx<R> *Yp = Y + (size_t)p * HD * MM;
    for (int j0 = 0; j0 < HD; j0 += kStep1JB) {
        R are[kStep1JB], aim[kStep1JB];
#pragma unroll
        for (int jj = 0; jj < kStep1JB; ++jj) are[jj] = aim[jj] = 0;
        // four degrees' loads in flight at a time (the loop is latency-bound otherwise)
#pragma unroll 4
        for (int l = l0; l <= L; ++l) {
            const int n = 2 * l + 1;
            const cx<R> x = Xp[xt_off(l) + (long long)(m1 + l) * n + (m2 + l)];
#pragma unroll
            for (int jj = 0; jj < kStep1JB; ++jj) {
                if (j0 + jj < HD) {
                    const R vv = sV[l * HD + j0 + jj];
                    are[jj] += vv * x.re;
                    aim[jj] += vv * x.im;
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < kStep1JB; ++jj)
            if (j0 + jj < HD) Yp[(size_t)(j0 + jj) * MM + i] = cx<R>{are[jj], aim[jj]};
    }
}

// (v, i) comes before (w, j): larger value first, then the smaller index
template <typename R>
__device__ __forceinline__ bool vol_before(R v, int i, R w, int j) {
    if (i == 0x7fffffff) return false;
    if (j == 0x7fffffff) return true;
    return v > w || (v == w && i < j);
}

// step 2 for a block of pairs: Xh[p][ib][i] = sum_j Vd[ib][j][i] Y[p][j][i] for i < count
// (count = M^2, or (L+1) M for real volumes: the orders m1 >= 0).  Each thread
// keeps PB pairs x BB angles of one entry in registers, so every Y value is
// read by ceil(n_beta / BB) threads and every table value by ceil(np / PB).
// Workgroups go to the eight XCDs in turn, in launch order: workgroup g serves
// XCD g % 8, which owns the entries [x span, (x + 1) span) and walks them in
// sub-blocks of kStep2Sub entries with every (pair block, angle block) of a
// sub-block launched together, so that its L2 keeps that sub-block's Y and
// table values (2.4 MB at the volume workload) while they are read again.
constexpr int kStep2Sub = 128, kXcds = 8;
template <typename R, int PB, int BB>
__global__ __launch_bounds__(kStep2Sub) void k_vol_step2(const cx<R> *__restrict__ Y, const R *__restrict__ Vd,
                                                         int np, int n_beta, int HD, int MM, int count, int span,
                                                         int npb, int nbb, cx<R> *__restrict__ Xh) {
    const int g = blockIdx.x, xcd = g % kXcds, slot = g / kXcds;
    const int per = npb * nbb, sub = slot / per, rem = slot - sub * per;
    const int pbk = rem / nbb, bbk = rem - pbk * nbb;
    const int off = sub * kStep2Sub + threadIdx.x, i = xcd * span + off;
    if (off >= span || i >= count) return;
    const int pa = pbk * PB, ba = bbk * BB;
    cx<R> acc[PB][BB];
#pragma unroll
    for (int a = 0; a < PB; ++a)
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[a][b] = cx<R>{0, 0};
    for (int j = 0; j < HD; ++j) {
        cx<R> y[PB];
        R v[BB];
#pragma unroll
        for (int a = 0; a < PB; ++a)
            y[a] = pa + a < np ? Y[((size_t)(pa + a) * HD + j) * MM + i] : cx<R>{0, 0};
#pragma unroll
        for (int b = 0; b < BB; ++b) v[b] = ba + b < n_beta ? Vd[((size_t)(ba + b) * HD + j) * MM + i] : R(0);
#pragma unroll
        for (int a = 0; a < PB; ++a)
#pragma unroll
            for (int b = 0; b < BB; ++b) {
                acc[a][b].re += v[b] * y[a].re;
                acc[a][b].im += v[b] * y[a].im;
            }
    }
#pragma unroll
    for (int a = 0; a < PB; ++a)
#pragma unroll
        for (int b = 0; b < BB; ++b)
            if (pa + a < np && ba + b < n_beta) Xh[((size_t)(pa + a) * n_beta + ba + b) * count + i] = acc[a][b];
}

template <typename R>
__device__ __forceinline__ void land_load(const cx<R> *__restrict__ Xp, int count, cx<R> *S, int tid, int nthr) {
    for (int i = tid; i < count; i += nthr) S[i] = Xp[i];
}

template <typename R>
__device__ __forceinline__ void land_twiddles(cx<R> *tw, int M, int tid, int nthr) {
    for (int k = tid; k < M; k += nthr) {
        double s, c;
        sincospi(-2.0 * (double)k / (double)M, &s, &c);
        tw[k] = cx<R>{(R)c, (R)s};
    }
}

// the best of one angle from each thread's candidate (bv, bi; bad: a NaN seen):
// first maximum in m1' M + m2' order, NaN if any value is NaN; rv, ri, rbad
// hold one entry per wave
template <typename R>
__device__ void land_best_reduce(R bv, int bi, int bad, int tid, int nthr, R *rv, int *ri, int *rbad, double *pv,
                                 int32_t *pi) {
    const int lane = tid & 63, wv = tid >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        const R v2 = __shfl_xor(bv, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        if (vol_before(v2, i2, bv, bi)) {
            bv = v2;
            bi = i2;
        }
        bad |= __shfl_xor(bad, o, 64);
    }
    if (lane == 0) {
        rv[wv] = bv;
        ri[wv] = bi;
        rbad[wv] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        for (int x = 1; x < (nthr >> 6); ++x) {
            if (vol_before(rv[x], ri[x], bv, bi)) {
                bv = rv[x];
                bi = ri[x];
            }
            bad |= rbad[x];
        }
        *pv = (bad || bi == 0x7fffffff) ? __builtin_nan("") : (double)bv;
        *pi = bi;
    }
}

// the best Re X of one angle held in LDS and the FULL write
template <typename R>
__device__ void land_epilogue(const cx<R> *S, int MM, cx<R> *Xo, int tid, int nthr, R *rv, int *ri, int *rbad,
                              double *pv, int32_t *pi) {
    R bv = 0;
    int bi = 0x7fffffff, bad = 0;
    for (int i = tid; i < MM; i += nthr) {
        const cx<R> x = S[i];
        if (Xo) Xo[i] = x;
        if (isnan(x.re)) {
            bad = 1;
        } else if (vol_before(x.re, i, bv, bi)) {
            bv = x.re;
            bi = i;
        }
    }
    land_best_reduce<R>(bv, bi, bad, tid, nthr, rv, ri, rbad, pv, pi);
}

// the 16x16x4 matrix-core product of either precision.  Both take
// A[l % 16][l / 16] and B[l / 16][l % 16] from lane l; the lane's four results
// are D rows 4 (l / 16) + r (FP32) or l / 16 + 4 r (FP64), r = 0..3, column l % 16.
template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int lk, int r) { return 4 * lk + r; }
};
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int lk, int r) { return lk + 4 * r; }
};

// Step 3 as two complex matrix products on the matrix cores,
// Xrow = S F, then X = F Xrow (F[a][b] = e^{-2 pi i ab / M}, symmetric), each
// as three real MFMA 16x16x4 products (Gauss: k1 = (Sr + Si) Fr, k2 = Sr (Fi - Fr),
// k3 = Si (Fr + Fi); re = k1 - k3, im = k1 + k2) over 16 x 16 output tiles of
// the order grid padded to NT tiles of 16; the twiddle table holds Fr, Fi - Fr
// and Fr + Fi.  Wave w owns row block w in the first product: it reads only
// that block and overwrites it after its last read, so a wave-level fence
// suffices between read and write.  In the second it owns column block w, and
// the BEST reduction and FULL write take X from its accumulators.
// FP32 plans use the FP32 products, FP64 plans the FP64 ones (Mfma<R>).

// waves per SIMD the complex-mode kernel is compiled for at 7 tiles: LDS holds
// two FP32 workgroups (14 waves per CU) or one FP64 one (7)
template <typename R, int NT>
constexpr int land_cx_waves() { return NT == 7 ? (sizeof(R) == 4 ? 4 : 2) : 1; }

// byte offset of the complex kernel's twiddle table: after the M x M landscape,
// 16-byte aligned
__host__ __device__ inline size_t land_cx_tw_off(int M, size_t cxb) { return ((size_t)M * M * cxb + 15) & ~(size_t)15; }

template <typename R, int NT>
__global__ __launch_bounds__(64 * NT, (land_cx_waves<R, NT>())) void k_vol_land_mfma(
    const cx<R> *__restrict__ Xh, int n_beta, int M, long long p0, cx<R> *__restrict__ Xfull,
    double *__restrict__ part_val, int32_t *__restrict__ part_idx) {
    extern __shared__ __align__(16) unsigned char vol_smem[];
    using V4 = typename Mfma<R>::v4;
    struct T3 {   // twiddle entry: the Gauss operands fr, fi - fr, fr + fi
        R a, b, c;
    };
    cx<R> *S = reinterpret_cast<cx<R> *>(vol_smem);   // [M][M]
    T3 *tw = reinterpret_cast<T3 *>(vol_smem + land_cx_tw_off(M, sizeof(cx<R>)));
    __shared__ R rv[NT];
    __shared__ int ri[NT], rbad[NT];
    constexpr int NTHR = 64 * NT;
    const int ib = blockIdx.x;
    const long long p = blockIdx.y;
    const int MM = M * M, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int k = tid; k < M; k += NTHR) {
        double sn, cs;
        sincospi(-2.0 * (double)k / (double)M, &sn, &cs);
        const R fr = (R)cs, fi = (R)sn;
        tw[k] = T3{fr, fi - fr, fr + fi};
    }
    land_load(Xh + ((size_t)p * n_beta + ib) * MM, MM, S, tid, NTHR);
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    // A rows m1 (first product) or c (second) past M, read clamped to M - 1, and
    // B columns past M only feed outputs that are never written: the loops mask
    // nothing but the orders e >= M of their last step (zero twiddles there)
    const int iac = min(wv * 16 + li, M - 1);
    const int e_main = M & ~3;
    V4 k1[NT], k2[NT], k3[NT];   // Gauss: re = k1 - k3, im = k1 + k2
    int tix[NT], tst[NT];
    auto product = [&](bool rows) {   // rows: S F with A = rows of S; else F (S F) with A = columns
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            k1[t] = V4{0, 0, 0, 0};
            k2[t] = V4{0, 0, 0, 0};
            k3[t] = V4{0, 0, 0, 0};
            const int j = t * 16 + li;   // B column
            tix[t] = (lk * j) % M;       // (e j) mod M for e = lk
            tst[t] = (4 * j) % M;
        }
        auto step = [&](int e0, bool tail) {
            const int e = e0 + lk;
            const int ec = tail ? min(e, M - 1) : e;
            const cx<R> x = rows ? S[iac * M + ec] : S[ec * M + iac];
            const R xs = x.re + x.im;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                T3 f = tw[tix[t]];
                if (tail && e >= M) f = T3{0, 0, 0};
                tix[t] += tst[t];
                if (tix[t] >= M) tix[t] -= M;
                // (xr + i xi)(fr + i fi) with three products
                k1[t] = Mfma<R>::mma(xs, f.a, k1[t]);
                k2[t] = Mfma<R>::mma(x.re, f.b, k2[t]);
                k3[t] = Mfma<R>::mma(x.im, f.c, k3[t]);
            }
        };
        for (int e0 = 0; e0 < e_main; e0 += 4) step(e0, false);
        if (e_main < M) step(e_main, true);
    };
    product(true);
    vol_wave_sync();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int j = t * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = wv * 16 + Mfma<R>::drow(lk, r);
            if (i < M && j < M) S[i * M + j] = cx<R>{k1[t][r] - k3[t][r], k1[t][r] + k2[t][r]};
        }
    }
    __syncthreads();
    product(false);
    // the epilogue from the accumulators: lane values X(m1' = j, m2' = c)
    cx<R> *Xo = Xfull ? Xfull + ((size_t)(p0 + p) * n_beta + ib) * MM : nullptr;
    R bv = 0;
    int bi = 0x7fffffff, bad = 0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int j = t * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = wv * 16 + Mfma<R>::drow(lk, r);
            if (c < M && j < M) {
                const R xre = k1[t][r] - k3[t][r];
                const int i = j * M + c;
                if (Xo) Xo[i] = cx<R>{xre, k1[t][r] + k2[t][r]};
                if (isnan(xre)) {
                    bad = 1;
                } else if (vol_before(xre, i, bv, bi)) {
                    bv = xre;
                    bi = i;
                }
            }
        }
    }
    land_best_reduce<R>(bv, bi, bad, tid, NTHR, rv, ri, rbad, part_val + (size_t)p * n_beta + ib,
                        part_idx + (size_t)p * n_beta + ib);
}


// Real volumes: X-hat(-m1, -m2) = conj X-hat(m1, m2), so only the
// rows m1 = 0..L of X-hat are formed, and X is real:
//   R(m1, k)   = sum_{m2} X-hat(m1, m2) F[m2][k]                      (complex, rows m1 >= 0)
//   X(m1', k)  = sum_{m1 = 0..L} c(m1) Re[F[m1][m1'] R(m1, k)],  c(0) = 1, c(m1 > 0) = 2.
// The first product: wave w computes column tile w for every row block of
// m1 >= 0 (the twiddle fragment is shared by the row blocks); its in-place
// write waits for a workgroup barrier, since every wave reads whole rows.
// The second: wave w owns column block w (as in the complex kernel), two real
// MFMA products per tile (re R x re F - im R x im F), over K = L + 1 orders.
// The BEST reduction and the FULL write take X from the accumulators, so LDS
// holds only the L + 1 rows of m1 >= 0 (about half of the complex kernel's).
// waves per SIMD the real-mode kernel is compiled for at 7 tiles (M = 97 .. 111):
// LDS holds four FP32 workgroups (28 waves per CU) or two FP64 ones (14), which
// 72 and 128 VGPRs respectively let run together
template <typename R, int NT>
constexpr int land_real_waves() { return NT == 7 ? (sizeof(R) == 4 ? 7 : 4) : 1; }

template <typename R, int NT>
__global__ __launch_bounds__(64 * NT, (land_real_waves<R, NT>())) void k_vol_land_mfma_real(const cx<R> *__restrict__ Xh, int n_beta, int M,
                                                                long long p0, cx<R> *__restrict__ Xfull,
                                                                double *__restrict__ part_val,
                                                                int32_t *__restrict__ part_idx) {
    extern __shared__ __align__(16) unsigned char vol_smem[];
    using V4 = typename Mfma<R>::v4;
    cx<R> *S = reinterpret_cast<cx<R> *>(vol_smem);   // [L + 1][M]: X-hat, then R, of the orders m1 >= 0
    __shared__ R rv[NT];
    __shared__ int ri[NT], rbad[NT];
    constexpr int NTHR = 64 * NT;
    constexpr int NRB = (NT * 16 / 2 + 1 + 15) / 16;   // row blocks covering m1 = 0..L, L < 8 NT
    const int ib = blockIdx.x;
    const long long p = blockIdx.y;
    const int MM = M * M, L = M / 2, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    cx<R> *tw = S + (L + 1) * M;
    cx<R> *scr = tw + M;   // [2][M]: rows formed on the vector units
    land_twiddles(tw, M, tid, NTHR);
    land_load(Xh + ((size_t)p * n_beta + ib) * (L + 1) * M, (L + 1) * M, S, tid, NTHR);
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    {   // first product: rows m1 = 0..L, column tile wv
        // One or two rows past the last full block of 16 (L + 1 = 16 n + 1 or
        // 16 n + 2, as at L = 48) would cost a whole block of matrix-core
        // products; the vector units form them first, into the scratch rows:
        // lane (kv, part) sums the orders e = part (mod 4) for column kv, then
        // the four parts add up.
        const int nrem = (L + 1) % 16;
        const bool row_valu = nrem == 1 || nrem == 2;
        const int nrb_run = row_valu ? (L + 1) / 16 : (L + 16) / 16;   // row blocks on the matrix cores
        if (row_valu) {
            const int kv = wv * 16 + (lane >> 2), part = lane & 3;
            for (int i = 0; i < nrem; ++i) {
                const int row = 16 * nrb_run + i;
                R ar = 0, ai = 0;
                if (kv < M) {
                    int ix = (part * kv) % M;
                    const int st = (4 * kv) % M;
                    for (int e = part; e < M; e += 4) {
                        const cx<R> x = S[row * M + e], f = tw[ix];
                        ar += x.re * f.re - x.im * f.im;
                        ai += x.re * f.im + x.im * f.re;
                        ix += st;
                        if (ix >= M) ix -= M;
                    }
                }
                ar += __shfl_xor(ar, 1, 64);
                ai += __shfl_xor(ai, 1, 64);
                ar += __shfl_xor(ar, 2, 64);
                ai += __shfl_xor(ai, 2, 64);
                if (part == 0 && kv < M) scr[i * M + kv] = cx<R>{ar, ai};
            }
        }
        V4 k1[NRB], k2[NRB], k3[NRB];   // Gauss: re = k1 - k3, im = k1 + k2
#pragma unroll
        for (int r = 0; r < NRB; ++r) {
            k1[r] = V4{0, 0, 0, 0};
            k2[r] = V4{0, 0, 0, 0};
            k3[r] = V4{0, 0, 0, 0};
        }
        // Output columns j >= M and rows past L (in a partial last block, whose
        // reads are clamped to row L) only feed outputs that are never written,
        // so the loop masks nothing but the orders e >= M of its last step
        // (their twiddles are zero; the clamped reads stay inside S).
        const int j = wv * 16 + li;
        int tix = (lk * j) % M;
        const int tst = (4 * j) % M;
        int rowo[NRB];
#pragma unroll
        for (int r = 0; r < NRB; ++r) rowo[r] = min(r * 16 + li, L) * M;
        auto step1 = [&](int e0, bool tail) {
            const int e = e0 + lk;
            cx<R> f = tw[tix];
            if (tail && e >= M) f = cx<R>{0, 0};
            tix += tst;
            if (tix >= M) tix -= M;
            const R fr = f.re, fi = f.im, fd = fi - fr, fs = fr + fi;
            const int ec = tail ? min(e, M - 1) : e;
#pragma unroll
            for (int r = 0; r < NRB; ++r) {
                if (r >= nrb_run) break;   // uniform
                const cx<R> x = S[rowo[r] + ec];
                k1[r] = Mfma<R>::mma(x.re + x.im, fr, k1[r]);
                k2[r] = Mfma<R>::mma(x.re, fd, k2[r]);
                k3[r] = Mfma<R>::mma(x.im, fs, k3[r]);
            }
        };
        const int e_main = M & ~3;
        for (int e0 = 0; e0 < e_main; e0 += 4) step1(e0, false);
        if (e_main < M) step1(e_main, true);
        __syncthreads();   // every wave has read its rows
#pragma unroll
        for (int r = 0; r < NRB; ++r) {
            if (r >= nrb_run) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = r * 16 + Mfma<R>::drow(lk, q);
                if (row <= L && j < M) S[row * M + j] = cx<R>{k1[r][q] - k3[r][q], k1[r][q] + k2[r][q]};
            }
        }
        if (row_valu)
            for (int i = tid; i < nrem * M; i += NTHR) S[16 * nrb_run * M + i] = scr[i];
        __syncthreads();
    }
    {   // second product: column block wv, all rows m1' of the output
        V4 acc[NT];
        int tix[NT], tst[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc[t] = V4{0, 0, 0, 0};
            const int j = t * 16 + li;
            tix[t] = (lk * j) % M;
            tst[t] = (4 * j) % M;
        }
        // columns c >= M of R (read clamped to column M - 1) and output rows
        // m1' >= M are never written; only the orders e > L of the last step
        // are masked
        const int iac = min(wv * 16 + li, M - 1);   // column c of R
        auto step2 = [&](int e0, bool tail) {
            const int e = e0 + lk;     // order m1 >= 0
            R xr = 0, xi = 0;
            if (!tail || e <= L) {
                const cx<R> x = S[e * M + iac];
                const R c = e == 0 ? R(1) : R(2);
                xr = c * x.re;
                xi = -c * x.im;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const cx<R> f = tw[tix[t]];
                tix[t] += tst[t];
                if (tix[t] >= M) tix[t] -= M;
                acc[t] = Mfma<R>::mma(xr, f.re, acc[t]);
                acc[t] = Mfma<R>::mma(xi, f.im, acc[t]);
            }
        };
        const int e_main2 = (L + 1) & ~3;
        for (int e0 = 0; e0 < e_main2; e0 += 4) step2(e0, false);
        if (e_main2 < L + 1) step2(e_main2, true);
        // the epilogue from the accumulators: lane values X(m1' = j, m2' = c)
        cx<R> *Xo = Xfull ? Xfull + ((size_t)(p0 + p) * n_beta + ib) * MM : nullptr;
        R bv = 0;
        int bi = 0x7fffffff, bad = 0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = t * 16 + li;   // output row m1'
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = wv * 16 + Mfma<R>::drow(lk, q);
                if (c < M && j < M) {
                    const R x = acc[t][q];
                    const int i = j * M + c;
                    if (Xo) Xo[i] = cx<R>{x, R(0)};
                    if (isnan(x)) {
                        bad = 1;
                    } else if (vol_before(x, i, bv, bi)) {
                        bv = x;
                        bi = i;
                    }
                }
            }
        }
        land_best_reduce<R>(bv, bi, bad, tid, NTHR, rv, ri, rbad, part_val + (size_t)p * n_beta + ib,
                            part_idx + (size_t)p * n_beta + ib);
    }
}

__global__ void k_vol_best(const double *__restrict__ part_val, const int32_t *__restrict__ part_idx, int n_pairs,
                           int n_beta, int M, long long p0, float *__restrict__ best_score,
                           int32_t *__restrict__ best_idx) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pairs) return;
    double bv = 0.0;
    int bb = -1, bi = -1;
    bool bad = false;
    for (int ib = 0; ib < n_beta; ++ib) {
        const double v = part_val[(size_t)p * n_beta + ib];
        if (isnan(v)) {
            bad = true;
            break;
        }
        if (bb < 0 || v > bv) {   // strict: the smaller angle index on ties
            bv = v;
            bb = ib;
            bi = part_idx[(size_t)p * n_beta + ib];
        }
    }
    const size_t o = (size_t)(p0 + p);
    if (best_score) best_score[o] = bad ? __builtin_nanf("") : (float)bv;
    if (best_idx) {
        best_idx[3 * o + 0] = bad ? -1 : bb;
        best_idx[3 * o + 1] = bad ? -1 : bi / M;
        best_idx[3 * o + 2] = bad ? -1 : bi % M;
    }
}

template <typename R>
hipError_t prepare_t(radsvd_vol_plan *p, const VolGrid &g, const void *A, const void *B, const double *U_in,
                     const double *V_in, hipStream_t s) {
    const cx<R> *Ac = reinterpret_cast<const cx<R> *>(A);
    const cx<R> *Bc = reinterpret_cast<const cx<R> *>(B);
    hipLaunchKernelGGL(k_vol_setup, dim3(1), dim3(256), 0, s, g, p->w, p->beta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int L1 = p->L + 1;
    if (U_in) hipLaunchKernelGGL(k_vol_user_mat, dim3(64), dim3(256), 0, s, U_in, p->K, p->HC, p->U, p->lamC);
    else hipLaunchKernelGGL(k_vol_C<R>, dim3(p->K, p->K), dim3(256), 0, s, Bc, p->n_tgt, p->K, p->NC, p->w, p->C);
    if (V_in) hipLaunchKernelGGL(k_vol_user_mat, dim3(64), dim3(256), 0, s, V_in, L1, p->HD, p->V, p->lamD);
    else hipLaunchKernelGGL(k_vol_D<R>, dim3(L1, L1), dim3(256), 0, s, Bc, p->n_tgt, p->K, p->NC, p->L, p->w, p->D);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    {   // the eigendecompositions still to do, in one launch
        const double *C[2];
        int K[2];
        void *log[2];
        double *U[2], *lam[2];
        int n = 0;
        if (!U_in) {
            C[n] = p->C, K[n] = p->K, log[n] = p->logC, U[n] = p->U, lam[n] = p->lamC;
            ++n;
        }
        if (!V_in) {
            C[n] = p->D, K[n] = L1, log[n] = p->logD, U[n] = p->V, lam[n] = p->lamD;
            ++n;
        }
        if (n) e = launch_eig_raw2(n, C, K, log, U, lam, s);
        if (e != hipSuccess) return e;
    }
    const int nbx = (p->NC + 255) / 256;
    const int nhb = (p->HC + kShellHB - 1) / kShellHB;
    const size_t sh_shells = (size_t)p->K * kShellHB * sizeof(double);
    hipLaunchKernelGGL(k_vol_shells<R>, dim3((unsigned)((long long)p->n_vol * nbx), nhb), dim3(256), sh_shells, s,
                       Ac, p->n_vol, p->K, p->NC, p->U, p->HC, p->w, reinterpret_cast<cx<R> *>(p->As));
    hipLaunchKernelGGL(k_vol_shells<R>, dim3((unsigned)((long long)p->n_tgt * nbx), nhb), dim3(256), sh_shells, s,
                       Bc, p->n_tgt, p->K, p->NC, p->U, p->HC, p->w, reinterpret_cast<cx<R> *>(p->Bs));
    const long long nvd = (long long)p->n_beta * ((p->HD + kWigJB - 1) / kWigJB) * p->M * p->M;
    hipLaunchKernelGGL(k_vol_wigner<R>, dim3((unsigned)((nvd + 255) / 256)), dim3(256),
                       (size_t)(p->L + 1) * p->HD * sizeof(double), s, p->beta,
                       p->n_beta, p->L, p->M, p->V, p->HD, p->real, reinterpret_cast<R *>(p->Vd));
    return hipGetLastError();
}

template <typename R, int NT>
hipError_t launch_land_mfma(const radsvd_vol_plan *p, int np, long long p0, cx<R> *Xf, size_t shmem, hipStream_t s) {
    const void *fn = p->real ? (const void *)k_vol_land_mfma_real<R, NT> : (const void *)k_vol_land_mfma<R, NT>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    if (p->real)
        hipLaunchKernelGGL((k_vol_land_mfma_real<R, NT>), dim3(p->n_beta, np), dim3(64 * NT), shmem, s,
                           reinterpret_cast<const cx<R> *>(p->Xh), p->n_beta, p->M, p0, Xf, p->part_val, p->part_idx);
    else
        hipLaunchKernelGGL((k_vol_land_mfma<R, NT>), dim3(p->n_beta, np), dim3(64 * NT), shmem, s,
                           reinterpret_cast<const cx<R> *>(p->Xh), p->n_beta, p->M, p0, Xf, p->part_val, p->part_idx);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_land(const radsvd_vol_plan *p, int np, long long p0, cx<R> *Xf, size_t shmem, hipStream_t s) {
    switch ((p->M + 15) / 16) {   // tiles of 16 orders; M <= 129 (FP32), <= 97 (FP64)
        case 1: return launch_land_mfma<R, 1>(p, np, p0, Xf, shmem, s);
        case 2: return launch_land_mfma<R, 2>(p, np, p0, Xf, shmem, s);
        case 3: return launch_land_mfma<R, 3>(p, np, p0, Xf, shmem, s);
        case 4: return launch_land_mfma<R, 4>(p, np, p0, Xf, shmem, s);
        case 5: return launch_land_mfma<R, 5>(p, np, p0, Xf, shmem, s);
        case 6: return launch_land_mfma<R, 6>(p, np, p0, Xf, shmem, s);
        case 7: return launch_land_mfma<R, 7>(p, np, p0, Xf, shmem, s);
        default:
            if constexpr (sizeof(R) == 4) {
                if ((p->M + 15) / 16 == 8) return launch_land_mfma<R, 8>(p, np, p0, Xf, shmem, s);
                if ((p->M + 15) / 16 == 9) return launch_land_mfma<R, 9>(p, np, p0, Xf, shmem, s);
            }
            return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t align_t(const radsvd_vol_plan *p, int flags, float *best_score, int32_t *best_idx, void *X_full,
                   hipStream_t s) {
    // X-hat of one (pair, angle) and the twiddles; real volumes keep only the orders m1 >= 0,
    // and two scratch rows; the complex kernel's twiddle entries hold three values
    const size_t shmem = p->real ? (size_t)((p->L + 3) * p->M + p->M) * sizeof(cx<R>)
                                 : land_cx_tw_off(p->M, sizeof(cx<R>)) + (size_t)p->M * 3 * sizeof(R);
    const long long n_pairs = (long long)p->n_vol * p->n_tgt;
    const int MM = p->M * p->M;
    cx<R> *Xf = (flags & RADSVD_OUT_FULL) ? reinterpret_cast<cx<R> *>(X_full) : nullptr;
    for (long long p0 = 0; p0 < n_pairs; p0 += p->chunk) {
        const int np = (int)std::min<long long>(p->chunk, n_pairs - p0);
        const long long NXT = xt_off(p->L + 1);
        hipLaunchKernelGGL(k_vol_xt<R>, dim3(p->L + 1, np), dim3(256), 0, s, reinterpret_cast<const cx<R> *>(p->As),
                           reinterpret_cast<const cx<R> *>(p->Bs), p->n_tgt, p0, p->NC, p->HC, NXT, p->real,
                           reinterpret_cast<cx<R> *>(p->Xt));
        const int nrow = p->real ? p->L + 1 : p->M;
        hipLaunchKernelGGL(k_vol_step1b<R>, dim3((nrow * p->M + 255) / 256, np), dim3(256), 0, s,
                           reinterpret_cast<const cx<R> *>(p->Xt), p->L, p->M, p->HD, NXT, p->V, nrow,
                           reinterpret_cast<cx<R> *>(p->Y));
        // step 2: 8 pairs x 8 angles per thread in FP32, 4 x 4 in FP64 (registers)
        constexpr int PB = sizeof(R) == 4 ? 8 : 4;
        const int count = nrow * p->M;
        const int span = (count + kXcds - 1) / kXcds, nsub = (span + kStep2Sub - 1) / kStep2Sub;
        const int npb = (np + PB - 1) / PB, nbb = (p->n_beta + PB - 1) / PB;
        const size_t nwg = (size_t)kXcds * nsub * npb * nbb;   // below 2^26 under the 1 GiB block bound
        if (nwg > 0x7fffffffu) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL((k_vol_step2<R, PB, PB>), dim3((unsigned)nwg), dim3(kStep2Sub), 0, s,
                           reinterpret_cast<const cx<R> *>(p->Y), reinterpret_cast<const R *>(p->Vd), np, p->n_beta,
                           p->HD, MM, count, span, npb, nbb, reinterpret_cast<cx<R> *>(p->Xh));
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = launch_land<R>(p, np, p0, Xf, shmem, s);
        if (e == hipSuccess && (flags & RADSVD_OUT_BEST))
            hipLaunchKernelGGL(k_vol_best, dim3((np + 255) / 256), dim3(256), 0, s, p->part_val, p->part_idx, np,
                               p->n_beta, p->M, p0, best_score, best_idx);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t vol_launch_prepare(radsvd_vol_plan *p, const VolGrid &g, const void *A, const void *B,
                              const double *U_in, const double *V_in, hipStream_t s) {
    if (p->prec == RADSVD_FP64) return prepare_t<double>(p, g, A, B, U_in, V_in, s);
    return prepare_t<float>(p, g, A, B, U_in, V_in, s);
}

hipError_t vol_launch_align(const radsvd_vol_plan *p, int flags, float *best_score, int32_t *best_idx,
                            void *X_full, hipStream_t s) {
    if (p->prec == RADSVD_FP64) return align_t<double>(p, flags, best_score, best_idx, X_full, s);
    return align_t<float>(p, flags, best_score, best_idx, X_full, s);
}

}  // namespace radsvd
