// Target-averaged kernel C (paper section 3.4, with the single-target kernel
// of section 3.3 and its Plancherel simplification, the q = 0 term excluded):
//
//   C[r][r'] = eta_r eta_r' / N_B * Re[ sum_{b,j} conj(B[b][r][j]) B[b][r'][j]
//                                       - (1/Q) sum_b conj(S[b][r]) S[b][r'] ],
//   S[b][r] = sum_j B[b][r][j]
//
// i.e. the q != 0 sum of the unitary angular spectra, evaluated in psi-space
// by the 1-D Plancherel identity.  The paper's positive constant factor is
// dropped (principal vectors are unchanged).  Everything accumulates in FP64.
// The Gram sum is split over target ranges; partial Gram matrices are reduced
// in a fixed order (deterministic).
//
// With a Gaussian translation prior (sigma > 0, the translation- and
// rotation-averaged objective of section 5) the two terms are weighted
// apart: E+(k_r, k_r') = exp(-sigma^2 (k_r - k_r')^2 / 2) on the full sum and
// E-(k_r) E-(k_r'), E-(k) = exp(-sigma^2 k^2 / 2), on the q = 0 term.  (The
// paper writes E- with the modified Bessel functions of order -1/2 and +1/2;
// both are elementary, sqrt(2 / (pi x)) cosh x and sinh x, and the product
// reduces to this exponential.)  Written as E+ times the q != 0 Gram plus
// (E+ - E- E-) times the q = 0 Gram, so sigma = 0 keeps the plain kernel.
#include "common.h"
#include "internal.h"

namespace radsvd {

template <typename R>
__global__ __launch_bounds__(256) void k_ringsum(const cx<R> *__restrict__ B, int n_tgt, int K, int Q,
                                                 double *__restrict__ S) {
    // one wavefront per (b, r)
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= n_tgt * K) return;
    const cx<R> *row = B + (size_t)wave * Q;
    double re = 0.0, im = 0.0;
    for (int j = lane; j < Q; j += 64) {
        re += (double)row[j].re;
        im += (double)row[j].im;
    }
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
    }
    if (lane == 0) {
        S[2 * (size_t)wave] = re;
        S[2 * (size_t)wave + 1] = im;
    }
}

// Partial Gram over targets b in [b0, b1): P[split][r][r'] =
// sum_b ( sum_j Re conj(B[b][r][j]) B[b][r'][j] - Re conj(S[b][r]) S[b][r'] / Q ),
// the q != 0 part of each target's term, for the 32x32 regions on and above
// the diagonal (the finalisation reads r <= r' only).  Real FP64 GEMM on
// v_mfma_f64_16x16x4f64 over the depth (b, j, re|im): a lane loads two
// complex samples (4 reals) of its row and feeds them to four depth steps;
// rows and columns use the same depth order, so the sum is the Gram entry.
// One workgroup per (region, target split); its four waves take every fourth
// target and add their sums in LDS in a fixed order.  Products of FP32 inputs
// are exact in FP64; everything accumulates in FP64.
template <typename R>
__global__ __launch_bounds__(256) void k_gram_partial(const cx<R> *__restrict__ B, const double *__restrict__ S,
                                                      int n_tgt, int K, int Q, int b_per_split,
                                                      double *__restrict__ P) {
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    __shared__ double red[3][16][64];
    const int NRB = (K + 31) / 32;
    // region index -> (ri, ci), ri <= ci, row-major over the upper triangle
    int ri = 0, rem = blockIdx.x;
    while (rem >= NRB - ri) {
        rem -= NRB - ri;
        ++ri;
    }
    const int ci = ri + rem;
    const int split = blockIdx.y;
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int r16 = l & 15, g = l >> 4;
    int rowA[2], rowB[2];
    bool okA[2], okB[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int ra = ri * 32 + 16 * i + r16, cb = ci * 32 + 16 * i + r16;
        okA[i] = ra < K;
        okB[i] = cb < K;
        rowA[i] = okA[i] ? ra : K - 1;
        rowB[i] = okB[i] ? cb : K - 1;
    }
    f64x4 acc[2][2], accS[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
            accS[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
        }
    const int b0 = split * b_per_split;
    const int b1 = min(n_tgt, b0 + b_per_split);
    // lane g of a chunk of 8 samples holds samples 2 g and 2 g + 1 (Q is even, so
    // both or neither are in range; rows past K and samples past Q read a valid
    // address and feed zeros)
    auto load4 = [&](const cx<R> *row, int j, bool ok, double (&v)[4]) __attribute__((always_inline)) {
        const bool use = ok && j < Q;
        const cx<R> *src = row + (j < Q ? j : Q - 2);
        const cx<R> x0 = src[0], x1 = src[1];
        v[0] = use ? (double)x0.re : 0.0;
        v[1] = use ? (double)x0.im : 0.0;
        v[2] = use ? (double)x1.re : 0.0;
        v[3] = use ? (double)x1.im : 0.0;
    };
    for (int b = b0 + w; b < b1; b += 4) {
        const cx<R> *Bb = B + (size_t)b * K * Q;
        const cx<R> *pa0 = Bb + (size_t)rowA[0] * Q, *pa1 = Bb + (size_t)rowA[1] * Q;
        const cx<R> *pb0 = Bb + (size_t)rowB[0] * Q, *pb1 = Bb + (size_t)rowB[1] * Q;
        // the next chunk is loaded while the current one feeds the MFMAs
        double a0[4], a1[4], c0[4], c1[4];
        load4(pa0, 2 * g, okA[0], a0);
        load4(pa1, 2 * g, okA[1], a1);
        load4(pb0, 2 * g, okB[0], c0);
        load4(pb1, 2 * g, okB[1], c1);
        for (int j0 = 0; j0 < Q; j0 += 8) {
            double na0[4], na1[4], nc0[4], nc1[4];
            const int jn = j0 + 8 + 2 * g;
            load4(pa0, jn, okA[0], na0);
            load4(pa1, jn, okA[1], na1);
            load4(pb0, jn, okB[0], nc0);
            load4(pb1, jn, okB[1], nc1);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], c0[s], acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], c1[s], acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], c0[s], acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], c1[s], acc[1][1], 0, 0, 0);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                a0[s] = na0[s];
                a1[s] = na1[s];
                c0[s] = nc0[s];
                c1[s] = nc1[s];
            }
        }
    }
    // the q = 0 terms: depth (b, re|im), lane group g -> target b + (g >> 1), part g & 1
    for (int bb = b0 + 2 * w; bb < b1; bb += 8) {
        const int b = bb + (g >> 1), part = g & 1;
        const bool okb = b < b1;
        const double *sb = S + (size_t)(okb ? b : b0) * K * 2;
        double sa[2], sc[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            sa[i] = (okb && okA[i]) ? sb[2 * rowA[i] + part] : 0.0;
            sc[i] = (okb && okB[i]) ? sb[2 * rowB[i] + part] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
                accS[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[i], sc[jj], accS[i][jj], 0, 0, 0);
    }
    // lane layout of the 16x16 FP64 output: element v of lane l is row l / 16 + 4 v, column l % 16
    const double iq = 1.0 / (double)Q;
    double out[16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int v = 0; v < 4; ++v) out[(i * 2 + jj) * 4 + v] = acc[i][jj][v] - accS[i][jj][v] * iq;
    // waves 1..3 hand their sums to wave 0, which adds them in order
    if (w > 0) {
#pragma unroll
        for (int e = 0; e < 16; ++e) red[w - 1][e][l] = out[e];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            double v = out[e];
            v += red[0][e][l];
            v += red[1][e][l];
            v += red[2][e][l];
            const int i = e >> 3, jj = (e >> 2) & 1, vv = e & 3;
            const int r = ri * 32 + 16 * i + g + 4 * vv, c = ci * 32 + 16 * jj + r16;
            if (r < K && c < K) P[((size_t)split * K + r) * K + c] = v;
        }
    }
}

// G0[r][c] = sum_b Re conj(S[b][r]) S[b][c] (the targets' q = 0 terms times Q),
// for r <= c; 16 x 16 entries per workgroup, 64 targets per LDS chunk
__global__ __launch_bounds__(256) void k_ring_gram(const double *__restrict__ S, int n_tgt, int K,
                                                   double *__restrict__ G0) {
    __shared__ double sr[64][16][2], sc[64][16][2];
    const int r0 = blockIdx.x * 16, c0 = blockIdx.y * 16;
    if (r0 > c0 + 15) return;   // below the diagonal (uniform per workgroup)
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    double acc = 0.0;
    for (int b0 = 0; b0 < n_tgt; b0 += 64) {
        for (int i = threadIdx.x; i < 64 * 16; i += 256) {
            const int bb = i >> 4, j = i & 15, b = b0 + bb;
            const bool okr = b < n_tgt && r0 + j < K, okc = b < n_tgt && c0 + j < K;
            sr[bb][j][0] = okr ? S[2 * ((size_t)b * K + r0 + j)] : 0.0;
            sr[bb][j][1] = okr ? S[2 * ((size_t)b * K + r0 + j) + 1] : 0.0;
            sc[bb][j][0] = okc ? S[2 * ((size_t)b * K + c0 + j)] : 0.0;
            sc[bb][j][1] = okc ? S[2 * ((size_t)b * K + c0 + j) + 1] : 0.0;
        }
        __syncthreads();
        for (int bb = 0; bb < 64; ++bb) acc += sr[bb][tr][0] * sc[bb][tc][0] + sr[bb][tr][1] * sc[bb][tc][1];
        __syncthreads();
    }
    if (r0 + tr < K && c0 + tc < K) G0[(size_t)(r0 + tr) * K + c0 + tc] = acc;
}

__global__ void k_C_finalize(const double *__restrict__ P, int nsplit, int n_tgt, int K, int Q,
                             const double *__restrict__ eta, const double *__restrict__ kr, double sigma,
                             const double *__restrict__ G0, double *__restrict__ C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * K) return;
    const int r = i / K, c = i - r * K;
    // symmetric by construction: evaluate the (min, max) entry for both
    const int a = r < c ? r : c, bb = r < c ? c : r;
    double g = 0.0;
    for (int s = 0; s < nsplit; ++s) g += P[((size_t)s * K + a) * K + bb];
    if (sigma > 0.0) {
        const double s2 = sigma * sigma, d = kr[a] - kr[bb];
        const double ep = exp(-0.5 * s2 * d * d);
        const double em2 = exp(-0.5 * s2 * (kr[a] * kr[a] + kr[bb] * kr[bb]));
        g = ep * g + (ep - em2) * G0[(size_t)a * K + bb] / (double)Q;
    }
    C[i] = eta[a] * eta[bb] * g / (double)n_tgt;
}

hipError_t launch_kernel_C(radsvd_plan *p, hipStream_t s) {
    const int K = p->K, Q = p->Q, nb = p->n_tgt;
    const int waves = nb * K;
    const int nrb = (K + 31) / 32, nreg = nrb * (nrb + 1) / 2;
    const int nsplit = p->gram_nsplit;
    const int bps = (nb + nsplit - 1) / nsplit;
    if (p->prec == RADSVD_FP64) {
        const cx<double> *B = reinterpret_cast<const cx<double> *>(p->B_polar);
        hipLaunchKernelGGL(k_ringsum<double>, dim3((waves + 3) / 4), dim3(256), 0, s, B, nb, K, Q,
                           p->ringsum);
        hipLaunchKernelGGL(k_gram_partial<double>, dim3(nreg, nsplit), dim3(256), 0, s, B,
                           p->ringsum, nb, K, Q, bps, p->gram_part);
    } else {
        const cx<float> *B = reinterpret_cast<const cx<float> *>(p->B_polar);
        hipLaunchKernelGGL(k_ringsum<float>, dim3((waves + 3) / 4), dim3(256), 0, s, B, nb, K, Q,
                           p->ringsum);
        hipLaunchKernelGGL(k_gram_partial<float>, dim3(nreg, nsplit), dim3(256), 0, s, B,
                           p->ringsum, nb, K, Q, bps, p->gram_part);
    }
    if (p->sigma_delta > 0.0)
        hipLaunchKernelGGL(k_ring_gram, dim3((K + 15) / 16, (K + 15) / 16), dim3(256), 0, s, p->ringsum, nb, K,
                           p->ring_gram);
    hipLaunchKernelGGL(k_C_finalize, dim3((K * K + 255) / 256), dim3(256), 0, s, p->gram_part, nsplit, nb, K, Q,
                       p->d_eta, p->d_k, p->sigma_delta, p->ring_gram, p->C);
    return hipGetLastError();
}

}  // namespace radsvd
