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
// the q != 0 part of each target's term.  64x64 output tile per block,
// 4x4 outputs per thread; the contraction index (b, j) is staged through LDS
// in chunks of 16 angles.
template <typename R>
__global__ __launch_bounds__(256) void k_gram_partial(const cx<R> *__restrict__ B, const double *__restrict__ S,
                                                      int n_tgt, int K, int Q, int b_per_split,
                                                      double *__restrict__ P) {
    constexpr int TT = 64, CH = 16;
    __shared__ double sre[2][TT][CH + 1];
    __shared__ double sim[2][TT][CH + 1];
    const int tr = blockIdx.x, tc = blockIdx.y, split = blockIdx.z;
    const int r0 = tr * TT, c0 = tc * TT;
    const int tid = threadIdx.x;
    const int ty = tid / 16, tx = tid % 16;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const int b0 = split * b_per_split;
    const int b1 = min(n_tgt, b0 + b_per_split);
    for (int b = b0; b < b1; ++b) {
        const cx<R> *Bb = B + (size_t)b * K * Q;
        for (int j0 = 0; j0 < Q; j0 += CH) {
            __syncthreads();
            for (int i = tid; i < 2 * TT * CH; i += 256) {
                const int side = i / (TT * CH);
                const int rem = i - side * TT * CH;
                const int rr = rem / CH, jj = rem - rr * CH;
                const int row = (side == 0 ? r0 : c0) + rr;
                const int j = j0 + jj;
                cx<R> v = {(R)0, (R)0};
                if (row < K && j < Q) v = Bb[(size_t)row * Q + j];
                sre[side][rr][jj] = (double)v.re;
                sim[side][rr][jj] = (double)v.im;
            }
            __syncthreads();
            for (int jj = 0; jj < CH; ++jj) {
                double ar[4], ai[4], br[4], bi[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    ar[i] = sre[0][ty * 4 + i][jj];
                    ai[i] = sim[0][ty * 4 + i][jj];
                    br[i] = sre[1][tx * 4 + i][jj];
                    bi[i] = sim[1][tx * 4 + i][jj];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] += ar[i] * br[j] + ai[i] * bi[j];
            }
        }
        // the q = 0 term of target b: Re conj(S[r]) S[r'] / Q
        const double *sb = S + (size_t)b * K * 2;
        const double iq = 1.0 / (double)Q;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = min(r0 + ty * 4 + i, K - 1);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = min(c0 + tx * 4 + j, K - 1);
                acc[i][j] -= (sb[2 * r] * sb[2 * c] + sb[2 * r + 1] * sb[2 * c + 1]) * iq;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + ty * 4 + i, c = c0 + tx * 4 + j;
            if (r < K && c < K) P[((size_t)split * K + r) * K + c] = acc[i][j];
        }
}

__global__ void k_C_finalize(const double *__restrict__ P, int nsplit, int n_tgt, int K,
                             const double *__restrict__ eta, double *__restrict__ C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * K) return;
    const int r = i / K, c = i - r * K;
    // symmetric by construction: evaluate the (min, max) entry for both
    const int a = r < c ? r : c, bb = r < c ? c : r;
    double g = 0.0;
    for (int s = 0; s < nsplit; ++s) g += P[((size_t)s * K + a) * K + bb];
    C[i] = eta[a] * eta[bb] * g / (double)n_tgt;
}

hipError_t launch_kernel_C(radsvd_plan *p, hipStream_t s) {
    const int K = p->K, Q = p->Q, nb = p->n_tgt;
    const int waves = nb * K;
    const int tiles = (K + 63) / 64;
    const int nsplit = p->gram_nsplit;
    const int bps = (nb + nsplit - 1) / nsplit;
    if (p->prec == RADSVD_FP64) {
        const cx<double> *B = reinterpret_cast<const cx<double> *>(p->B_polar);
        hipLaunchKernelGGL(k_ringsum<double>, dim3((waves + 3) / 4), dim3(256), 0, s, B, nb, K, Q,
                           p->ringsum);
        hipLaunchKernelGGL(k_gram_partial<double>, dim3(tiles, tiles, nsplit), dim3(256), 0, s, B,
                           p->ringsum, nb, K, Q, bps, p->gram_part);
    } else {
        const cx<float> *B = reinterpret_cast<const cx<float> *>(p->B_polar);
        hipLaunchKernelGGL(k_ringsum<float>, dim3((waves + 3) / 4), dim3(256), 0, s, B, nb, K, Q,
                           p->ringsum);
        hipLaunchKernelGGL(k_gram_partial<float>, dim3(tiles, tiles, nsplit), dim3(256), 0, s, B,
                           p->ringsum, nb, K, Q, bps, p->gram_part);
    }
    hipLaunchKernelGGL(k_C_finalize, dim3((K * K + 255) / 256), dim3(256), 0, s, p->gram_part, nsplit, nb, K,
                       p->d_eta, p->C);
    return hipGetLastError();
}

}  // namespace radsvd
