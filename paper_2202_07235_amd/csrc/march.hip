// Principal-mode marching and the landscape quality measures of the paper.
//
// Marching (section 5): a low rank H gives a coarse landscape of every pair;
// the best-scoring targets of each image are then evaluated again at a higher
// rank (align_pairs_list).  k_top_targets picks those candidates.
//
// Quality (section 3.5): for an approximate landscape X_est (low rank) and the
// full one X_ref, the relative error in the Frobenius norm over the whole
// array, the correlation over the whole array, and per pair the true
// percentile f of the approximate alignment: the fraction of the pair's
// X_ref values (over its whole landscape) that are <= X_ref at the argmax of
// X_est.  A wave per pair for short landscapes, a workgroup per pair for long
// ones.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace radsvd {

// (v, i) precedes (w, j) in the candidate order: larger score first, then the
// smaller target; NaN never precedes a number
__device__ __forceinline__ bool cand_before(float v, int i, float w, int j) {
    const bool nv = isnan(v), nw = isnan(w);
    if (nv != nw) return nw;
    if (!nv && v != w) return v > w;
    return i < j;
}

// One workgroup per image: k passes, each taking the first entry (in the
// candidate order) after the previous pick.  Entries with a NaN score are never
// picked; slots beyond the finite entries get -1.
__global__ __launch_bounds__(256) void k_top_targets(const float *__restrict__ score, int n_tgt, int k,
                                                     int32_t *__restrict__ cand) {
    __shared__ float sv[4];
    __shared__ int si[4];
    const int a = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const float *row = score + (size_t)a * n_tgt;
    float pv = INFINITY;
    int pi = -1;   // previous pick; everything precedes (+inf, -1) except NaN
    for (int c = 0; c < k; ++c) {
        float bv = NAN;
        int bi = 0x7fffffff;
        for (int b = tid; b < n_tgt; b += blockDim.x) {
            const float v = row[b];
            if (isnan(v)) continue;
            const bool after = (c == 0) ? true : cand_before(pv, pi, v, b);
            if (after && cand_before(v, b, bv, bi)) {
                bv = v;
                bi = b;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const float v2 = __shfl_xor(bv, o, 64);
            const int i2 = __shfl_xor(bi, o, 64);
            if (cand_before(v2, i2, bv, bi)) {
                bv = v2;
                bi = i2;
            }
        }
        if (lane == 0) {
            sv[w] = bv;
            si[w] = bi;
        }
        __syncthreads();
        bv = sv[0];
        bi = si[0];
        for (int x = 1; x < (int)(blockDim.x >> 6); ++x)
            if (cand_before(sv[x], si[x], bv, bi)) {
                bv = sv[x];
                bi = si[x];
            }
        __syncthreads();
        const bool found = !isnan(bv) && bi < n_tgt;
        if (tid == 0) cand[(size_t)a * k + c] = found ? bi : -1;
        if (!found) {
            for (int c2 = c + 1 + tid; c2 < k; c2 += blockDim.x) cand[(size_t)a * k + c2] = -1;
            return;   // uniform: every thread read the same bv, bi
        }
        pv = bv;
        pi = bi;
    }
}

template <typename R>
__device__ __forceinline__ double re_at(const R *X, size_t i) {
    return (double)X[2 * i];   // complex interleaved: the real part
}

// One wave per pair: f[pair], and the pair's sums
// stats[pair] = {sum e^2 - 2 e r + r^2, sum r^2, sum e, sum r, sum e^2, sum e r} of the real parts.
template <typename R>
__global__ __launch_bounds__(256) void k_landscape_pair_stats(const R *__restrict__ Xe, const R *__restrict__ Xr,
                                                              long long n_pairs, int len, float *__restrict__ f,
                                                              double *__restrict__ stats) {
    const int lane = threadIdx.x & 63;
    for (long long pair = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); pair < n_pairs;
         pair += (long long)gridDim.x * 4) {
        const size_t base = (size_t)pair * len;
        // argmax of X_est (ties: smallest index; a non-finite value makes f NaN)
        double bv = -INFINITY;
        int bi = 0x7fffffff;
        int bad = 0;
        double sd = 0, srr = 0, se = 0, sr = 0, see = 0, ser = 0;
        for (int i = lane; i < len; i += 64) {
            const double e = re_at(Xe, base + i), r = re_at(Xr, base + i);
            if (!isfinite(e) || !isfinite(r)) bad = 1;
            if (e > bv) {
                bv = e;
                bi = i;
            }
            const double d = e - r;
            sd += d * d;
            srr += r * r;
            se += e;
            sr += r;
            see += e * e;
            ser += e * r;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(bv, o, 64);
            const int i2 = __shfl_xor(bi, o, 64);
            if (v2 > bv || (v2 == bv && i2 < bi)) {
                bv = v2;
                bi = i2;
            }
            bad |= __shfl_xor(bad, o, 64);
            sd += __shfl_xor(sd, o, 64);
            srr += __shfl_xor(srr, o, 64);
            se += __shfl_xor(se, o, 64);
            sr += __shfl_xor(sr, o, 64);
            see += __shfl_xor(see, o, 64);
            ser += __shfl_xor(ser, o, 64);
        }
        // fraction of X_ref values <= X_ref at that argmax
        const double thr = bad ? 0.0 : re_at(Xr, base + bi);
        int cnt = 0;
        if (!bad)
            for (int i = lane; i < len; i += 64) cnt += re_at(Xr, base + i) <= thr ? 1 : 0;
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) {
            f[pair] = bad ? NAN : (float)((double)cnt / (double)len);
            double *st = stats + 6 * (size_t)pair;
            st[0] = sd;
            st[1] = srr;
            st[2] = se;
            st[3] = sr;
            st[4] = see;
            st[5] = ser;
        }
    }
}

// The same per-pair measures for long landscapes (volume landscapes hold
// n_beta M^2 values per pair, far more than one wave should scan): one
// 512-thread workgroup per pair, each thread a strided set of indices, the
// partial results combined in fixed order (lanes by the xor tree, then waves
// in index order).
constexpr int kLongStatsThreads = 512;
constexpr int kLongLandscape = 16384;   // from this length on, a workgroup per pair

template <typename R>
__global__ __launch_bounds__(kLongStatsThreads) void k_landscape_pair_stats_long(
    const R *__restrict__ Xe, const R *__restrict__ Xr, long long n_pairs, int len, float *__restrict__ f,
    double *__restrict__ stats) {
    constexpr int NW = kLongStatsThreads / 64;
    __shared__ double sv[NW][6];
    __shared__ double sb[NW];
    __shared__ int si[NW], sbad[NW], scnt[NW];
    __shared__ double sthr;
    __shared__ int sbad_all;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (long long pair = blockIdx.x; pair < n_pairs; pair += gridDim.x) {
        const size_t base = (size_t)pair * len;
        double bv = -INFINITY;
        int bi = 0x7fffffff;
        int bad = 0;
        double sd = 0, srr = 0, se = 0, sr = 0, see = 0, ser = 0;
        for (int i = tid; i < len; i += kLongStatsThreads) {
            const double e = re_at(Xe, base + i), r = re_at(Xr, base + i);
            if (!isfinite(e) || !isfinite(r)) bad = 1;
            if (e > bv) {
                bv = e;
                bi = i;
            }
            const double d = e - r;
            sd += d * d;
            srr += r * r;
            se += e;
            sr += r;
            see += e * e;
            ser += e * r;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(bv, o, 64);
            const int i2 = __shfl_xor(bi, o, 64);
            if (v2 > bv || (v2 == bv && i2 < bi)) {
                bv = v2;
                bi = i2;
            }
            bad |= __shfl_xor(bad, o, 64);
            sd += __shfl_xor(sd, o, 64);
            srr += __shfl_xor(srr, o, 64);
            se += __shfl_xor(se, o, 64);
            sr += __shfl_xor(sr, o, 64);
            see += __shfl_xor(see, o, 64);
            ser += __shfl_xor(ser, o, 64);
        }
        if (lane == 0) {
            sb[w] = bv;
            si[w] = bi;
            sbad[w] = bad;
            sv[w][0] = sd;
            sv[w][1] = srr;
            sv[w][2] = se;
            sv[w][3] = sr;
            sv[w][4] = see;
            sv[w][5] = ser;
        }
        __syncthreads();
        if (tid == 0) {
            double tv = sb[0];
            int ti = si[0], tb = sbad[0];
            double acc[6] = {sv[0][0], sv[0][1], sv[0][2], sv[0][3], sv[0][4], sv[0][5]};
#pragma unroll 1
            for (int x = 1; x < NW; ++x) {
                if (sb[x] > tv || (sb[x] == tv && si[x] < ti)) {
                    tv = sb[x];
                    ti = si[x];
                }
                tb |= sbad[x];
                for (int k = 0; k < 6; ++k) acc[k] += sv[x][k];
            }
            double *st = stats + 6 * (size_t)pair;
            for (int k = 0; k < 6; ++k) st[k] = acc[k];
            sbad_all = tb;
            sthr = tb ? 0.0 : re_at(Xr, base + ti);
        }
        __syncthreads();
        const int allbad = sbad_all;
        const double thr = sthr;
        int cnt = 0;
        if (!allbad)
            for (int i = tid; i < len; i += kLongStatsThreads) cnt += re_at(Xr, base + i) <= thr ? 1 : 0;
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) scnt[w] = cnt;
        __syncthreads();
        if (tid == 0) {
            long long c = 0;
#pragma unroll 1
            for (int x = 0; x < NW; ++x) c += scnt[x];
            f[pair] = allbad ? NAN : (float)((double)c / (double)len);
        }
        __syncthreads();   // the shared slots are reused by the next pair
    }
}

// summary = {relative Frobenius error, correlation, mean f} from the pair sums,
// reduced in pair order by one workgroup (each thread a contiguous range,
// then the ranges in thread order)
__global__ __launch_bounds__(256) void k_landscape_summary(const double *__restrict__ stats,
                                                           const float *__restrict__ f, long long n_pairs, int len,
                                                           double *__restrict__ summary) {
    __shared__ double part[256][7];
    const int tid = threadIdx.x;
    const long long per = (n_pairs + 255) / 256;
    const long long p0 = std::min(n_pairs, per * tid), p1 = std::min(n_pairs, p0 + per);
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (long long p = p0; p < p1; ++p) {
        for (int k = 0; k < 6; ++k) acc[k] += stats[6 * p + k];
        acc[6] += (double)f[p];
    }
    for (int k = 0; k < 7; ++k) part[tid][k] = acc[k];
    __syncthreads();
    if (tid == 0) {
        double s[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int x = 0; x < 256; ++x)
            for (int k = 0; k < 7; ++k) s[k] += part[x][k];
        const double N = (double)n_pairs * len;
        const double cov = s[5] - s[2] * s[3] / N;
        const double ve = s[4] - s[2] * s[2] / N, vr = s[1] - s[3] * s[3] / N;
        summary[0] = sqrt(s[0] / s[1]);
        summary[1] = cov / sqrt(ve * vr);
        summary[2] = s[6] / (double)n_pairs;
    }
}

hipError_t launch_top_targets(int n_img, int n_tgt, const float *score, int k, int32_t *cand, hipStream_t s) {
    hipLaunchKernelGGL(k_top_targets, dim3(n_img), dim3(256), 0, s, score, n_tgt, k, cand);
    return hipGetLastError();
}

hipError_t launch_landscape_metrics(long long n_pairs, int len, const void *X_est, const void *X_ref, int fp64,
                                    float *f, double *stats, double *summary, hipStream_t s) {
    if (len >= kLongLandscape) {
        const int blocks = (int)std::min<long long>(n_pairs, 1 << 20);
        if (fp64)
            hipLaunchKernelGGL(k_landscape_pair_stats_long<double>, dim3(blocks), dim3(kLongStatsThreads), 0, s,
                               reinterpret_cast<const double *>(X_est), reinterpret_cast<const double *>(X_ref),
                               n_pairs, len, f, stats);
        else
            hipLaunchKernelGGL(k_landscape_pair_stats_long<float>, dim3(blocks), dim3(kLongStatsThreads), 0, s,
                               reinterpret_cast<const float *>(X_est), reinterpret_cast<const float *>(X_ref),
                               n_pairs, len, f, stats);
    } else {
        const int blocks = (int)std::min<long long>((n_pairs + 3) / 4, 1 << 20);
        if (fp64)
            hipLaunchKernelGGL(k_landscape_pair_stats<double>, dim3(blocks), dim3(256), 0, s,
                               reinterpret_cast<const double *>(X_est), reinterpret_cast<const double *>(X_ref),
                               n_pairs, len, f, stats);
        else
            hipLaunchKernelGGL(k_landscape_pair_stats<float>, dim3(blocks), dim3(256), 0, s,
                               reinterpret_cast<const float *>(X_est), reinterpret_cast<const float *>(X_ref),
                               n_pairs, len, f, stats);
    }
    hipLaunchKernelGGL(k_landscape_summary, dim3(1), dim3(256), 0, s, stats, f, n_pairs, len, summary);
    return hipGetLastError();
}

}  // namespace radsvd
