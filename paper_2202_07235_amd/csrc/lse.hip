// lse_img[a] = log sum_b exp(lse_pair[a][b]): one workgroup per image, a
// fixed-order two-pass (max, then sum) reduction, hence deterministic.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace radsvd {

__global__ __launch_bounds__(256) void k_lse_img(const float *__restrict__ lp, int n_tgt,
                                                 float *__restrict__ out) {
    __shared__ float red[4];
    __shared__ int rnan[4];
    const int a = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const float *row = lp + (size_t)a * n_tgt;
    float mx = -INFINITY;
    int nan_seen = 0;
    for (int b = tid; b < n_tgt; b += blockDim.x) {
        const float v = row[b];
        if (isnan(v)) nan_seen = 1;
        else mx = fmaxf(mx, v);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        nan_seen |= __shfl_xor(nan_seen, o, 64);
    }
    if (lane == 0) {
        red[w] = mx;
        rnan[w] = nan_seen;
    }
    __syncthreads();
    float bmx = red[0];
    int anynan = rnan[0];
    for (int i = 1; i < 4; ++i) {
        bmx = fmaxf(bmx, red[i]);
        anynan |= rnan[i];
    }
    __syncthreads();
    float s = 0.f;
    for (int b = tid; b < n_tgt; b += blockDim.x) s += expf(row[b] - bmx);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) red[w] = s;
    __syncthreads();
    if (tid == 0) {
        const float tot = red[0] + red[1] + red[2] + red[3];
        out[a] = anynan ? NAN : bmx + logf(tot);
    }
}

hipError_t launch_lse_img(int n_img, int n_tgt, const float *lse_pair, float *lse_img, hipStream_t s) {
    hipLaunchKernelGGL(k_lse_img, dim3(n_img), dim3(256), 0, s, lse_pair, n_tgt, lse_img);
    return hipGetLastError();
}

}  // namespace radsvd
