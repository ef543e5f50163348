// Internal plan and launchers of rotational volume alignment (paper section 4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "radsvd.h"

namespace radsvd {

constexpr int kVolMaxK = 128;
constexpr int kVolMaxL32 = 64;    // FP32: the M x M landscape of one angle fits LDS up to M = 129
constexpr int kVolMaxL64 = 48;    // FP64: up to M = 97
constexpr int kVolMaxM = 2 * kVolMaxL32 + 1;
constexpr int kVolMaxBeta = 256;
constexpr int kVolMaxChunk = 32768;               // pairs per block of pairs (grid y)
constexpr size_t kVolChunkBytes = size_t(1) << 30;

struct VolGrid {   // host arrays handed over as kernel arguments
    int K, n_beta;
    double w[kVolMaxK];
    double beta[kVolMaxBeta];
};

}  // namespace radsvd

struct radsvd_vol_plan {
    int K, L, M, NC, HC, HD, n_beta, prec, n_vol, n_tgt;
    int chunk;                 // pairs per block of pairs
    int user_U, user_V;
    int real;                  // real volumes: half the orders, real X
    char *ws;
    size_t ws_bytes;
    double *w, *beta;          // [K], [n_beta]
    double *C, *U, *lamC;      // [K][K], [K][K] (column h = eigenvector h), [K]
    double *D, *V, *lamD;      // [L+1][L+1], [L+1][L+1], [L+1]
    void *logC, *logD;         // Jacobi rotation logs
    void *As, *Bs;             // principal shells [n][H_C][(L+1)^2] complex
    void *Vd;                  // [n_beta][H_D][M][M] real: [v_j^T d](beta)
    void *Xt;                  // [chunk][sum_l (2l+1)^2] complex: step 1, degree-major
    void *Y;                   // [chunk][H_D][M][M] complex: step 1b
    void *Xh;                  // [chunk][n_beta][count] complex: step 2 (count = M^2, or (L+1) M real)
    double *part_val;          // [chunk][n_beta]: best Re X of one angle (NaN: a NaN seen)
    int32_t *part_idx;         // [chunk][n_beta]: its m1' M + m2'
};

namespace radsvd {

hipError_t vol_launch_prepare(radsvd_vol_plan *p, const VolGrid &g, const void *A, const void *B,
                              const double *U_in, const double *V_in, hipStream_t s);
hipError_t vol_launch_align(const radsvd_vol_plan *p, int flags, float *best_score, int32_t *best_idx,
                            void *X_full, hipStream_t s);

}  // namespace radsvd
