// Host-side plan layout and kernel launchers of the radsvd library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "radsvd.h"

namespace radsvd {

constexpr int kMaxK = 128;
constexpr int kMaxQ = 512;
constexpr int kMaxH = 32;
constexpr int kMaxT = 64;
constexpr int kEigMaxSweeps = 40;

// Grid description passed by value to the setup kernel (fits the 4 KB
// kernel-argument limit).
struct GridArgs {
    int K, Q, T;
    double k[kMaxK];
    double w[kMaxK];
    double delta[kMaxT][2];
};

// Tile geometry of the fast (MFMA) Hermitian path.
constexpr int kFastTA = 8;     // images per tile   (16 MFMA rows: re and im rows)
constexpr int kFastTB = 16;    // targets per tile  (16 MFMA columns)

}  // namespace radsvd

struct radsvd_plan {
    int K, Q, H, T, prec, herm, products, n_img, n_tgt;
    int M;       // Q / 2
    int Qc;      // frequencies stored: herm ? Q/2 + 1 : Q
    int H8;      // H rounded up to a multiple of 8 (fast operand rows)
    int nplanes; // fast operand planes (bf16: 1/2/3; fp32: 1)
    int na_pad, nb_pad;   // counts padded to the fast tile sizes
    int user_U;
    int tile_b;
    void *stream_hint;
    char *ws;
    size_t ws_bytes;
    const void *A_polar, *B_polar;
    // workspace sub-buffers (device)
    double *d_k, *d_eta, *d_delta;    // [K], [K], [T][2]
    void *phase;                      // [T][K][Q] cx<R>
    double *C;                        // [K][K]
    double *U;                        // [K][K] (column h = eigenvector h)
    double *lam;                      // [K]
    void *Ueta;                       // [K][H] R : U[r][h] * eta_r
    double *ringsum;                  // [n_tgt][K] complex FP64
    double *gram_part;                // [nsplit][K][K]
    void *eig_log;                    // Jacobi rotation log
    int gram_nsplit;
    void *Ag;                         // [n_img][Qc][H] cx<R>        generic operands
    void *Bg;                         // [n_tgt][T][Qc][H] cx<R>
    void *Af;                         // fast operands (tile-major planes)
    void *Bf;
    size_t Af_bytes, Bf_bytes;
};

namespace radsvd {

// prepare.hip
hipError_t launch_setup(radsvd_plan *p, const GridArgs &g, hipStream_t s);
hipError_t launch_ueta(radsvd_plan *p, const double *U_src, int ld, hipStream_t s);
hipError_t launch_user_U(radsvd_plan *p, const double *U_in, hipStream_t s);
hipError_t launch_principal_rings(radsvd_plan *p, hipStream_t s);
// kernel_c.hip
hipError_t launch_kernel_C(radsvd_plan *p, hipStream_t s);
// eig.hip
hipError_t launch_eig(radsvd_plan *p, hipStream_t s);
size_t eig_log_bytes(int K);
// pairs_generic.hip
hipError_t launch_pairs_generic(const radsvd_plan *p, int flags, float inv_s2, float *best_score,
                                int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full,
                                hipStream_t s);
// pairs_fast.hip
bool fast_path_supported(const radsvd_plan *p, int flags);
bool fast_tile_ok(int tile_b);
hipError_t launch_pairs_fast(const radsvd_plan *p, int flags, float inv_s2, float *best_score,
                             int32_t *best_m, int32_t *best_t, float *lse_pair, hipStream_t s);
// lse.hip
hipError_t launch_lse_img(int n_img, int n_tgt, const float *lse_pair, float *lse_img, hipStream_t s);
// backward.hip
size_t backward_bytes(const radsvd_plan *p);
hipError_t launch_backward(const radsvd_plan *p, float inv_s2, const float *lse_img,
                           const float *glse, void *gB, double *gU, void *ws, hipStream_t s);

// batched.hip
size_t batched_bytes(int n_jobs);
hipError_t launch_pairs_batched(const radsvd_plan *const *plans, int n_jobs, const radsvd_job_out *outs,
                                void *ws, hipStream_t s);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace radsvd
