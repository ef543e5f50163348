// Host-side plan layout and kernel launchers of the radsvd library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "radsvd.h"

namespace radsvd {

constexpr int kMaxK = 128;
constexpr int kMaxQ = 512;
constexpr int kMaxRefine = 64;   // largest refinement factor of align_refine_rotation
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

// Fragment-ordered operands of the fast path.  For one (tile, q) an operand
// block holds, plane after plane, the 64-lane register fragments of the
// 16-row (images: Re and Im row per image) or 16-column (targets) matrix
// operand, in the order the wavefront loads them: lane l's 16 (or 8) bytes at
// l * 16 (or l * 8), so that one load instruction reads one contiguous 1 KB
// (512 B) block.  The depth index of the real embedding of conj(a) b is
// k = c * H8 + h with c = 0 / 1 the first / second block:
//   image Re row [ar | ai], image Im row [-ai | ar], target column [br | bi].
// Formats (kFragF32, kFragBF16, kFragF32B):
// * BF16 planes: chunks of 16 h (v_mfma_f32_16x16x32_bf16; lane l: row
//   l % 16, c = (l / 16) / 2, h = 16 chunk + 8 ((l / 16) % 2) + 0..7) and,
//   when H8 is an odd multiple of 8, one half chunk of 8 h
//   (v_mfma_f32_16x16x16_bf16; lane l: c = (l / 16) / 2,
//   h = 4 ((l / 16) % 2) + 0..3, 8 bytes per lane).
// * FP32 in BF16 fragment order (one plane, split into bf16 terms in
//   registers): the same lane mapping with FP32 values; a chunk is two 1 KB
//   halves (lane l's values 0..3, then 4..7, 16 bytes each), the half chunk
//   one 1 KB block (lane l's 4 values).
// * FP32 plane: chunks of 16 consecutive k (v_mfma_f32_16x16x4_f32; lane l's
//   element j feeds the chunk's MFMA j with k = 16 chunk + 4 j + l / 16).
//
// The eight-wave kernel (Q = 384, 512, split bf16 with 6 products) uses the
// paired slot order: lane l of a full chunk holds h = 16 chunk + 4 (l / 16)
// + 0..3, slots 0..3 for c = 0 and 4..7 for c = 1 (half chunk: h = 16 NF +
// 2 (l / 16) + 0..1, slots 0..1 and 2..3).  A Re row and the Im row of the
// same image then hold the same values, [ar | ai] and [-ai | ar], so the
// image operand stores each value once (kFragBF16D): lane l keeps 8 bytes
// (4 for the half chunk) of its "own" part, ar for even rows and ai for odd
// rows, and receives the other part from lane l ^ 1 in registers.
// kFragF32P holds the targets as FP32 in the paired order: per full chunk a
// 1 KB half of br (lane l's 4 values at 16 l) and one of bi; the half chunk
// one 1 KB block of [br h0, br h1, bi h0, bi h1].
constexpr int kFragF32 = 0, kFragBF16 = 1, kFragF32B = 2, kFragBF16D = 3, kFragF32P = 4;
__host__ __device__ inline int frag_plane_bytes(int fmt, int H8) {
    if (fmt == kFragBF16) return (H8 / 16) * 1024 + ((H8 % 16) ? 512 : 0);
    if (fmt == kFragF32B || fmt == kFragF32P) return (H8 / 16) * 2048 + ((H8 % 16) ? 1024 : 0);
    if (fmt == kFragBF16D) return (H8 / 16) * 512 + ((H8 % 16) ? 256 : 0);
    return (H8 / 8) * 1024;
}
// plans that run the eight-wave pair kernel (and use the paired layouts)
__host__ __device__ inline bool wide_plan(int prec, int products, int hermitian, int Q) {
    return hermitian && prec == RADSVD_BF16X3 && products == 6 && (Q == 384 || Q == 512);
}
// byte offset of element (row, c, h) within one plane of an operand block
__host__ __device__ inline int frag_elem_offset(int fmt, int H8, int row, int c, int h) {
    if (fmt != kFragF32) {
        const bool b16 = fmt == kFragBF16;
        const int nfull = H8 / 16;
        if (h < 16 * nfull) {
            const int hb = h >> 4, hh = h & 15;
            const int g = 2 * c + (hh >> 3), e = hh & 7;
            return b16 ? hb * 1024 + (16 * g + row) * 16 + e * 2
                       : hb * 2048 + (e >> 2) * 1024 + (16 * g + row) * 16 + (e & 3) * 4;
        }
        const int hh = h - 16 * nfull;
        const int g = 2 * c + (hh >> 2), e = hh & 3;
        return b16 ? nfull * 1024 + (16 * g + row) * 8 + e * 2 : nfull * 2048 + (16 * g + row) * 16 + e * 4;
    }
    const int k = c * H8 + h;
    const int chunk = k >> 4, kk = k & 15;
    return chunk * 1024 + (16 * (kk & 3) + row) * 16 + (kk >> 2) * 4;
}

}  // namespace radsvd

struct radsvd_plan {
    int K, Q, H, T, prec, herm, products, n_img, n_tgt;
    int M;       // Q / 2
    int Qc;      // frequencies stored: herm ? Q/2 + 1 : Q
    int H8;      // H rounded up to a multiple of 8 (fast operand rows)
    int nplanes_a, nplanes_b;   // fast operand planes, images / targets
    int ffmt_a, ffmt_b;         // fast operand formats (kFragF32, kFragBF16, kFragF32B)
    int na_pad, nb_pad;   // counts padded to the fast tile sizes
    int user_U;
    int band;    // image tiles per XCD band of the fast path's tile order (0 = default)
    int waves;   // waves per CU of the fast path (0 = default; 4 or 8, align_set_waves)
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
    double *ring_gram;                // [K][K] sum_b Re conj(S_b,r) S_b,r' (translation-averaged kernel only)
    double sigma_delta;               // Gaussian translation prior of kernel C (0: none)
    void *eig_log;                    // Jacobi rotation log
    int gram_nsplit;
    // generic operands: written by align_prepare where the fused path cannot
    // serve the plan, else on first need (the backward pass) by
    // ensure_generic_layout; g_ready says whether they hold the plan's values
    mutable int g_ready;
    void *Ag;                         // [n_img][H][Qc] cx<R>        generic operands (q fastest)
    void *Bg;                         // [n_tgt][T][H][Qc] cx<R>
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
// the same solver on any symmetric K x K FP64 matrix (K <= kMaxK); log of eig_log_bytes(K)
hipError_t launch_eig_raw(const double *C, int K, void *log, double *U, double *lam, hipStream_t s);
// n <= 2 independent decompositions in one launch (one workgroup each)
hipError_t launch_eig_raw2(int n, const double *const *C, const int *K, void *const *log, double *const *U,
                           double *const *lam, hipStream_t s);
size_t eig_log_bytes(int K);
// pairs_generic.hip
hipError_t launch_pairs_generic(const radsvd_plan *p, int flags, float inv_s2, float *best_score,
                                int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full,
                                hipStream_t s);
// pairs_fast.hip
bool fast_path_supported(const radsvd_plan *p, int flags);
bool fast_band_ok(int band);
// writes the generic operand layout if it is not written yet (on stream s)
hipError_t ensure_generic_layout(const radsvd_plan *p, hipStream_t s);
// workgroups per CU the four-wave fused kernel runs this plan at (1 or 2)
int fast_plan_wpc(const radsvd_plan *p);
// whether align_set_waves may give this plan `waves` waves per CU (0, 4, 8)
bool fast_waves_ok(const radsvd_plan *p, int waves);
constexpr int kDefaultBand = 8;
hipError_t launch_pairs_fast(const radsvd_plan *p, int flags, float inv_s2, float *best_score,
                             int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full, hipStream_t s);
// pairs_generic.hip, list mode: pairs [n][2] (image, target); outputs at list positions
hipError_t launch_pairs_list(const radsvd_plan *p, int flags, float inv_s2, int n, const int32_t *pairs,
                             float *best_score, int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full,
                             hipStream_t s);
// march.hip
hipError_t launch_top_targets(int n_img, int n_tgt, const float *score, int k, int32_t *cand, hipStream_t s);
hipError_t launch_landscape_metrics(long long n_pairs, int len, const void *X_est, const void *X_ref, int fp64,
                                    float *f, double *stats, double *summary, hipStream_t s);
constexpr int kMaxTopK = 1024;   // candidates per image of align_top_targets
// refine.hip
hipError_t launch_refine_rotation(const radsvd_plan *p, const int32_t *best_m, const int32_t *best_t, int Rf,
                                  float *fine_score, int32_t *fine_m, hipStream_t s);
// lse.hip
hipError_t launch_lse_img(int n_img, int n_tgt, const float *lse_pair, float *lse_img, hipStream_t s);
// backward.hip
size_t backward_bytes(const radsvd_plan *p);
hipError_t launch_backward(const radsvd_plan *p, float inv_s2, const float *lse_img,
                           const float *glse, void *gB, double *gU, void *ws, hipStream_t s);

// batched.hip
size_t batched_bytes(int n_jobs);
// the no-allocation batched launch: job table and queues in a static device
// array of kNoAllocScratchBytes per GPU (RADSVD_NOALLOC_MAX_JOBS jobs)
constexpr size_t kNoAllocScratchBytes = 256 * 1024;
hipError_t noalloc_scratch(void **out);
bool batched_supported(const radsvd_plan *p);
hipError_t launch_pairs_batched(const radsvd_plan *const *plans, int n_jobs, const radsvd_job_out *outs,
                                void *ws, hipStream_t s);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace radsvd
