#pragma once
// Fused Hermitian pair kernel on the gfx950 matrix cores.
//
// Paper section 3.3 (two-step evaluation with principal rings, steps 1-2) for
// Hermitian inputs (real images, whose transforms are conjugate-symmetric):
//   step 1  S[q] = sum_h conj(At[a][h][q]) Bt[b][t][h][q],   q in [0, M], M = Q/2
//   step 2  X[m] = sum_{q<Q} S[q] exp(-2 pi i q m / Q)        (S[Q-q] = conj S[q])
// then the maximum over (t, m) (section 2.7) and/or the log-sum-exp, without
// the landscape ever leaving the chip.
//
// Workgroup = 4 wavefronts = one tile of 8 images x 16 targets (128 pairs);
// the translations t are looped inside the workgroup.
//
// Step 1 runs on MFMA.  For one q the contraction is a real GEMM with
//   rows  = (image, re/im)           16 = 8 images x {Re S, Im S}
//   cols  = target                   16
//   depth = (product, re/im part, h) the real embedding of conj(a) * b:
//           Re-row [ar | ai], Im-row [-ai | ar], column [br | bi]
// FP32:   v_mfma_f32_16x16x4_f32, depth 2*H8.
// BF16x3: v_mfma_f32_16x16x32_bf16 over the split products (hi*hi, hi*mid,
//         mid*hi [, mid*mid, hi*lo, lo*hi]); FP32 accumulation.  A half chunk
//         (ranks an odd multiple of 8) runs on v_mfma_f32_16x16x16_bf16 in an
//         accumulation chain of its own; with six products, two products of the
//         half chunk share one v_mfma_f32_16x16x32_bf16 instead.
// The prepare kernel writes the operands of each (tile, q) as one block in
// register-fragment order (frag_elem_offset), so every load instruction of a
// wavefront reads one contiguous 1 KB (or 512 B) span.
//
// Step 2: every pair is owned by two lanes (l and l + 32 of one wavefront).
// The half-spectrum S[0..M] becomes the length-M complex sequence
//   Z[k] = (S[k] + conj S[M-k]) + i W_Q^k (S[k] - conj S[M-k]),
// whose length-M DFT z gives X[2n] = Re z[n], X[2n+1] = Im z[n].  Lane
// e = 0 holds Z at even k, lane e = 1 at odd k; each runs an in-register
// FFT of length L = M/2, and one radix-2 stage across the two lanes
// (v_permlane32_swap) completes z.  Everything in step 2 is FP32 VALU.
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace radsvd {
namespace fastk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

template <int N>
using IC = std::integral_constant<int, N>;

template <int B, int E, class F>
__device__ __forceinline__ void sfor(F &&f) {
    if constexpr (B < E) {
        f(IC<B>{});
        sfor<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------------------
// compile-time twiddles: cos / sin of 2 pi num / den with exact octant
// reduction and Taylor series on [0, pi/4]
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double sin_poly(double x) {
    double x2 = x * x, t = x, s = x;
    for (int n = 1; n < 14; ++n) {
        t *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
        s += t;
    }
    return s;
}
constexpr double cos_poly(double x) {
    double x2 = x * x, t = 1.0, s = 1.0;
    for (int n = 1; n < 14; ++n) {
        t *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
        s += t;
    }
    return s;
}
// returns cos (want_sin = false) or sin of 2 pi num / den
constexpr double trig2pi(long num, long den, bool want_sin) {
    long n = num % den;
    if (n < 0) n += den;
    const long a = 8 * n;
    const long o = a / den;
    const long r = a - o * den;
    const double th = (kPi / 4.0) * ((double)r / (double)den);
    const double thc = (kPi / 4.0) * ((double)(den - r) / (double)den);
    double c = 0, s = 0;
    switch (o) {
    case 0: c = cos_poly(th); s = sin_poly(th); break;
    case 1: c = sin_poly(thc); s = cos_poly(thc); break;
    case 2: c = -sin_poly(th); s = cos_poly(th); break;
    case 3: c = -cos_poly(thc); s = sin_poly(thc); break;
    case 4: c = -cos_poly(th); s = -sin_poly(th); break;
    case 5: c = -sin_poly(thc); s = -cos_poly(thc); break;
    case 6: c = sin_poly(th); s = -cos_poly(th); break;
    default: c = cos_poly(thc); s = -sin_poly(thc); break;
    }
    return want_sin ? s : c;
}

// v * W_N^E, W_N = exp(-2 pi i / N)
template <long E, long N>
__device__ __forceinline__ cx<float> twmul(cx<float> v) {
    constexpr long e = ((E % N) + N) % N;
    if constexpr (e == 0) {
        return v;
    } else if constexpr (4 * e == N) {
        return {v.im, -v.re};
    } else if constexpr (2 * e == N) {
        return {-v.re, -v.im};
    } else if constexpr (4 * e == 3 * N) {
        return {-v.im, v.re};
    } else {
        constexpr float c = (float)trig2pi(e, N, false);
        constexpr float s = (float)(-trig2pi(e, N, true));
        return {v.re * c - v.im * s, v.re * s + v.im * c};
    }
}

// ---------------------------------------------------------------------------
// in-register mixed-radix DIF FFT (radices 4, then 2, then 3)
// ---------------------------------------------------------------------------
constexpr int ct_nst(int n) {
    int s = 0;
    while (n % 4 == 0) { n /= 4; ++s; }
    while (n % 2 == 0) { n /= 2; ++s; }
    while (n % 3 == 0) { n /= 3; ++s; }
    return s;
}
constexpr int ct_radix(int n, int st) {
    int s = 0;
    while (n % 4 == 0) { if (s == st) return 4; n /= 4; ++s; }
    while (n % 2 == 0) { if (s == st) return 2; n /= 2; ++s; }
    while (n % 3 == 0) { if (s == st) return 3; n /= 3; ++s; }
    return 1;
}
constexpr int ct_len(int n, int st) {
    int L = n;
    for (int s = 0; s < st; ++s) L /= ct_radix(n, s);
    return L;
}
// register position of output frequency f
constexpr int ct_pos(int n, int f) {
    int pos = 0, L = n;
    const int ns = ct_nst(n);
    for (int s = 0; s < ns; ++s) {
        const int R = ct_radix(n, s);
        L /= R;
        pos += (f % R) * L;
        f /= R;
    }
    return pos;
}

template <int R>
__device__ __forceinline__ void dft_r(cx<float> *v) {
    if constexpr (R == 2) {
        cx<float> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        cx<float> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        cx<float> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        cx<float> u = cmul_mi(t3);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, u);
        v[3] = csub(t1, u);
    } else {
        const float h = 0.86602540378443864676f;
        cx<float> a = v[0];
        cx<float> t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
        cx<float> m = {a.re - 0.5f * t1.re, a.im - 0.5f * t1.im};
        cx<float> u = {h * t2.im, -h * t2.re};
        v[0] = cadd(a, t1);
        v[1] = cadd(m, u);
        v[2] = csub(m, u);
    }
}

template <int N, int S>
__device__ __forceinline__ void fft_stage(cx<float> (&x)[N]) {
    constexpr int R = ct_radix(N, S);
    constexpr int L = ct_len(N, S);
    constexpr int span = L / R;
    sfor<0, N / L>([&](auto blk) {
        sfor<0, span>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            constexpr int base = decltype(blk)::value * L + k;
            cx<float> v[R];
            sfor<0, R>([&](auto r) { v[decltype(r)::value] = x[base + decltype(r)::value * span]; });
            dft_r<R>(v);
            x[base] = v[0];
            sfor<1, R>([&](auto pp) {
                constexpr int p = decltype(pp)::value;
                x[base + p * span] = twmul<(long)k * p, L>(v[p]);
            });
        });
    });
}

template <int N>
__device__ __forceinline__ void reg_fft(cx<float> (&x)[N]) {
    sfor<0, ct_nst(N)>([&](auto S) { fft_stage<N, decltype(S)::value>(x); });
}

__device__ __forceinline__ float perm_swap_lo(float vdst, float vsrc, float &vsrc_out) {
    // lanes 32..63 of vdst <-> lanes 0..31 of vsrc
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(vdst), __float_as_uint(vsrc), false, false);
    vsrc_out = __uint_as_float(r[1]);
    return __uint_as_float(r[0]);
}

struct Args {
    const void *Af;            // fast operands, images
    const void *Bf;            // fast operands, targets
    int n_img, n_tgt, T;
    int nTA, nTB;              // tile counts
    int band;                  // image tiles per XCD band (tile order only)
    int H8;
    int nplanes;
    int flags;
    float inv_s2;
    float *best_score;
    int32_t *best_m, *best_t;
    float *lse_pair;
    cx<float> *X_full;         // FULL output [n_img][n_tgt][T][Q] (real landscape, imaginary parts 0)
};

// tile index of workgroup `wg`: workgroups are dealt round-robin to the 8
// XCDs; consecutive workgroups of one XCD walk a band of `band` image tiles
// with the target tile advancing every `band`, so the XCD's concurrently
// resident workgroups share image and target operand rows in its L2.
// linear tile index -> (image tile, target tile) in bands of `band` image tiles
__device__ __forceinline__ void band_tile(int lin, int nTA, int nTB, int band, int &ta, int &tb) {
    const int bi = lin / (band * nTB);
    const int rows = min(band, nTA - bi * band);
    const int in_band = lin - bi * band * nTB;
    ta = bi * band + in_band % rows;
    tb = in_band / rows;
}
__device__ __forceinline__ void tile_of(int wg, int nwg, int nTA, int nTB, int band, int &ta, int &tb) {
    const int xcd = wg & 7;
    const int full = nwg >> 3, rem = nwg & 7;
    const int lin = xcd * full + min(xcd, rem) + (wg >> 3);
    band_tile(lin, nTA, nTB, band, ta, tb);
}

// Contraction precision of the fused kernel.
//   KIND 0: FP32 operands, v_mfma_f32_16x16x4_f32
//   KIND 1: bf16 (one product), v_mfma_f32_16x16x32_bf16 (+ 16x16x16 for a half chunk)
//   KIND 2: split bf16, products hi*hi, hi*mid, mid*hi
//   KIND 3: split bf16, + mid*mid, hi*lo, lo*hi; the image operand is stored
//           as its three bf16 planes, the target operand as FP32 values in
//           bf16 fragment order, split in registers
template <int KIND>
struct Prec {
    static constexpr int NPL = KIND == 0 ? 1 : (KIND == 3 ? 3 : (KIND == 2 ? 2 : 1));   // planes multiplied
    static constexpr int NPL_B = KIND == 3 ? 1 : NPL;                                   // target planes loaded
    static constexpr int NPROD = KIND == 3 ? 6 : (KIND == 2 ? 3 : 1);
    static constexpr int pa(int p) { return p == 2 ? 1 : (p == 3 ? 1 : (p == 5 ? 2 : 0)); }   // A plane
    static constexpr int pb(int p) { return p == 1 ? 1 : (p == 3 ? 1 : (p == 4 ? 2 : 0)); }   // B plane
};

// registers per lane of one job's operands (the Frag layouts below)
template <int KIND, int NF, int HF>
constexpr int frag_regs() {
    return KIND == 3 ? Prec<3>::NPL * (4 * NF + 2 * HF) + 8 * NF + 4 * HF
                     : 2 * Prec<KIND>::NPL * (4 * NF + 2 * HF);
}

// One job's operand registers: NF full chunks (16 bytes per lane) and, for
// BF16 ranks that are odd multiples of 8, one half chunk (8 bytes per lane),
// per loaded plane, for the image rows (a) and the target columns (b).
template <int KIND, int NF, int HF>
struct Frag {
    u32x4 a[Prec<KIND>::NPL][NF > 0 ? NF : 1];
    u32x4 b[Prec<KIND>::NPL][NF > 0 ? NF : 1];
    u32x2 ah[Prec<KIND>::NPL];
    u32x2 bh[Prec<KIND>::NPL];
};
// KIND 3: the image planes as loaded; for the targets the FP32 values
// themselves, 8 per lane and chunk (two 16-byte halves), 4 in the half chunk
template <int NF, int HF>
struct Frag<3, NF, HF> {
    u32x4 a[3][NF > 0 ? NF : 1];
    u32x2 ah[3];
    u32x4 b[NF > 0 ? NF : 1][2];
    u32x4 bh;
};

// x = hi + mid + lo in bf16 (round to nearest even at each step; the
// remainders x - hi and x - hi - mid are exact in FP32), two values at a time
// on v_cvt_pk_bf16_f32.  Same terms as the host-side split of the bf16 planes.
__device__ __forceinline__ void split3_pair(unsigned x0, unsigned x1, unsigned &hi, unsigned &mid, unsigned &lo) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    f32x2 x = {__uint_as_float(x0), __uint_as_float(x1)};
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2));
    x = f32x2{x[0] - __uint_as_float(hi << 16), x[1] - __uint_as_float(hi & 0xffff0000u)};
    mid = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2));
    x = f32x2{x[0] - __uint_as_float(mid << 16), x[1] - __uint_as_float(mid & 0xffff0000u)};
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2));
}
// 8 FP32 values (r0: values 0..3, r1: 4..7) -> bf16x8 hi, mid, lo
__device__ __forceinline__ void split3_frag8(const u32x4 &r0, const u32x4 &r1, u32x4 (&pl)[3]) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const u32x4 &r = d < 2 ? r0 : r1;
        unsigned h, m, o;
        split3_pair(r[2 * (d & 1)], r[2 * (d & 1) + 1], h, m, o);
        pl[0][d] = h;
        pl[1][d] = m;
        pl[2][d] = o;
    }
}
// 4 FP32 values -> bf16x4 hi, mid, lo
__device__ __forceinline__ void split3_frag4(const u32x4 &r, u32x2 (&pl)[3]) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        unsigned h, m, o;
        split3_pair(r[2 * d], r[2 * d + 1], h, m, o);
        pl[0][d] = h;
        pl[1][d] = m;
        pl[2][d] = o;
    }
}

// Workgroups per CU by default (see k_pairs_fast): two where the LDS holds two
// and one job's operand registers leave room for a second wave per SIMD
// without spills (fr: frag_regs of the instantiation).
__host__ __device__ constexpr int fast_wpc_rule(int Q, int fr) {
    return (Q <= 128 || (Q <= 192 && fr <= 30) || (Q == 256 && fr <= 24)) ? 2 : 1;
}
template <int Q, int KIND, int NF, int HF>
constexpr int fast_wg_per_cu() {
    return fast_wpc_rule(Q, frag_regs<KIND, NF, HF>());
}
// Staging buffers for the MFMA results: two (round parity) unless a single one
// lets a second workgroup fit in the LDS (Q = 256: 16 + 64 KB).
template <int Q, int WPC>
constexpr int fast_nstage() {
    static_assert(WPC == 1 || (WPC == 2 && Q <= 256), "two workgroups per CU fit the LDS up to Q = 256");
    return (Q == 256 && WPC == 2) ? 1 : 2;
}
// LDS bytes of one workgroup
template <int Q, int WPC>
constexpr size_t fast_lds_bytes() {
    return (size_t)(fast_nstage<Q, WPC>() * 16 * 128 + (Q / 8) * 256) * sizeof(cx<float>);
}
// the rule at run time (kind: 0 FP32, 1 BF16, 2 split bf16 with 3 products, 3 with 6)
inline int fast_default_wpc(int kind, int Q, int H8) {
    const int NF = kind == 0 ? H8 / 8 : H8 / 16, HF = kind == 0 ? 0 : ((H8 % 16) ? 1 : 0);
    int fr;
    switch (kind) {
    case 0: fr = 2 * Prec<0>::NPL * (4 * NF + 2 * HF); break;
    case 1: fr = 2 * Prec<1>::NPL * (4 * NF + 2 * HF); break;
    case 2: fr = 2 * Prec<2>::NPL * (4 * NF + 2 * HF); break;
    default: fr = Prec<3>::NPL * (4 * NF + 2 * HF) + 8 * NF + 4 * HF; break;
    }
    return fast_wpc_rule(Q, fr);
}
// angle counts with both occupancies compiled (the other one for the tuner)
__host__ __device__ constexpr bool fast_alt_q(int Q) { return Q == 128 || Q == 192 || Q == 256; }

// One tile (ta, tb) for all translations.  Q angles; KIND contraction
// precision; NF, HF operand chunks per plane (FP32: NF = H8 / 8 chunks of 16
// depth values, HF = 0; BF16: NF = H8 / 16, HF = 1 when H8 is an odd multiple
// of 8).  Called by all 256 threads of a workgroup; smem_raw holds
// (2 * 16 * 128 + Q / 8 * 256) complex FP32 values (160 KB at Q = 512).
// Begins and ends at a barrier.
// FULL: the landscape is also written out (RADSVD_OUT_FULL; a separate
// instantiation, so that the BEST/LSE kernels keep their register allocation).
template <int Q, int KIND, int NF, int HF, int WPC, bool FULL = false, class ArgsT>
__device__ __forceinline__ void fast_tile(const ArgsT &args, int ta_in, int tb_in, unsigned char *smem_raw) {
    constexpr int M = Q / 2;
    constexpr int L = M / 2;          // Z values per lane
    constexpr int LH = L / 2;         // in registers; the other LH in LDS
    constexpr int NRP = M / 16;       // paired rounds: q in [8R, 8R+8) with M - q
    constexpr bool BF = KIND != 0;
    using PR = Prec<KIND>;
    static_assert(M % 16 == 0, "Q must be a multiple of 32");

    // staging of MFMA results, double-buffered by round parity: [NSTAGE][16][128]
    constexpr int NSTAGE = fast_nstage<Q, WPC>();
    cx<float> *stage = reinterpret_cast<cx<float> *>(smem_raw);
    cx<float> *upper = stage + NSTAGE * 16 * 128;                 // [LH][256]

    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63;
    const int e = l >> 5;               // 0: even-k lane, 1: odd-k lane
    const int P = 32 * w + (l & 31);    // pair within the tile
    const int pa = P >> 4, pb = P & 15;
    // Every scalar of the tile is workgroup-uniform.  Said explicitly, so that a
    // caller passing them in vector registers (a function call) still gets
    // scalar buffer descriptors and offsets instead of per-lane loops.
    const int ta = __builtin_amdgcn_readfirstlane(ta_in), tb = __builtin_amdgcn_readfirstlane(tb_in);
    const int flags = __builtin_amdgcn_readfirstlane(args.flags);
    const int nT = __builtin_amdgcn_readfirstlane(args.T), nTB = __builtin_amdgcn_readfirstlane(args.nTB);
    const float inv_s2 = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(args.inv_s2)));
    auto uniform_ptr = [](const void *q) {
        const unsigned long long u = reinterpret_cast<unsigned long long>(q);
        const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)u);
        const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(u >> 32));
        return reinterpret_cast<const char *>(((unsigned long long)hi << 32) | lo);
    };
    const char *Af = uniform_ptr(args.Af), *Bf = uniform_ptr(args.Bf);
    const bool do_best = flags & RADSVD_OUT_BEST;
    const bool do_lse = flags & RADSVD_OUT_LSE;
    const bool do_full = FULL && (flags & RADSVD_OUT_FULL);

    // ---- MFMA operands: fragment-ordered blocks, one per (tile, q) ----
    // Lane l reads bytes [16 l, 16 l + 16) of each full chunk and [8 l, 8 l + 8)
    // of the half chunk; the block of frequency q starts at q * BB.  Job J of
    // this wave reads frequency q = 8R + 2w + j (lower, j = 0, 1) or
    // M - 8R - 2w - (j - 2) (upper, j = 2, 3); the wave part of q lives in the
    // per-lane offsets, the round part is a compile-time scalar offset.
    const int g = l >> 4, i16 = l & 15;        // MFMA output: rows 4g..4g+3, column i16
    constexpr bool F32B = KIND == 3;              // targets: FP32 values in bf16 fragment order
    constexpr int PB = NF * 1024 + HF * 512;      // bytes per bf16 / FP32 plane
    constexpr int BBA = PR::NPL * PB;             // bytes per (tile, q) block, images
    constexpr int PBB = F32B ? 2 * PB : PB;       // bytes per target plane
    constexpr int BBB = PR::NPL_B * PBB;          // bytes per (tile, q) block, targets
    const int vloA = 2 * w * BBA, vhiA = (M / 2 + 7 - 2 * w) * BBA;
    const int vloB = 2 * w * BBB, vhiB = (M / 2 + 7 - 2 * w) * BBB;
    const int vFA_lo = 16 * l + vloA, vFA_hi = 16 * l + vhiA;
    const int vHA_lo = 8 * l + NF * 1024 + vloA, vHA_hi = 8 * l + NF * 1024 + vhiA;
    const int vFB_lo = 16 * l + vloB, vFB_hi = 16 * l + vhiB;
    const int vHB_lo = (F32B ? 16 : 8) * l + NF * (F32B ? 2048 : 1024) + vloB;
    const int vHB_hi = (F32B ? 16 : 8) * l + NF * (F32B ? 2048 : 1024) + vhiB;
    const char *Abase = Af + (size_t)ta * (M + 1) * BBA;
    const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
        (void *)Abase, (short)0, (M + 1) * BBA, 0x00020000);


    float run_best = -INFINITY;
    int run_idx = 0x7fffffff;
    bool run_nan = false;
    float run_m = -INFINITY, run_s = 0.f;

    auto rsrcB = [&](int t) {
        const char *Bbase = Bf + ((size_t)t * nTB + tb) * (M + 1) * BBB;
        return __builtin_amdgcn_make_buffer_rsrc((void *)Bbase, (short)0, (M + 1) * BBB, 0x00020000);
    };
    // job J = 4R + j: upper (j >= 2) or lower, and its compile-time block offset
    auto job_upper = [](int J) { return (J & 3) >= 2; };
    // block index of job J (times the block size of a side gives its scalar offset)
    auto job_blk = [](int J) {
        const int R = J >> 2, j = J & 3;
        return (j < 2) ? (8 * R + (j & 1)) : (8 * (NRP - 1 - R) + 1 - (j & 1));
    };
    using FragT = Frag<KIND, NF, HF>;
    // bf16 pairs (-1, 0) and (0, -1) for the remainders of the split, kept in
    // registers: folded into an instruction as the inline constant -1.0, the
    // first pair was read as (0, -1) on gfx950
    unsigned dmask0 = 0x0000bf80u, dmask1 = 0xbf800000u;
    if constexpr (KIND == 3) asm volatile("" : "+v"(dmask0), "+v"(dmask1));
    auto load_at = [&](const __amdgpu_buffer_rsrc_t &rB, bool upper, int blk, FragT &f) {
        const int soffA = blk * BBA, soffB = blk * BBB;
        const int vFA = upper ? vFA_hi : vFA_lo, vHA = upper ? vHA_hi : vHA_lo;
        const int vFB = upper ? vFB_hi : vFB_lo, vHB = upper ? vHB_hi : vHB_lo;
#pragma unroll
        for (int pl = 0; pl < PR::NPL; ++pl) {
#pragma unroll
            for (int hb = 0; hb < NF; ++hb)
                f.a[pl][hb] = __builtin_amdgcn_raw_buffer_load_b128(rA, vFA + pl * PB + hb * 1024, soffA, 0);
            if constexpr (HF) f.ah[pl] = __builtin_amdgcn_raw_buffer_load_b64(rA, vHA + pl * PB, soffA, 0);
        }
        if constexpr (F32B) {
#pragma unroll
            for (int hb = 0; hb < NF; ++hb)
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2)
                    f.b[hb][s2] = __builtin_amdgcn_raw_buffer_load_b128(rB, vFB + hb * 2048 + s2 * 1024, soffB, 0);
            if constexpr (HF) f.bh = __builtin_amdgcn_raw_buffer_load_b128(rB, vHB, soffB, 0);
        } else {
#pragma unroll
            for (int pl = 0; pl < PR::NPL; ++pl) {
#pragma unroll
                for (int hb = 0; hb < NF; ++hb)
                    f.b[pl][hb] = __builtin_amdgcn_raw_buffer_load_b128(rB, vFB + pl * PB + hb * 1024, soffB, 0);
                if constexpr (HF) f.bh[pl] = __builtin_amdgcn_raw_buffer_load_b64(rB, vHB + pl * PB, soffB, 0);
            }
        }
    };
    // The MFMAs of one job accumulate in several independent chains (a
    // product's predecessor in its chain is several instructions back, so the
    // wave does not wait on each result), summed in a fixed order at the end.
    // Full chunks and the half chunk (v_mfma_f32_16x16x16_bf16) never share a
    // chain: every chain has a single MFMA opcode.
    // Chains per kind (measured): split bf16 with 3 products 3 + 2; the other
    // kinds one chain each (with 6 products more chains cost prefetch depth
    // or VALU and measured slower; FP32 measured slower too).
    constexpr int NCF = KIND == 2 ? 3 : 1;
    constexpr int NCH = KIND == 2 ? 2 : 1;
    // KIND 3 issues its half-chunk products as full-size MFMAs in the chain of the full chunks
    constexpr bool HALF_SEP = HF && KIND != 3;
    auto mma = [&](const FragT &f, auto &&after_hi) -> f32x4 {
        f32x4 ac[NCF], ah[NCH];
#pragma unroll
        for (int c = 0; c < NCF; ++c) ac[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < NCH; ++c) ah[c] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (F32B) {
            // Split in three stages, each followed by the products it completes,
            // so that the bf16 conversions of one stage run beside the MFMAs of
            // the one before: hi -> hi*hi; mid -> hi*mid, mid*hi, mid*mid;
            // lo -> hi*lo, lo*hi (the products and order of the stored planes).
            typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            // (the image planes come from memory; only the target values are split)
            constexpr int NFA = NF > 0 ? NF : 1;
            u32x4 pb_[NFA][3];
            u32x2 pbh[3];
            unsigned rb[NFA][8], rbh[4];   // residuals (FP32 bits)
#pragma unroll
            for (int hb = 0; hb < NF; ++hb)
#pragma unroll
                for (int e = 0; e < 8; ++e) rb[hb][e] = f.b[hb][e >> 2][e & 3];
#pragma unroll
            for (int e = 0; e < 4; ++e) rbh[e] = f.bh[e];
            // one term of a pair of values: convert (round to nearest even), then
            // leave the exact remainder x - term for the next term, one bf16 dot
            // product each (x + (-1) t0 + 0 t1: exact products, exact difference)
            auto term = [&](unsigned &x0, unsigned &x1, bool last) -> unsigned {
                const bf16x2 t = __builtin_convertvector(f32x2{__uint_as_float(x0), __uint_as_float(x1)}, bf16x2);
                if (!last) {
                    x0 = __float_as_uint(__builtin_amdgcn_fdot2_f32_bf16(t, __builtin_bit_cast(bf16x2, dmask0),
                                                                         __uint_as_float(x0), false));
                    x1 = __float_as_uint(__builtin_amdgcn_fdot2_f32_bf16(t, __builtin_bit_cast(bf16x2, dmask1),
                                                                         __uint_as_float(x1), false));
                }
                return __builtin_bit_cast(unsigned, t);
            };
            auto stage = [&](auto KK) {
                constexpr int k = decltype(KK)::value;
#pragma unroll
                for (int hb = 0; hb < NF; ++hb)
#pragma unroll
                    for (int d = 0; d < 4; ++d) pb_[hb][k][d] = term(rb[hb][2 * d], rb[hb][2 * d + 1], k == 2);
                if constexpr (HF) {
#pragma unroll
                    for (int d = 0; d < 2; ++d) pbh[k][d] = term(rbh[2 * d], rbh[2 * d + 1], k == 2);
                }
            };
            auto prod = [&](auto PP) {
                constexpr int p = decltype(PP)::value;
#pragma unroll
                for (int hb = 0; hb < NF; ++hb) {
                    f32x4 &c = ac[(p * NF + hb) % NCF];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, f.a[PR::pa(p)][hb]),
                                                               __builtin_bit_cast(bf16x8, pb_[hb][PR::pb(p)]), c, 0, 0, 0);
                }
            };
            // Half chunk: two products share one v_mfma_f32_16x16x32_bf16.  A lane's
            // eight depth slots hold its four slots of the first product, then its
            // four of the second, in A and in B alike, so the sum over the 32 slots
            // is the sum of the two 16-deep products (the 16x16x16 form costs about
            // as much issue time as the 16x16x32 one).  Pairs (A planes | B planes):
            // hi*mid + hi*hi and mid*mid + lo*hi after the mid stage, mid*hi + hi*lo
            // after the lo stage.
            auto half2 = [&](const u32x2 &a0, const u32x2 &a1, const u32x2 &b0, const u32x2 &b1) {
                const u32x4 av = {a0[0], a0[1], a1[0], a1[1]};
                const u32x4 bv = {b0[0], b0[1], b1[0], b1[1]};
                ac[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                               __builtin_bit_cast(bf16x8, bv), ac[0], 0, 0, 0);
            };
            stage(IC<0>{});
            after_hi();
            prod(IC<0>{});
            stage(IC<1>{});
            prod(IC<1>{});
            prod(IC<2>{});
            prod(IC<3>{});
            if constexpr (HF) {
                half2(f.ah[0], f.ah[0], pbh[1], pbh[0]);
                half2(f.ah[1], f.ah[2], pbh[1], pbh[0]);
            }
            stage(IC<2>{});
            prod(IC<4>{});
            prod(IC<5>{});
            if constexpr (HF) half2(f.ah[1], f.ah[0], pbh[0], pbh[2]);
            // instruction order for the scheduler: the conversions of the next
            // stage between the MFMAs of the current one
            constexpr int NPAIR = 4 * NF + 2 * HF;         // value pairs of the target operand
            __builtin_amdgcn_sched_group_barrier(0x002, 3 * NPAIR, 0);   // hi
            __builtin_amdgcn_sched_group_barrier(0x200, 2, 0);           // the previous job's result to LDS
            if constexpr (NF > 0) {
                __builtin_amdgcn_sched_group_barrier(0x008, NF, 0);      // hi*hi
                __builtin_amdgcn_sched_group_barrier(0x002, 3 * NPAIR, 0);   // mid
                __builtin_amdgcn_sched_group_barrier(0x008, NF, 0);      // hi*mid
                __builtin_amdgcn_sched_group_barrier(0x002, NPAIR / 2, 0);   // lo, first half
                __builtin_amdgcn_sched_group_barrier(0x008, NF, 0);      // mid*hi
                __builtin_amdgcn_sched_group_barrier(0x002, NPAIR / 2, 0);   // lo, second half
                __builtin_amdgcn_sched_group_barrier(0x008, 3 * NF + 3 * HF, 0);   // the rest
            }
        } else if constexpr (BF) {
            after_hi();
#pragma unroll
            for (int p = 0; p < PR::NPROD; ++p) {
#pragma unroll
                for (int hb = 0; hb < NF; ++hb) {
                    f32x4 &c = ac[(p * NF + hb) % NCF];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, f.a[PR::pa(p)][hb]),
                                                               __builtin_bit_cast(bf16x8, f.b[PR::pb(p)][hb]), c, 0, 0, 0);
                }
                if constexpr (HF) {
                    f32x4 &c = ah[p % NCH];
                    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, f.ah[PR::pa(p)]),
                                                                 __builtin_bit_cast(s16x4, f.bh[PR::pb(p)]), c, 0, 0, 0);
                }
            }
        } else {
            after_hi();
#pragma unroll
            for (int hb = 0; hb < NF; ++hb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    f32x4 &c = ac[(hb * 4 + j) % NCF];
                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(f.a[0][hb][j]), __uint_as_float(f.b[0][hb][j]),
                                                            c, 0, 0, 0);
                }
        }
        f32x4 acc = ac[0];
#pragma unroll
        for (int c = 1; c < NCF; ++c) acc += ac[c];
        if constexpr (HALF_SEP) {
            f32x4 hs = ah[0];
#pragma unroll
            for (int c = 1; c < NCH; ++c) hs += ah[c];
            if constexpr (NF > 0) acc += hs;
            else acc = hs;
        }
        return acc;
    };
    // staging slot layout: pair P at element P ^ (16 * bit 5 of P) (halves LDS bank conflicts
    // of the MFMA-layout writes; a wave's reads stay within one 32-pair block)
    auto sidx = [](int P) { return P ^ (((P >> 5) & 1) << 4); };
    // rows 4g..4g+3 of the 16x16 block: images 2g, 2g+1 (Re, Im) at target column i16
    auto put = [&](cx<float> *sb, int slot, f32x4 v) {
        sb[slot * 128 + sidx((2 * g) * 16 + i16)] = cx<float>{v[0], v[1]};
        sb[slot * 128 + sidx((2 * g + 1) * 16 + i16)] = cx<float>{v[2], v[3]};
    };
    const int Ps = sidx(P);

    constexpr int FRAG_REGS = frag_regs<KIND, NF, HF>();
    // prefetch depth in jobs: as deep as the registers beside the FFT state allow
    // split bf16 from FP32: a job's result goes to LDS during the next job (after
    // its hi terms), so the wave does not wait for the MFMA chain; the prefetch
    // depth leaves room for the split's registers
    constexpr bool PIPE_PUT = F32B;
    // (two workgroups per CU where the default is one: 256 registers per lane,
    // so at most two jobs ahead)
    constexpr int D0 = PIPE_PUT ? (FRAG_REGS <= 24 ? 4 : (FRAG_REGS <= 32 ? 3 : 2))
                                : (FRAG_REGS <= 24 ? 5 : (FRAG_REGS <= 48 ? 3 : 2));
    constexpr int D = (WPC == 2 && fast_wg_per_cu<Q, KIND, NF, HF>() == 1 && D0 > 2) ? 2 : D0;
    constexpr int NJ = 4 * NRP;
    FragT fr[D + 1];

    for (int t = 0; t < nT; ++t) {
        const __amdgpu_buffer_rsrc_t rB = rsrcB(t);
        // the lane's parity, opaque per translation: the fold's per-lane twiddles
        // are then formed where they are used, not kept live across the loop
        int et = e;
        asm volatile("" : "+v"(et));
        cx<float> x[LH];
        sfor<0, D>([&](auto II) {
            constexpr int J = decltype(II)::value;
            load_at(rB, job_upper(J), job_blk(J), fr[J]);
        });
        // ---------------- step 1: contraction, paired rounds ----------------
        // One barrier per round: round R stages into buffer R & 1, so the fold of
        // round R (reads) overlaps the MFMAs and staging of round R + 1 (other
        // buffer); the barrier of round R + 1 orders fold(R) before round R + 2
        // reuses the buffer.
        sfor<0, NRP>([&](auto RR) {
            constexpr int R = decltype(RR)::value;
            cx<float> *sb = stage + (NSTAGE == 2 ? (R & 1) * (16 * 128) : 0);
            f32x4 pend = {0.f, 0.f, 0.f, 0.f};
            auto slot = [](int jj) { return (jj < 2 ? 0 : 8) + (jj & 1); };
            sfor<0, 4>([&](auto JJ) {
                constexpr int J = 4 * R + decltype(JJ)::value;
                if constexpr (J + D < NJ) {
                    load_at(rB, job_upper(J + D), job_blk(J + D), fr[(J + D) % (D + 1)]);
                } else if constexpr (J + D == NJ) {
                    // middle frequency q = M/2, wave 0 (whose lower offsets are the bare lane part)
                    if (w == 0) load_at(rB, false, M / 2, fr[(J + D) % (D + 1)]);
                }
                // keep the prefetch ahead of this job's MFMAs (the scheduler would otherwise
                // sink the loads and shorten the prefetch distance)
                __builtin_amdgcn_sched_barrier(0);
                constexpr int jj = decltype(JJ)::value;
                const f32x4 acc = mma(fr[J % (D + 1)], [&]() {
                    if constexpr (PIPE_PUT && jj > 0) put(sb, slot(jj - 1) + 2 * w, pend);
                });
                if constexpr (PIPE_PUT) pend = acc;
                else put(sb, slot(jj) + 2 * w, acc);
            });
            if constexpr (PIPE_PUT) put(sb, slot(3) + 2 * w, pend);
            __syncthreads();
            // Z fold: lane e owns k = 8R + 2jj + e (k and M - k have equal parity)
            sfor<0, 4>([&](auto JJ) {
                constexpr int jj = decltype(JJ)::value;
                cx<float> lo = sb[(2 * jj + e) * 128 + Ps];        // S[k]
                cx<float> hi = sb[(8 + 2 * jj + e) * 128 + Ps];    // S[M - k]
                if constexpr (R == 0 && jj == 0) {
                    if (e == 0) {   // S[0], S[M] are real
                        lo.im = 0.f;
                        hi.im = 0.f;
                    }
                }
                const cx<float> u = {lo.re + hi.re, lo.im - hi.im};
                const cx<float> v = {lo.re - hi.re, lo.im + hi.im};
                // * W_Q^k, k = 8R + 2jj + e: the lane picks its twiddle
                constexpr int k0 = 8 * R + 2 * jj;
                constexpr float c0 = (float)trig2pi(k0, Q, false), s0 = (float)(-trig2pi(k0, Q, true));
                constexpr float c1 = (float)trig2pi(k0 + 1, Q, false), s1 = (float)(-trig2pi(k0 + 1, Q, true));
                const float tc = et ? c1 : c0, ts = et ? s1 : s0;
                const cx<float> p = {v.re * tc - v.im * ts, v.re * ts + v.im * tc};
                x[4 * R + jj] = cx<float>{u.re - p.im, u.im + p.re};                  // Z[k]
                const cx<float> zc = {u.re + p.im, p.re - u.im};                      // Z[M - k]
                constexpr int ubase = LH - 4 * R - jj;                                 // upper slot + e
                if constexpr (R == 0 && jj == 0) {
                    if (e == 1) upper[(ubase - 1) * 256 + tid] = zc;
                } else {
                    upper[(ubase - e) * 256 + tid] = zc;
                }
            });
            // one staging buffer: the next round (or the middle frequency) writes it again
            if constexpr (NSTAGE == 1) __syncthreads();
        });
        {   // middle frequency q = M/2 (even): Z[M/2] = 2 S[M/2], upper slot 0 of lane e = 0
            cx<float> *sb = stage + (NSTAGE == 2 ? (NRP & 1) * (16 * 128) : 0);   // not the last round's buffer
            if (w == 0) {
                const f32x4 acc = mma(fr[NJ % (D + 1)], []() {});
                put(sb, 0, acc);
            }
            __syncthreads();
            const cx<float> sm = sb[Ps];
            if (e == 0) upper[tid] = cx<float>{2.f * sm.re, 2.f * sm.im};
            __syncthreads();
        }

        // ---------------- step 2: FFT over q, on chip ----------------
        // DIF split of the length-L sequence: u[k] = x[k] + x[k+LH] (even outputs),
        // v[k] = (x[k] - x[k+LH]) W_L^k (odd outputs, parked in LDS)
        sfor<0, LH>([&](auto KK) {
            constexpr int k = decltype(KK)::value;
            const cx<float> b = upper[k * 256 + tid];
            const cx<float> a = x[k];
            x[k] = cadd(a, b);
            upper[k * 256 + tid] = twmul<k, L>(csub(a, b));
        });
        float bv[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};   // even-lo, even-hi, odd-lo, odd-hi
        int bi[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};  // m of the winning (re, im) pair
        float br[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};   // that pair's re value
        float lse_mx = -INFINITY, lse_sum = 0.f;
        bool nanX = false;
        auto half_pass = [&](auto PARITY) {
            constexpr int par = decltype(PARITY)::value;   // 0: even n, 1: odd n
            reg_fft<LH>(x);   // x[pos(f)] = E[2f + par] (lane 0) / O[2f + par] (lane 1)
            sfor<0, LH / 2>([&](auto FF) {
                constexpr int f = decltype(FF)::value;
                constexpr int ra = ct_pos(LH, f), rb = ct_pos(LH, f + LH / 2);
                float nre, nim;
                x[ra].re = perm_swap_lo(x[ra].re, x[rb].re, nre);
                x[rb].re = nre;
                x[ra].im = perm_swap_lo(x[ra].im, x[rb].im, nim);
                x[rb].im = nim;
                const cx<float> a = x[ra];          // E[n]
                cx<float> b = x[rb];                // O[n], n = 2f + par + e L/2
                if (e) b = cx<float>{b.im, -b.re}; // W_M^{L/2} = -i
                const cx<float> tw = twmul<2 * f + par, M>(b);
                x[ra] = cadd(a, tw);                // z[n]     -> X[2n], X[2n+1]
                x[rb] = csub(a, tw);                // z[n + L] -> X[2n + M], X[2n + M + 1]
            });
            // z at register 0 sums every folded value (each FFT output depends on
            // every input, and IEEE arithmetic never turns a NaN or an infinity
            // back into a finite value), so both of its parts are finite exactly
            // when the whole landscape of this lane pair is (barring overflow)
            if constexpr (par == 0)
                nanX = !__builtin_isfinite(x[ct_pos(LH, 0)].re) || !__builtin_isfinite(x[ct_pos(LH, 0)].im);
            if constexpr (FULL) {
                if (do_full && ta * 8 + pa < args.n_img && tb * 16 + pb < args.n_tgt) {
                    // this lane's part of its pair's landscape row: X[2 n] = Re z[n], X[2 n + 1] = Im z[n]
                    cx<float> *xo = args.X_full +
                                    (((size_t)(ta * 8 + pa) * args.n_tgt + (tb * 16 + pb)) * (size_t)nT + t) * Q + e * (Q / 4);
                    sfor<0, LH / 2>([&](auto FF) {
                        constexpr int m0 = 4 * decltype(FF)::value + 2 * par;
                        const cx<float> zl = x[ct_pos(LH, decltype(FF)::value)];
                        const cx<float> zh = x[ct_pos(LH, decltype(FF)::value + LH / 2)];
                        xo[m0] = cx<float>{zl.re, 0.f};
                        xo[m0 + 1] = cx<float>{zl.im, 0.f};
                        xo[m0 + M] = cx<float>{zh.re, 0.f};
                        xo[m0 + M + 1] = cx<float>{zh.im, 0.f};
                    });
                }
            }
            if (do_best) {
                sfor<0, LH / 2>([&](auto FF) {
                    constexpr int f = decltype(FF)::value;
                    constexpr int m0 = 4 * f + 2 * par;
                    const cx<float> zl = x[ct_pos(LH, f)], zh = x[ct_pos(LH, f + LH / 2)];
                    // a pair (re at m, im at m + 1) replaces the winner only when strictly
                    // larger, so earlier m keep ties; NaN never wins (fmaxf drops it)
                    const float ml = fmaxf(zl.re, zl.im), mh = fmaxf(zh.re, zh.im);
                    if (ml > bv[2 * par]) { bv[2 * par] = ml; bi[2 * par] = m0; br[2 * par] = zl.re; }
                    if (mh > bv[2 * par + 1]) { bv[2 * par + 1] = mh; bi[2 * par + 1] = m0 + M; br[2 * par + 1] = zh.re; }
                });
            }
            if (do_lse) {
                float mx = -INFINITY;
                sfor<0, LH / 2>([&](auto FF) {
                    constexpr int f = decltype(FF)::value;
                    const cx<float> zl = x[ct_pos(LH, f)], zh = x[ct_pos(LH, f + LH / 2)];
                    mx = fmaxf(mx, fmaxf(fmaxf(zl.re, zl.im), fmaxf(zh.re, zh.im)));
                });
                const float s = inv_s2, sm = s * mx;
                float acc = 0.f;
                sfor<0, LH / 2>([&](auto FF) {
                    constexpr int f = decltype(FF)::value;
                    const cx<float> zl = x[ct_pos(LH, f)], zh = x[ct_pos(LH, f + LH / 2)];
                    acc += __expf(fmaf(s, zl.re, -sm)) + __expf(fmaf(s, zl.im, -sm)) +
                           __expf(fmaf(s, zh.re, -sm)) + __expf(fmaf(s, zh.im, -sm));
                });
                const float nm = fmaxf(lse_mx, sm);
                lse_sum = lse_sum * __expf(lse_mx - nm) + acc * __expf(sm - nm);
                lse_mx = nm;
            }
        };
        half_pass(IC<0>{});
        sfor<0, LH>([&](auto KK) { x[decltype(KK)::value] = upper[decltype(KK)::value * 256 + tid]; });
        half_pass(IC<1>{});

        const bool isnanX = nanX || __builtin_isnan(__shfl_xor(nanX ? __builtin_nanf("") : 0.f, 32, 64));
        if (do_best) {
            // the winning pair's im value when its re value is smaller
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) bi[c4] += (br[c4] == bv[c4]) ? 0 : 1;
            // lane-local winner: ties go to the smaller m (even/odd interleave)
            float b0 = bv[0];
            int i0 = bi[0];
            auto take = [&](float v, int i) {
                if (v > b0 || (v == b0 && i < i0)) { b0 = v; i0 = i; }
            };
            take(bv[2], bi[2]);
            take(bv[1], bi[1]);
            take(bv[3], bi[3]);
            i0 += e * L;
            const float ob = __shfl_xor(b0, 32, 64);
            const int oi = __shfl_xor(i0, 32, 64);
            if (ob > b0 || (ob == b0 && oi < i0)) { b0 = ob; i0 = oi; }
            if (isnanX) run_nan = true;
            if (b0 > run_best) { run_best = b0; run_idx = t * Q + i0; }
        }
        if (do_lse) {
            const float om = __shfl_xor(lse_mx, 32, 64), os = __shfl_xor(lse_sum, 32, 64);
            const float nm = fmaxf(lse_mx, om);
            const float tot = lse_sum * __expf(lse_mx - nm) + os * __expf(om - nm);
            if (isnanX) run_nan = true;
            const float rm = fmaxf(run_m, nm);
            run_s = run_s * __expf(run_m - rm) + tot * __expf(nm - rm);
            run_m = rm;
        }
        __syncthreads();   // upper[] and stage[] are reused by the next translation
    }

    const int a = ta * 8 + pa, b = tb * 16 + pb;
    if (e == 0 && a < args.n_img && b < args.n_tgt) {
        const size_t o = (size_t)a * args.n_tgt + b;
        if (do_best) {
            if (run_nan) {
                args.best_score[o] = __builtin_nanf("");
                args.best_m[o] = -1;
                args.best_t[o] = -1;
            } else {
                args.best_score[o] = run_best;
                args.best_m[o] = run_idx % Q;
                args.best_t[o] = run_idx / Q;
            }
        }
        if (do_lse) args.lse_pair[o] = run_nan ? __builtin_nanf("") : run_m + __logf(run_s);
    }
}

// Workgroups per CU.  Up to Q = 192, and at Q = 256 with one staging buffer,
// the LDS (staging and parked Z values, at most 80 KB) leaves room for a
// second workgroup, and the registers are then held to 256 per lane: two waves
// per SIMD hide each other's memory waits (4096 x 4096 pairs, 9 translations,
// 6 products: Q = 128, H = 24 46.1 -> 31.2 ms; Q = 192, H = 16 52.8 -> 33.8
// ms; Q = 256, H = 16 68.5 -> 47.5 ms; FP32, Q = 256, H = 24 81.9 -> 70.6
// ms).  With more operand registers per job (Q = 192 beyond 30, Q = 256 beyond
// 24) the spills cost more than the second wave gains (Q = 192, H = 32: 78.3
// -> 87.8 ms; Q = 256, H = 24, 6 products: 88.5 -> 99.0 ms); beyond Q = 256
// the LDS holds one workgroup.  That rule is the default; at Q = 128, 192 and
// 256 the other occupancy is compiled as well (two workgroups per CU where the
// rule says one then prefetch at most two jobs ahead), and a plan may ask for
// either (align_set_waves), which is what the tile tuner times.

// WPC workgroups per CU
template <int Q, int KIND, int NF, int HF, int WPC, bool FULL>
__global__ __launch_bounds__(256, WPC) void k_pairs_fast(Args args) {
    extern __shared__ unsigned char smem_raw[];
    int ta, tb;
    tile_of(blockIdx.x, gridDim.x, args.nTA, args.nTB, args.band, ta, tb);
    fast_tile<Q, KIND, NF, HF, WPC, FULL>(args, ta, tb, smem_raw);
}

template <int Q, int KIND, int NF, int HF, int WPC, bool FULL>
static hipError_t launch_v(const Args &a, int nwg, hipStream_t s) {
    constexpr size_t shmem = fast_lds_bytes<Q, WPC>();
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute((const void *)k_pairs_fast<Q, KIND, NF, HF, WPC, FULL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    hipLaunchKernelGGL((k_pairs_fast<Q, KIND, NF, HF, WPC, FULL>), dim3(nwg), dim3(256), shmem, s, a);
    return hipGetLastError();
}

// ALT: the occupancy other than the default (only where fast_alt_q)
template <int Q, int KIND, int NF, int HF, bool ALT, bool FULL>
static hipError_t launch_o(const Args &a, int nwg, hipStream_t s) {
    constexpr int d = fast_wg_per_cu<Q, KIND, NF, HF>();
    if constexpr (ALT) {
        if constexpr (fast_alt_q(Q)) return launch_v<Q, KIND, NF, HF, 3 - d, FULL>(a, nwg, s);
        else return hipErrorNotSupported;
    } else {
        return launch_v<Q, KIND, NF, HF, d, FULL>(a, nwg, s);
    }
}

// operand chunk geometry of rank H8 (8, 16, 24 or 32)
template <int Q, int KIND, bool ALT, bool FULL>
static hipError_t launch_h(const Args &a, int nwg, int H8, hipStream_t s) {
    if constexpr (KIND == 0) {
        switch (H8) {
        case 8: return launch_o<Q, 0, 1, 0, ALT, FULL>(a, nwg, s);
        case 16: return launch_o<Q, 0, 2, 0, ALT, FULL>(a, nwg, s);
        case 24: return launch_o<Q, 0, 3, 0, ALT, FULL>(a, nwg, s);
        case 32: return launch_o<Q, 0, 4, 0, ALT, FULL>(a, nwg, s);
        default: return hipErrorNotSupported;
        }
    } else {
        switch (H8) {
        case 8: return launch_o<Q, KIND, 0, 1, ALT, FULL>(a, nwg, s);
        case 16: return launch_o<Q, KIND, 1, 0, ALT, FULL>(a, nwg, s);
        case 24: return launch_o<Q, KIND, 1, 1, ALT, FULL>(a, nwg, s);
        case 32: return launch_o<Q, KIND, 2, 0, ALT, FULL>(a, nwg, s);
        default: return hipErrorNotSupported;
        }
    }
}

// FULL: the instantiations that also write the landscape (default occupancy)
template <int KIND, bool FULL = false>
static hipError_t launch_kind(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    switch (Q) {
    case 64: return launch_h<64, KIND, false, FULL>(a, nwg, H8, s);
    case 96: return launch_h<96, KIND, false, FULL>(a, nwg, H8, s);
    case 128: return launch_h<128, KIND, false, FULL>(a, nwg, H8, s);
    case 192: return launch_h<192, KIND, false, FULL>(a, nwg, H8, s);
    case 256: return launch_h<256, KIND, false, FULL>(a, nwg, H8, s);
    case 384: return launch_h<384, KIND, false, FULL>(a, nwg, H8, s);
    case 512: return launch_h<512, KIND, false, FULL>(a, nwg, H8, s);
    default: return hipErrorNotSupported;
    }
}

// the other occupancy (Q = 128, 192, 256)
template <int KIND>
static hipError_t launch_kind_alt(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    switch (Q) {
    case 128: return launch_h<128, KIND, true, false>(a, nwg, H8, s);
    case 192: return launch_h<192, KIND, true, false>(a, nwg, H8, s);
    case 256: return launch_h<256, KIND, true, false>(a, nwg, H8, s);
    default: return hipErrorNotSupported;
    }
}

// one translation unit per contraction precision (compiled in parallel)
hipError_t launch_fast_fp32(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_bf16(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_bf16x3(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_bf16x3_6(const Args &a, int Q, int nwg, int H8, hipStream_t s);
// with the FULL output (pairs_fast_full_*.hip)
hipError_t launch_fast_full_fp32(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_full_bf16(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_full_bf16x3(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_full_bf16x3_6(const Args &a, int Q, int nwg, int H8, hipStream_t s);
// the occupancy other than the default, Q = 128, 192, 256 (pairs_fast_occ_*.hip)
hipError_t launch_fast_alt_fp32(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_alt_bf16(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_alt_bf16x3(const Args &a, int Q, int nwg, int H8, hipStream_t s);
hipError_t launch_fast_alt_bf16x3_6(const Args &a, int Q, int nwg, int H8, hipStream_t s);
// eight-wave kernel of the plans wide_plan() selects (pairs_wide.hip)
hipError_t launch_wide(const Args &a, int Q, int nwg, int H8, hipStream_t s);

}  // namespace fastk
}  // namespace radsvd
