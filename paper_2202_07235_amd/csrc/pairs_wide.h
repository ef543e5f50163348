#pragma once
// Eight-wave fused Hermitian pair kernel for Q = 384 and 512 (split bf16,
// six products).
//
// Paper section 3.3 (two-step evaluation with principal rings): per
// frequency q the contraction S[q] = sum_h conj(At[a][h][q]) Bt[b][t][h][q]
// (step 1), then X[m] = sum_q S[q] exp(-2 pi i q m / Q) (step 2), with the
// maximum over (t, m) (section 2.7) and/or the log-sum-exp (section 2.6) on
// chip.  The arithmetic is that of k_pairs_fast; the organisation differs.
//
// At Q = 512 the values one 8 x 16 tile holds between the two steps (Q/2 + 1
// complex per pair) take half of the register file and most of the LDS, so
// one workgroup fits per compute unit.  With four waves, one per SIMD, a wave
// that waits for its operand loads leaves its SIMD idle; this kernel runs the
// same tile with eight waves, two per SIMD, and each pair owned by four lanes.
//
// Lanes.  Wave w owns image w of the tile and its 16 targets; lane l takes
// target p = l & 15 with u = (l >> 4) & 1 and e = l >> 5, and holds the
// folded values Z[4 i + 2 u + e], i < M/4 (M = Q/2): those with i < M/8 in
// registers while the contraction runs, the others in LDS until the
// transform.  Z is the fold of k_pairs_fast: Z[k] = (S[k] + conj S[M-k])
// + i W_Q^k (S[k] - conj S[M-k]), and z = DFT_M(Z) gives X[2m] = Re z[m],
// X[2m+1] = Im z[m].
//
// Transform.  Each lane takes the length-M/4 DFT of its values (in
// registers); a radix-2 step across u (lanes l, l ^ 16, v_permlane16_swap)
// gives the length-M/2 DFTs X_e of the even and odd Z, and one across e
// (lanes l, l ^ 32, v_permlane32_swap) gives z.  In each cross-lane step a
// lane does half of the butterflies; per-lane twiddles come from tables in LDS.
//
// Operands.  The image planes are stored once per value (kFragBF16D): a lane
// loads 8 bytes (4 for the half chunk) and builds the Re-row fragment
// [ar | ai] or the Im-row fragment [-ai | ar] with the other half from lane
// l ^ 1 (one DPP move and one sign flip per register).  The targets come as
// FP32 in the paired order (kFragF32P) and are split into hi, mid and lo in
// registers, as in k_pairs_fast.
#include "pairs_fast.h"

namespace radsvd {
namespace fastk {

template <int Q>
struct WideGeom {
    static constexpr int M = Q / 2;
    static constexpr int L4 = M / 4;       // folded values per lane
    static constexpr int LO = L4 / 2;      // i < LO: in registers during the contraction
    static constexpr int NRP = M / 16;     // rounds of 16 frequencies
    // LDS bytes
    static constexpr int STAGE = 0;                        // [16][128] complex: one round's S values
    static constexpr int ZTAB = STAGE + 16 * 128 * 8;      // [M]      W_Q^k
    static constexpr int ZST = ZTAB + M * 8;               // [512][L4 - LO + 1] values i >= LO
    static constexpr int ZLD = L4 - LO + 1;                // row length (padded: lanes fall on distinct banks)
    static constexpr int BYTES = ZST + 512 * ZLD * 8;
};
static_assert(WideGeom<512>::BYTES <= 160 * 1024 && WideGeom<384>::BYTES <= 160 * 1024, "LDS");

// twiddle table of one angle count (all 512 threads; ends with a barrier)
template <int Q>
__device__ void wide_tables(unsigned char *smem) {
    using G = WideGeom<Q>;
    constexpr int M = G::M;
    cx<float> *ztab = reinterpret_cast<cx<float> *>(smem + G::ZTAB);
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)i / (double)Q, &sn, &cs);
        ztab[i] = cx<float>{(float)cs, (float)(-sn)};   // exp(-2 pi i k / Q), rounded from FP64
    }
    __syncthreads();
}

// reg_fft with a scheduling barrier after every GROUP butterflies: each
// butterfly reads and writes its values in place, but without the barriers
// the scheduler interleaves a whole stage and its temporaries then exceed the
// register budget of two waves per SIMD
template <int N, int S, int GROUP>
__device__ __forceinline__ void fft_stage_lp(cx<float> (&x)[N]) {
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
            if constexpr ((decltype(blk)::value * span + k + 1) % GROUP == 0) __builtin_amdgcn_sched_barrier(0);
        });
    });
}
#ifndef WIDE_FG
#define WIDE_FG 2
#endif
template <int N, int GROUP>
__device__ __forceinline__ void reg_fft_lp(cx<float> (&x)[N]) {
    sfor<0, ct_nst(N)>([&](auto S) { fft_stage_lp<N, decltype(S)::value, GROUP>(x); });
}

// 8-byte LDS accesses of complex values (cx<float> alone is only 4-byte
// aligned, which would split each access in two and limit its immediate
// offset to 1 KB)
typedef float f32x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cx<float> lds_ld(const cx<float> *p) {
    const f32x2v v = *reinterpret_cast<const f32x2v *>(p);
    return cx<float>{v[0], v[1]};
}
__device__ __forceinline__ void lds_st(cx<float> *p, cx<float> v) {
    *reinterpret_cast<f32x2v *>(p) = f32x2v{v.re, v.im};
}

template <int NF, int HF>
struct WFrag {
    u32x2 a[3][NF > 0 ? NF : 1];   // image planes: this lane's own part
    unsigned ah[3];                 // half chunk, own part
    u32x4 b[NF > 0 ? NF : 1][2];    // targets, FP32: br half, bi half
    u32x4 bh;                       // half chunk: br h0, br h1, bi h0, bi h1
};

// lane l reads lane l ^ 1 (quad permutation 1, 0, 3, 2)
__device__ __forceinline__ unsigned dpp_pair_swap(unsigned x) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, 0xB1, 0xF, 0xF, false);
}

__device__ __forceinline__ float perm16_swap(float vdst, float vsrc, float &vsrc_out) {
    // odd rows (lanes 16-31, 48-63) of vdst <-> even rows (0-15, 32-47) of vsrc
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(vdst), __float_as_uint(vsrc), false, false);
    vsrc_out = __uint_as_float(r[1]);
    return __uint_as_float(r[0]);
}

// One tile (ta, tb) for all translations; 512 threads; the twiddle tables of
// Q must be in LDS.  Begins and ends at a barrier.
template <int Q, int NF, int HF, class ArgsT>
__device__ __forceinline__ void wide_tile(const ArgsT &args, int ta_in, int tb_in, unsigned char *smem) {
    using G = WideGeom<Q>;
    constexpr int M = G::M, L4 = G::L4, LO = G::LO, NRP = G::NRP;
    static_assert(M % 16 == 0 && L4 % 2 == 0, "Q");
    cx<float> *stage = reinterpret_cast<cx<float> *>(smem + G::STAGE);
    const cx<float> *ztab0 = reinterpret_cast<const cx<float> *>(smem + G::ZTAB);
    cx<float> *zst = reinterpret_cast<cx<float> *>(smem + G::ZST);

    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63;
    const int p = l & 15, u = (l >> 4) & 1, e = l >> 5, c = 2 * u + e;
    const int ta = __builtin_amdgcn_readfirstlane(ta_in), tb = __builtin_amdgcn_readfirstlane(tb_in);
    const int flags = __builtin_amdgcn_readfirstlane(args.flags);
    const int nT = __builtin_amdgcn_readfirstlane(args.T), nTB = __builtin_amdgcn_readfirstlane(args.nTB);
    const float inv_s2 = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(args.inv_s2)));
    auto uniform_ptr = [](const void *q) {
        const unsigned long long v = reinterpret_cast<unsigned long long>(q);
        const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)v);
        const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(v >> 32));
        return reinterpret_cast<const char *>(((unsigned long long)hi << 32) | lo);
    };
    const char *Af = uniform_ptr(args.Af), *Bf = uniform_ptr(args.Bf);
    const bool do_best = flags & RADSVD_OUT_BEST;
    const bool do_lse = flags & RADSVD_OUT_LSE;

    // staging slot of pair P = 16 image + target (halves LDS bank conflicts of the result writes)
    auto sidx = [](int P) { return P ^ (((P >> 5) & 1) << 4); };
    const int Ps = sidx(16 * w + p);
    const int g = l >> 4, i16 = l & 15;    // MFMA result: rows 4g..4g+3 (images 2g, 2g+1), column i16

    // ---- operands: one block per (tile, q); the wave's frequency is scalar ----
    constexpr int PBA = NF * 512 + HF * 256;     // bytes per image plane
    constexpr int BBA = 3 * PBA;                 // image block
    constexpr int BBB = NF * 2048 + HF * 1024;   // target block
    const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(Af + (size_t)ta * (M + 1) * BBA), (short)0, (M + 1) * BBA, 0x00020000);
    auto rsrcB = [&](int t) {
        const char *Bb = Bf + ((size_t)t * nTB + tb) * (M + 1) * BBB;
        return __builtin_amdgcn_make_buffer_rsrc((void *)Bb, (short)0, (M + 1) * BBB, 0x00020000);
    };
    // job J of this wave: round J / 2; waves 0-3 take q = 8 R + 2 w + j (staging
    // slot 2 w + j), waves 4-7 q = M - 8 R - 2 (w - 4) - j (slot 8 + 2 (w - 4) + j);
    // job 2 NRP of wave 0 is the middle frequency M / 2
    constexpr int NJ = 2 * NRP;
    const bool lowerw = w < 4;
    const int wq = __builtin_amdgcn_readfirstlane(lowerw ? 2 * w : 2 * (w - 4));
    auto job_q = [&](int J) { return lowerw ? 8 * (J >> 1) + wq + (J & 1) : M - 8 * (J >> 1) - wq - (J & 1); };
    auto job_slot = [&](int J) { return (lowerw ? 0 : 8) + wq + (J & 1); };
    using FragT = WFrag<NF, HF>;
    auto load_at = [&](const __amdgpu_buffer_rsrc_t &rB, int q, FragT &f) {
        const int soffA = q * BBA, soffB = q * BBB;
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
#pragma unroll
            for (int hb = 0; hb < NF; ++hb)
                f.a[pl][hb] = __builtin_amdgcn_raw_buffer_load_b64(rA, 8 * l + pl * PBA + hb * 512, soffA, 0);
            if constexpr (HF) f.ah[pl] = __builtin_amdgcn_raw_buffer_load_b32(rA, 4 * l + pl * PBA + NF * 512, soffA, 0);
        }
#pragma unroll
        for (int hb = 0; hb < NF; ++hb)
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
                f.b[hb][s2] = __builtin_amdgcn_raw_buffer_load_b128(rB, 16 * l + hb * 2048 + s2 * 1024, soffB, 0);
        if constexpr (HF) f.bh = __builtin_amdgcn_raw_buffer_load_b128(rB, 16 * l + NF * 2048, soffB, 0);
    };

    // bf16 pairs (-1, 0) and (0, -1) for the exact remainders of the split (in
    // registers: as the folded inline constant -1.0 the first pair was read as
    // (0, -1) on gfx950)
    unsigned dmask0 = 0x0000bf80u, dmask1 = 0xbf800000u;
    asm volatile("" : "+v"(dmask0), "+v"(dmask1));
    // odd rows are Im rows: their own part is ai, which enters as -ai
    const unsigned sgn = (l & 1) ? 0x80008000u : 0u;

    // One job: the six split-bf16 products on v_mfma_f32_16x16x32_bf16 in one
    // accumulation chain (the order of k_pairs_fast); after_hi() runs once the
    // hi terms exist (the previous job's result goes to LDS there).
    auto mma = [&](const FragT &f, auto &&after_hi) -> f32x4 {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        constexpr int NFA = NF > 0 ? NF : 1;
        f32x4 ac = {0.f, 0.f, 0.f, 0.f};
        // image fragments: own part (sign-flipped in Im rows), then lane l ^ 1's
        u32x4 A[3][NFA];
        u32x2 Ah[3];
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
#pragma unroll
            for (int hb = 0; hb < NF; ++hb) {
                const u32x2 o = f.a[pl][hb];
                A[pl][hb] = u32x4{o[0] ^ sgn, o[1] ^ sgn, dpp_pair_swap(o[0]), dpp_pair_swap(o[1])};
            }
            if constexpr (HF) Ah[pl] = u32x2{f.ah[pl] ^ sgn, dpp_pair_swap(f.ah[pl])};
        }
        u32x4 pb_[NFA][3];
        u32x2 pbh[3];
        unsigned rb[NFA][8], rbh[4];
#pragma unroll
        for (int hb = 0; hb < NF; ++hb)
#pragma unroll
            for (int q = 0; q < 8; ++q) rb[hb][q] = f.b[hb][q >> 2][q & 3];
#pragma unroll
        for (int q = 0; q < 4; ++q) rbh[q] = f.bh[q];
        auto term = [&](unsigned &x0, unsigned &x1, bool last) -> unsigned {
            const bf16x2 tt = __builtin_convertvector(f32x2{__uint_as_float(x0), __uint_as_float(x1)}, bf16x2);
            if (!last) {
                x0 = __float_as_uint(__builtin_amdgcn_fdot2_f32_bf16(tt, __builtin_bit_cast(bf16x2, dmask0),
                                                                     __uint_as_float(x0), false));
                x1 = __float_as_uint(__builtin_amdgcn_fdot2_f32_bf16(tt, __builtin_bit_cast(bf16x2, dmask1),
                                                                     __uint_as_float(x1), false));
            }
            return __builtin_bit_cast(unsigned, tt);
        };
        auto stage_k = [&](auto KK) {
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
        using PR = Prec<3>;
        auto prod = [&](auto PP) {
            constexpr int pp = decltype(PP)::value;
#pragma unroll
            for (int hb = 0; hb < NF; ++hb)
                ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A[PR::pa(pp)][hb]),
                                                            __builtin_bit_cast(bf16x8, pb_[hb][PR::pb(pp)]), ac, 0, 0, 0);
        };
        // half chunk: two products in one 16x16x32 MFMA (a lane's first four depth
        // slots from the first product, the next four from the second, in A and B)
        auto half2 = [&](const u32x2 &a0, const u32x2 &a1, const u32x2 &b0, const u32x2 &b1) {
            const u32x4 av = {a0[0], a0[1], a1[0], a1[1]};
            const u32x4 bv = {b0[0], b0[1], b1[0], b1[1]};
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                        __builtin_bit_cast(bf16x8, bv), ac, 0, 0, 0);
        };
        stage_k(IC<0>{});
        after_hi();
        prod(IC<0>{});
        stage_k(IC<1>{});
        prod(IC<1>{});
        prod(IC<2>{});
        prod(IC<3>{});
        if constexpr (HF) {
            half2(Ah[0], Ah[0], pbh[1], pbh[0]);
            half2(Ah[1], Ah[2], pbh[1], pbh[0]);
        }
        stage_k(IC<2>{});
        prod(IC<4>{});
        prod(IC<5>{});
        if constexpr (HF) half2(Ah[1], Ah[0], pbh[0], pbh[2]);
        return ac;
    };
    const int put0 = sidx((2 * g) * 16 + i16), put1 = sidx((2 * g + 1) * 16 + i16);
    auto put = [&](int slot, f32x4 v) {
        lds_st(stage + slot * 128 + put0, cx<float>{v[0], v[1]});
        lds_st(stage + slot * 128 + put1, cx<float>{v[2], v[3]});
    };
    // Z[k] from S[k] (lo) and S[M - k] (hi)
    auto zfold = [](cx<float> lo, cx<float> hi, cx<float> tw) {
        const cx<float> uu = {lo.re + hi.re, lo.im - hi.im};
        const cx<float> vv = {lo.re - hi.re, lo.im + hi.im};
        const cx<float> pp = cmul(vv, tw);
        return cx<float>{uu.re - pp.im, uu.im + pp.re};
    };

    // per-lane element offsets of the fold's LDS accesses (kept as integers: the
    // pointers stay LDS pointers)
    const int spc = (4 - c) & 3;   // s' of the upper values is spc + 4 t2
    const int st_lo = c * 128 + Ps;      // lower values: slots c + 4 t2 and 8 + c + 4 t2
    const int st_up = spc * 128 + Ps;    // upper values: slots s' and 8 + s'
    const int zt_lo = c;                 // W_Q^{8 R + c + 4 t2}
    const int zt_up = M - spc - 8 * (NRP - 1) - 4;   // W_Q^{M - 8 R - spc - 4 t2}
    // zst entry of i = L4 - 2 R - t2 - (c != 0) is i - LO = (2 NRP - 1 - 2 R - t2) + (1 - (c != 0))
    const int zs_base = tid * G::ZLD + (c != 0 ? 0 : 1);

    // lane factor of the twiddles across e: W_M^{LO u + L4 e} = 1, W_8 (u), -i (e), W_8^3 (both)
    constexpr float r2 = 0.70710678118654752440f;
    const cx<float> lam = u ? (e ? cx<float>{-r2, -r2} : cx<float>{r2, -r2}) : (e ? cx<float>{0.f, -1.f} : cx<float>{1.f, 0.f});

    float run_best = -INFINITY;
    int run_idx = 0x7fffffff;
    bool run_nan = false;
    float run_m = -INFINITY, run_s = 0.f;

#ifndef WIDE_D
#define WIDE_D 2
#endif
    constexpr int D = WIDE_D;   // jobs in flight beyond the current one
    FragT fr[D + 1];
    {
        const __amdgpu_buffer_rsrc_t rB0 = rsrcB(0);
        sfor<0, D>([&](auto II) { load_at(rB0, job_q(decltype(II)::value), fr[decltype(II)::value]); });
    }
    for (int t = 0; t < nT; ++t) {
        const __amdgpu_buffer_rsrc_t rB = rsrcB(t);
#ifdef WIDE_NOPF
        if (t > 0) sfor<0, D>([&](auto II) { load_at(rB, job_q(decltype(II)::value), fr[decltype(II)::value]); });
#endif
        cx<float> x[LO];
        // ---------------- step 1: contraction, rounds of 16 frequencies ----------------
        sfor<0, NRP>([&](auto RR) {
            constexpr int R = decltype(RR)::value;
            f32x4 pend = {0.f, 0.f, 0.f, 0.f};
            sfor<0, 2>([&](auto JJ) {
                constexpr int jj = decltype(JJ)::value;
                constexpr int J = 2 * R + jj;
                if constexpr (J + D < NJ) {
                    load_at(rB, job_q(J + D), fr[(J + D) % (D + 1)]);
                } else if constexpr (J + D == NJ) {
                    if (w == 0) load_at(rB, M / 2, fr[(J + D) % (D + 1)]);
                }
                // keep the prefetch ahead of this job's MFMAs
                __builtin_amdgcn_sched_barrier(0);
                const f32x4 acc = mma(fr[J % (D + 1)], [&]() {
                    if constexpr (jj > 0) put(job_slot(J - 1), pend);
                });
                pend = acc;
            });
            put(job_slot(2 * R + 1), pend);
            __syncthreads();
            // fold: this lane's Z[k], k = 4 i + c, of the round's frequencies.
            // Addresses are per-lane bases (made opaque each round, so that the
            // compiler does not precompute every round's addresses into
            // registers) plus compile-time offsets.
            {
                int osl = st_lo, osu = st_up, ozl = zt_lo, ozu = zt_up, ozs = zs_base;
                asm volatile("" : "+v"(osl), "+v"(osu), "+v"(ozl), "+v"(ozu), "+v"(ozs));
                const cx<float> *sl = stage + osl, *su = stage + osu, *zl = ztab0 + ozl, *zu = ztab0 + ozu;
                cx<float> *zs = zst + ozs;
#pragma unroll
                for (int t2 = 0; t2 < 2; ++t2) {   // k = 8 R + c + 4 t2: i = 2 R + t2, in registers
                    cx<float> lo = lds_ld(sl + t2 * 512);          // S[k]       (slot c + 4 t2)
                    cx<float> hi = lds_ld(sl + 1024 + t2 * 512);   // S[M - k]   (slot 8 + c + 4 t2)
                    if (R == 0 && t2 == 0 && c == 0) {         // S[0] and S[M] are real
                        lo.im = 0.f;
                        hi.im = 0.f;
                    }
                    x[2 * R + t2] = zfold(lo, hi, lds_ld(zl + 8 * R + 4 * t2));
                    // computed here: left to the scheduler, the fold sinks to the
                    // transform and keeps its three inputs live instead of one result
                    asm volatile("" : "+v"(x[2 * R + t2].re), "+v"(x[2 * R + t2].im));
                }
#pragma unroll
                for (int t2 = 0; t2 < 2; ++t2) {   // k' = M - 8 R - s', s' = spc + 4 t2: i >= LO, to LDS
                    if (R > 0 || t2 > 0 || c != 0) {           // k' = M does not exist
                        const cx<float> lo = lds_ld(su + 1024 + t2 * 512);   // S[k']       (slot 8 + s')
                        const cx<float> hi = lds_ld(su + t2 * 512);          // S[M - k']   (slot s')
                        // i = L4 - 2 R - t2 - (c != 0): entry (i - LO) of the lane's zst row
                        const int col = 2 * NRP - 1 - 2 * R - t2;   // past the lane's base entry
                        lds_st(zs + col, zfold(lo, hi, lds_ld(zu + 8 * (NRP - 1 - R) + 4 * (1 - t2))));
                    }
                }
            }
            __syncthreads();   // the next round writes the staging buffer again
        });
        // middle frequency M / 2: Z[M/2] = 2 S[M/2], class 0, i = LO
        if (w == 0) put(0, mma(fr[NJ % (D + 1)], []() {}));
        __syncthreads();
        if (c == 0) {
            const cx<float> sm = lds_ld(stage + Ps);
            lds_st(zst + tid * G::ZLD, cx<float>{2.f * sm.re, 2.f * sm.im});
        }
        __syncthreads();
        // ---------------- step 2: transform, on chip ----------------
        // DIF split of the lane's sequence (x[i], i < LO, in registers; x[LO + i]
        // in the lane's zst row): x[i] + x[LO + i] has the even outputs of its
        // length-L4 DFT, (x[i] - x[LO + i]) W_{L4}^i the odd ones (back to LDS);
        // each half then takes one pass, so only L4 / 2 values are in registers
        cx<float> *zrow = zst + tid * G::ZLD;
        sfor<0, LO>([&](auto II) {
            constexpr int i = decltype(II)::value;
            const cx<float> b = lds_ld(zrow + i);
            const cx<float> a = x[i];
            x[i] = cadd(a, b);
            lds_st(zrow + i, twmul<i, L4>(csub(a, b)));
        });
        constexpr int F4 = LO / 2;   // butterflies per lane of a cross-lane step in one pass
        const int moff = LO * u + L4 * e;   // z index offset of this lane
        const bool do_full = flags & RADSVD_OUT_FULL;
        float bv[2][2], br[2][2];    // [pass][z index below / above M/2]: best of max(re, im), its re
        int bi[2][2];                //                                 landscape index of that pair
        float lse_mx = -INFINITY, lse_sum = 0.f;
        int bad = 0;
        auto half_pass = [&](auto PARITY) {
            constexpr int par = decltype(PARITY)::value;   // this lane's DFT outputs 2 n + par
            reg_fft_lp<LO, WIDE_FG>(x);                    // x[ct_pos(LO, n)] = output 2 n + par
            sfor<0, F4>([&](auto FF) {   // across u (lanes l, l ^ 16): n = 2 f + par + LO u
                constexpr int f = decltype(FF)::value;
                constexpr int ra = ct_pos(LO, f), rb = ct_pos(LO, f + F4);
                float nre, nim;
                x[ra].re = perm16_swap(x[ra].re, x[rb].re, nre);
                x[rb].re = nre;
                x[ra].im = perm16_swap(x[ra].im, x[rb].im, nim);
                x[rb].im = nim;
                const cx<float> a = x[ra];
                cx<float> b = x[rb];
                if (u) b = cx<float>{b.im, -b.re};          // W_{M/2}^{LO} = -i
                const cx<float> tt = twmul<2 * f + par, M / 2>(b);
                x[ra] = cadd(a, tt);   // X_e[n]
                x[rb] = csub(a, tt);   // X_e[n + L4]
            });
            sfor<0, F4>([&](auto FF) {   // across e (lanes l, l ^ 32): m = 2 f + par + LO u + L4 e
                constexpr int f = decltype(FF)::value;
                constexpr int ra = ct_pos(LO, f), rb = ct_pos(LO, f + F4);
                float nre, nim;
                x[ra].re = perm_swap_lo(x[ra].re, x[rb].re, nre);
                x[rb].re = nre;
                x[ra].im = perm_swap_lo(x[ra].im, x[rb].im, nim);
                x[rb].im = nim;
                const cx<float> a = x[ra];
                const cx<float> tt = twmul<2 * f + par, M>(cmul(x[rb], lam));
                x[ra] = cadd(a, tt);   // z[m]
                x[rb] = csub(a, tt);   // z[m + M / 2]
            });
            // every output sums every folded value, so one output per lane tells
            // whether the landscape of the pair is finite (barring overflow)
            if constexpr (par == 0) {
                const cx<float> z0 = x[ct_pos(LO, 0)];
                bad = (!__builtin_isfinite(z0.re) || !__builtin_isfinite(z0.im)) ? 1 : 0;
            }
            if (do_full && ta * 8 + w < args.n_img && tb * 16 + p < args.n_tgt) {
                // this lane's part of its pair's landscape row: X[2 n] = Re z[n], X[2 n + 1] = Im z[n]
                cx<float> *xo = args.X_full +
                                (((size_t)(ta * 8 + w) * args.n_tgt + (tb * 16 + p)) * (size_t)nT + t) * Q + 2 * moff;
                sfor<0, F4>([&](auto FF) {
                    constexpr int m0 = 4 * decltype(FF)::value + 2 * par;
                    const cx<float> za = x[ct_pos(LO, decltype(FF)::value)];
                    const cx<float> zb = x[ct_pos(LO, decltype(FF)::value + F4)];
                    xo[m0] = cx<float>{za.re, 0.f};
                    xo[m0 + 1] = cx<float>{za.im, 0.f};
                    xo[m0 + M] = cx<float>{zb.re, 0.f};
                    xo[m0 + M + 1] = cx<float>{zb.im, 0.f};
                });
            }
            if (do_best) {
                // a (re at 2 m, im at 2 m + 1) pair replaces the winner only when
                // strictly larger, so earlier m keep ties; NaN never wins (fmaxf drops it)
                float va = -INFINITY, vb = -INFINITY, ra_ = -INFINITY, rb_ = -INFINITY;
                int fa = 0, fb = 0;
                sfor<0, F4>([&](auto FF) {
                    constexpr int f = decltype(FF)::value;
                    const cx<float> za = x[ct_pos(LO, f)], zb = x[ct_pos(LO, f + F4)];
                    const float ma = fmaxf(za.re, za.im), mb = fmaxf(zb.re, zb.im);
                    if (ma > va) { va = ma; fa = f; ra_ = za.re; }
                    if (mb > vb) { vb = mb; fb = f; rb_ = zb.re; }
                });
                bv[par][0] = va; br[par][0] = ra_; bi[par][0] = 2 * (2 * fa + par + moff);
                bv[par][1] = vb; br[par][1] = rb_; bi[par][1] = 2 * (2 * fb + par + moff + M / 2);
            }
            if (do_lse) {
                float mx = -INFINITY;
                sfor<0, F4>([&](auto FF) {
                    constexpr int f = decltype(FF)::value;
                    const cx<float> za = x[ct_pos(LO, f)], zb = x[ct_pos(LO, f + F4)];
                    mx = fmaxf(mx, fmaxf(fmaxf(za.re, za.im), fmaxf(zb.re, zb.im)));
                });
                const float sm = inv_s2 * mx;
                float acc = 0.f;
                sfor<0, F4>([&](auto FF) {
                    constexpr int f = decltype(FF)::value;
                    const cx<float> za = x[ct_pos(LO, f)], zb = x[ct_pos(LO, f + F4)];
                    acc += __expf(fmaf(inv_s2, za.re, -sm)) + __expf(fmaf(inv_s2, za.im, -sm)) +
                           __expf(fmaf(inv_s2, zb.re, -sm)) + __expf(fmaf(inv_s2, zb.im, -sm));
                });
                const float nm = fmaxf(lse_mx, sm);
                lse_sum = lse_sum * __expf(lse_mx - nm) + acc * __expf(sm - nm);
                lse_mx = nm;
            }
        };
        half_pass(IC<0>{});
        sfor<0, LO>([&](auto II) { x[decltype(II)::value] = lds_ld(zrow + decltype(II)::value); });
        half_pass(IC<1>{});

        const int bad16 = __shfl_xor(bad, 16, 64), bad32 = __shfl_xor(bad, 32, 64);
        bad |= bad16 | bad32;
        bad |= __shfl_xor(bad, 32, 64);
        if (bad) run_nan = true;
        if (do_best) {
            // the winner of each tracker (its im value when its re value is smaller),
            // then the lane's best with ties to the smaller index
            float b0 = -INFINITY;
            int i0 = 0x7fffffff;
#pragma unroll
            for (int pp = 0; pp < 2; ++pp)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float v = bv[pp][h];
                    const int ix = bi[pp][h] + ((br[pp][h] == v) ? 0 : 1);
                    if (v > b0 || (v == b0 && ix < i0)) { b0 = v; i0 = ix; }
                }
            auto take = [&](int mask) {
                const float ob = __shfl_xor(b0, mask, 64);
                const int oi = __shfl_xor(i0, mask, 64);
                if (ob > b0 || (ob == b0 && oi < i0)) { b0 = ob; i0 = oi; }
            };
            take(16);
            take(32);
            if (b0 > run_best) { run_best = b0; run_idx = t * Q + i0; }
        }
        if (do_lse) {
            float lm = lse_mx, ls = lse_sum;
            auto merge = [&](int mask) {
                const float om = __shfl_xor(lm, mask, 64), os = __shfl_xor(ls, mask, 64);
                const float nm = fmaxf(lm, om);
                ls = ls * __expf(lm - nm) + os * __expf(om - nm);
                lm = nm;
            };
            merge(16);
            merge(32);
            const float rm = fmaxf(run_m, lm);
            run_s = run_s * __expf(run_m - rm) + ls * __expf(lm - rm);
            run_m = rm;
        }
        // the next translation's first jobs (issued once this translation's values
        // are consumed, so that they do not add to the transform's registers)
#ifndef WIDE_NOPF
        if (t + 1 < nT) {
#else
        if (false) {
#endif
            const __amdgpu_buffer_rsrc_t rB1 = rsrcB(t + 1);
            sfor<0, D>([&](auto II) { load_at(rB1, job_q(decltype(II)::value), fr[decltype(II)::value]); });
        }
        __syncthreads();   // zst and the staging buffer are reused by the next translation
    }

    const int a = ta * 8 + w, b = tb * 16 + p;
    if ((l >> 4) == 0 && a < args.n_img && b < args.n_tgt) {
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

template <int Q, int NF, int HF>
#ifndef WIDE_LB
#define WIDE_LB 1
#endif
__global__ __attribute__((amdgpu_flat_work_group_size(1, WIDE_LB ? 512 : 256))) void k_pairs_wide(Args args) {
    extern __shared__ unsigned char smem_raw[];
    wide_tables<Q>(smem_raw);
    int ta, tb;
    tile_of(blockIdx.x, gridDim.x, args.nTA, args.nTB, args.band, ta, tb);
    wide_tile<Q, NF, HF>(args, ta, tb, smem_raw);
}

template <int Q, int NF, int HF>
static hipError_t launch_wide_v(const Args &a, int nwg, hipStream_t s) {
    constexpr size_t shmem = WideGeom<Q>::BYTES;
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute((const void *)k_pairs_wide<Q, NF, HF>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    hipLaunchKernelGGL((k_pairs_wide<Q, NF, HF>), dim3(nwg), dim3(512), shmem, s, a);
    return hipGetLastError();
}

template <int Q>
static hipError_t launch_wide_h(const Args &a, int nwg, int H8, hipStream_t s) {
    switch (H8) {
    case 8: return launch_wide_v<Q, 0, 1>(a, nwg, s);
    case 16: return launch_wide_v<Q, 1, 0>(a, nwg, s);
    case 24: return launch_wide_v<Q, 1, 1>(a, nwg, s);
    case 32: return launch_wide_v<Q, 2, 0>(a, nwg, s);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_wide(const Args &a, int Q, int nwg, int H8, hipStream_t s);

}  // namespace fastk
}  // namespace radsvd
