// Fused Hermitian pair kernel on the gfx950 matrix cores.
//
// Paper section 3.3 (two-step evaluation with principal rings, steps 1-2) for
// Hermitian inputs (real images, section 2.5 conjugacy):
//   step 1  S[q] = sum_h conj(At[a][h][q]) Bt[b][t][h][q],   q in [0, M], M = Q/2
//   step 2  X[m] = sum_{q<Q} S[q] exp(-2 pi i q m / Q)        (S[Q-q] = conj S[q])
// then the maximum over (t, m) (section 2.6) and/or the log-sum-exp, without
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
// BF16x3: v_mfma_f32_16x16x32_bf16 over the concatenated split products
//         (hi*hi, hi*mid, mid*hi [, mid*mid, hi*lo, lo*hi]); FP32 accumulation.
// The operand layout written by the prepare kernel keeps, for a fixed (tile,
// q), the 8 (16) image (target) rows contiguous: [row][plane][re|im][h].
//
// Step 2: every pair is owned by two lanes (l and l + 32 of one wavefront).
// The half-spectrum S[0..M] becomes the length-M complex sequence
//   Z[k] = (S[k] + conj S[M-k]) + i W_Q^k (S[k] - conj S[M-k]),
// whose length-M DFT z gives X[2n] = Re z[n], X[2n+1] = Im z[n].  Lane
// e = 0 holds Z at even k, lane e = 1 at odd k; each runs an in-register
// FFT of length L = M/2, and one radix-2 stage across the two lanes
// (v_permlane32_swap) completes z.  Everything in step 2 is FP32 VALU.
#include <string.h>

#include <type_traits>

#include "common.h"
#include "internal.h"

namespace radsvd {
namespace fastk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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
    int H8;
    int rowElems;              // elements per (row) = nplanes * 2 * H8
    int nprod;                 // split products (bf16) ; unused for FP32
    int planeA[6], planeB[6];  // plane of each product term
    int flags;
    float inv_s2;
    float *best_score;
    int32_t *best_m, *best_t;
    float *lse_pair;
};

// tile index of workgroup `wg`: workgroups are dealt round-robin to the 8
// XCDs; consecutive workgroups of one XCD walk an 8-row band of image tiles
// with the target tile advancing every 8, so the XCD's concurrently resident
// workgroups share image and target operand rows in its L2.
__device__ __forceinline__ void tile_of(int wg, int nwg, int nTA, int nTB, int &ta, int &tb) {
    const int xcd = wg & 7;
    const int full = nwg >> 3, rem = nwg & 7;
    const int lin = xcd * full + min(xcd, rem) + (wg >> 3);
    const int band = lin / (8 * nTB);
    const int rows = min(8, nTA - band * 8);
    const int in_band = lin - band * 8 * nTB;
    ta = band * 8 + in_band % rows;
    tb = in_band / rows;
}

template <int Q, bool BF16, int MODE>
__global__ __launch_bounds__(256, 1) void k_pairs_fast(Args args) {
    constexpr int M = Q / 2;
    constexpr int L = M / 2;        // per-lane FFT length (complex)
    constexpr int NRF = M / 8;      // full rounds of 8 frequencies; q = M handled last
    static_assert(M % 8 == 0, "Q must be a multiple of 16");

    __shared__ cx<float> stage[2][8][128];

    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wavefront (uniform)
    const int l = tid & 63;
    const int e = l >> 5;           // 0: even-k lane, 1: odd-k lane
    const int P = 32 * w + (l & 31);// pair within the tile
    const int pa = P >> 4, pb = P & 15;

    int ta, tb;
    tile_of(blockIdx.x, gridDim.x, args.nTA, args.nTB, ta, tb);

    // ---- MFMA operand roles of this lane ----
    const int g = l >> 4;           // k-group of the MFMA operand
    const int i16 = l & 15;         // row (A) / column (B) of the MFMA operand
    const int H8 = args.H8;
    const int rowE = args.rowElems;
    const int esz = BF16 ? 2 : 4;
    const int ai = i16 >> 1, rt = i16 & 1;
    // BF16: lane covers 8 h-values: part c = g >> 1, h block (g & 1) (+ 2 * hb_hi)
    // FP32: lane covers H8/2 h-values: part c = g >> 1, half (g & 1)
    const int c = g >> 1, hsub = g & 1;
    const int cc = rt ? 1 - c : c;
    const unsigned negm = (rt == 1 && c == 0) ? (BF16 ? 0x80008000u : 0x80000000u) : 0u;
    const int hoff = BF16 ? 8 * hsub : (H8 / 2) * hsub;
    const int voffA = (ai * rowE + cc * H8 + hoff) * esz;
    const int voffB = (i16 * rowE + c * H8 + hoff) * esz;
    const int nhb = (H8 + 15) >> 4;               // BF16: h blocks of 16 per lane pair
    const bool padlast = BF16 && ((H8 >> 3) & 1) && hsub == 1;
    const unsigned padm = padlast ? 0u : 0xffffffffu;

    const size_t rowBytes = (size_t)rowE * esz;
    const size_t qBytesA = (size_t)8 * rowBytes;   // one q of an image tile
    const size_t qBytesB = (size_t)16 * rowBytes;  // one q of a target tile
    const char *Abase = reinterpret_cast<const char *>(args.Af) + (size_t)ta * (M + 1) * qBytesA;
    const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
        (void *)Abase, (short)0, (int)((M + 1) * qBytesA), 0x00020000);

    // running results over t
    float run_best = -INFINITY;
    int run_idx = 0x7fffffff;
    bool run_nan = false;
    float run_m = -INFINITY, run_s = 0.f;

    for (int t = 0; t < args.T; ++t) {
        const char *Bbase = reinterpret_cast<const char *>(args.Bf) +
                            ((size_t)t * args.nTB + tb) * (M + 1) * qBytesB;
        const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
            (void *)Bbase, (short)0, (int)((M + 1) * qBytesB), 0x00020000);

        // one frequency q: 16x16 block of [Re S; Im S](image, target)
        auto contract = [&](int q) -> f32x4 {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const int sA = q * (int)qBytesA, sB = q * (int)qBytesB;
            if constexpr (BF16) {
                for (int p = 0; p < args.nprod; ++p) {
                    const int pA = args.planeA[p] * 2 * H8 * 2, pB = args.planeB[p] * 2 * H8 * 2;
                    for (int hb = 0; hb < nhb; ++hb) {
                        u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rA, voffA, sA + pA + 32 * hb, 0);
                        u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(rB, voffB, sB + pB + 32 * hb, 0);
                        a ^= negm;
                        if (hb == nhb - 1) {
                            a &= padm;
                            b &= padm;
                        }
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
                    }
                }
            } else {
                for (int hc = 0; hc < (H8 >> 3); ++hc) {
                    u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rA, voffA, sA + 16 * hc, 0);
                    u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(rB, voffB, sB + 16 * hc, 0);
                    a ^= negm;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[j]), __uint_as_float(b[j]),
                                                                  acc, 0, 0, 0);
                }
            }
            return acc;
        };
        // rows 4g..4g+3 of the block: images 2g, 2g+1 (Re, Im) at target column i16
        auto put = [&](int buf, int qq, f32x4 v) {
            stage[buf][qq][(2 * g) * 16 + i16] = cx<float>{v[0], v[1]};
            stage[buf][qq][(2 * g + 1) * 16 + i16] = cx<float>{v[2], v[3]};
        };

        cx<float> st[L];
        sfor<0, NRF>([&](auto RR) {
            constexpr int R = decltype(RR)::value;
            constexpr int buf = R & 1;
            const int q0 = 8 * R + 2 * w;
            f32x4 a0 = contract(q0);
            f32x4 a1 = contract(q0 + 1);
            put(buf, 2 * w, a0);
            put(buf, 2 * w + 1, a1);
            __syncthreads();
            sfor<0, 4>([&](auto JJ) {
                constexpr int j = decltype(JJ)::value;
                st[4 * R + j] = stage[buf][2 * j + e][P];
            });
        });
        {   // q = M (Nyquist): real, kept in the imaginary slot of lane e = 0's S[0]
            constexpr int buf = NRF & 1;
            if (w == 0) {
                f32x4 a0 = contract(M);
                put(buf, 0, a0);
            }
            __syncthreads();
            const float sM = stage[buf][0][P].re;
            if (e == 0) st[0].im = sM;
        }

        // ---- Z sequence (in place): lane 0 even k, lane 1 odd k ----
        auto zpair = [&](cx<float> &x, cx<float> &y, auto kk) {
            constexpr int k = decltype(kk)::value;
            const cx<float> u = {x.re + y.re, x.im - y.im};      // S[k] + conj S[M-k]
            const cx<float> v = {x.re - y.re, x.im + y.im};      // S[k] - conj S[M-k]
            const cx<float> p = twmul<k, Q>(v);
            x = cx<float>{u.re - p.im, u.im + p.re};              // Z[k]
            y = cx<float>{u.re + p.im, p.re - u.im};              // Z[M-k]
        };
        if (e == 0) {
            const float s0 = st[0].re, sM = st[0].im;
            st[0] = cx<float>{s0 + sM, s0 - sM};
            sfor<1, L / 2>([&](auto II) {
                constexpr int ii = decltype(II)::value;
                zpair(st[ii], st[L - ii], IC<2 * ii>{});
            });
            st[L / 2] = cx<float>{2.f * st[L / 2].re, 2.f * st[L / 2].im};
        } else {
            sfor<0, L / 2>([&](auto II) {
                constexpr int ii = decltype(II)::value;
                zpair(st[ii], st[L - 1 - ii], IC<2 * ii + 1>{});
            });
        }

        reg_fft<L>(st);   // lane 0: E[f] = DFT_L(Z[2k']), lane 1: O[f] = DFT_L(Z[2k'+1])

        // ---- cross-lane radix-2 and epilogue ----
        float bl = -INFINITY, bh = -INFINITY;
        int il = 0x7fffffff, ih = 0x7fffffff;
        float mx = -INFINITY;
        float firstX = 0.f;
        sfor<0, L / 2>([&](auto JJ) {
            constexpr int j = decltype(JJ)::value;
            constexpr int ra = ct_pos(L, j), rb = ct_pos(L, L / 2 + j);
            // lane 0 sends E[L/2 + j], lane 1 sends O[j]
            float nre, nim;
            st[ra].re = perm_swap_lo(st[ra].re, st[rb].re, nre);
            st[rb].re = nre;
            st[ra].im = perm_swap_lo(st[ra].im, st[rb].im, nim);
            st[rb].im = nim;
            const cx<float> a = st[ra];          // E[n]
            cx<float> b = st[rb];                // O[n], n = j + e L/2
            if (e) b = cx<float>{b.im, -b.re};   // W_M^{L/2} = -i
            const cx<float> tw = twmul<j, M>(b);
            st[ra] = cadd(a, tw);                // z[n]     -> X[2n], X[2n+1]
            st[rb] = csub(a, tw);                // z[n + L] -> X[2n + M], X[2n + M + 1]
            if constexpr (j == 0) firstX = st[ra].re;
        });
        if constexpr (MODE & 1) {
            sfor<0, L / 2>([&](auto JJ) {
                constexpr int j = decltype(JJ)::value;
                const cx<float> zl = st[ct_pos(L, j)], zh = st[ct_pos(L, L / 2 + j)];
                if (zl.re > bl) { bl = zl.re; il = 2 * j; }
                if (zl.im > bl) { bl = zl.im; il = 2 * j + 1; }
                if (zh.re > bh) { bh = zh.re; ih = 2 * j + M; }
                if (zh.im > bh) { bh = zh.im; ih = 2 * j + M + 1; }
            });
        }
        if constexpr (MODE & 2) {
            sfor<0, L / 2>([&](auto JJ) {
                constexpr int j = decltype(JJ)::value;
                const cx<float> zl = st[ct_pos(L, j)], zh = st[ct_pos(L, L / 2 + j)];
                mx = fmaxf(mx, fmaxf(fmaxf(zl.re, zl.im), fmaxf(zh.re, zh.im)));
            });
        }
        const bool isnanX = __builtin_isnan(firstX) || __builtin_isnan(__shfl_xor(firstX, 32, 64));
        if constexpr (MODE & 1) {
            // lane-local winner (low half wins ties), then across the lane pair
            if (bh > bl) { bl = bh; il = ih; }
            il += e * L;
            const float ob = __shfl_xor(bl, 32, 64);
            const int oi = __shfl_xor(il, 32, 64);
            if (ob > bl || (ob == bl && oi < il)) { bl = ob; il = oi; }
            if (isnanX) run_nan = true;
            const int gidx = t * Q + il;
            if (bl > run_best) { run_best = bl; run_idx = gidx; }
        }
        if constexpr (MODE & 2) {
            const float s = args.inv_s2;
            mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
            const float sm = s * mx;
            float acc = 0.f;
            sfor<0, L / 2>([&](auto JJ) {
                constexpr int j = decltype(JJ)::value;
                const cx<float> zl = st[ct_pos(L, j)], zh = st[ct_pos(L, L / 2 + j)];
                acc += __expf(fmaf(s, zl.re, -sm)) + __expf(fmaf(s, zl.im, -sm)) +
                       __expf(fmaf(s, zh.re, -sm)) + __expf(fmaf(s, zh.im, -sm));
            });
            acc += __shfl_xor(acc, 32, 64);
            if (isnanX) run_nan = true;
            const float nm = fmaxf(run_m, sm);
            run_s = run_s * __expf(run_m - nm) + acc * __expf(sm - nm);
            run_m = nm;
        }
        __syncthreads();
    }

    const int a = ta * 8 + pa, b = tb * 16 + pb;
    if (e == 0 && a < args.n_img && b < args.n_tgt) {
        const size_t o = (size_t)a * args.n_tgt + b;
        if constexpr (MODE & 1) {
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
        if constexpr (MODE & 2) args.lse_pair[o] = run_nan ? __builtin_nanf("") : run_m + __logf(run_s);
    }
}

template <int Q, bool BF16>
static hipError_t launch_q(const Args &a, int nwg, int mode, hipStream_t s) {
    switch (mode) {
    case 1: hipLaunchKernelGGL((k_pairs_fast<Q, BF16, 1>), dim3(nwg), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_pairs_fast<Q, BF16, 2>), dim3(nwg), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_pairs_fast<Q, BF16, 3>), dim3(nwg), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

template <bool BF16>
static hipError_t launch_prec(const Args &a, int Q, int nwg, int mode, hipStream_t s) {
    switch (Q) {
    case 64: return launch_q<64, BF16>(a, nwg, mode, s);
    case 96: return launch_q<96, BF16>(a, nwg, mode, s);
    case 128: return launch_q<128, BF16>(a, nwg, mode, s);
    case 192: return launch_q<192, BF16>(a, nwg, mode, s);
    case 256: return launch_q<256, BF16>(a, nwg, mode, s);
    case 384: return launch_q<384, BF16>(a, nwg, mode, s);
    case 512: return launch_q<512, BF16>(a, nwg, mode, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace fastk

static bool fast_q_ok(int Q) {
    return Q == 64 || Q == 96 || Q == 128 || Q == 192 || Q == 256 || Q == 384 || Q == 512;
}

bool fast_path_supported(const radsvd_plan *p, int flags) {
    if (!p->herm || p->prec == RADSVD_FP64 || !p->Af || !p->Bf) return false;
    if (flags & ~(RADSVD_OUT_BEST | RADSVD_OUT_LSE)) return false;
    return fast_q_ok(p->Q);
}

bool fast_tile_ok(int tile_b) { return tile_b == 0 || tile_b == 16; }

hipError_t launch_pairs_fast(const radsvd_plan *p, int flags, float inv_s2, float *best_score,
                             int32_t *best_m, int32_t *best_t, float *lse_pair, hipStream_t s) {
    fastk::Args a;
    memset(&a, 0, sizeof(a));
    a.Af = p->Af;
    a.Bf = p->Bf;
    a.n_img = p->n_img;
    a.n_tgt = p->n_tgt;
    a.T = p->T;
    a.nTA = p->na_pad / kFastTA;
    a.nTB = p->nb_pad / kFastTB;
    a.H8 = p->H8;
    a.rowElems = p->nplanes * 2 * p->H8;
    const bool bf = p->prec != RADSVD_FP32;
    if (bf) {
        static const int pa3[6] = {0, 0, 1, 1, 0, 2};
        static const int pb3[6] = {0, 1, 0, 1, 2, 0};
        a.nprod = p->prec == RADSVD_BF16 ? 1 : p->products;
        for (int i = 0; i < 6; ++i) {
            a.planeA[i] = pa3[i];
            a.planeB[i] = pb3[i];
        }
    }
    a.flags = flags;
    a.inv_s2 = inv_s2;
    a.best_score = best_score;
    a.best_m = best_m;
    a.best_t = best_t;
    a.lse_pair = lse_pair;
    const int nwg = a.nTA * a.nTB;
    const int mode = flags & 3;
    return bf ? fastk::launch_prec<true>(a, p->Q, nwg, mode, s)
              : fastk::launch_prec<false>(a, p->Q, nwg, mode, s);
}

}  // namespace radsvd
