// Shared device helpers of the radsvd HIP library (gfx950).
//
// * cx<R>        : interleaved complex value (matches complex64 / complex128).
// * bf16 helpers : round-to-nearest-even split of an FP32 value into
//                  hi + mid + lo bf16 terms (each term is the rounding of what
//                  the previous terms left), the operand format of the
//                  split-precision contraction.
// * FftPlan / lds_fft_dif : in-place mixed-radix (8, 4, 2, 3) decimation-in-
//                  frequency FFT of sequences held in LDS; the output of
//                  frequency f sits at position fft_pos(f).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace radsvd {

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return {a.re * s, a.im * s}; }
// -i * a
template <typename R>
__device__ __forceinline__ cx<R> cmul_mi(cx<R> a) { return {a.im, -a.re}; }

// ---------------------------------------------------------------------------
// bf16 (round to nearest even; NaN kept quiet)
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u;
    __builtin_memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float x;
    __builtin_memcpy(&x, &u, 4);
    return x;
}
// x = hi + mid + lo (+ a remainder below 2^-24 |x|).  x - hi and the next
// remainder are exact in FP32.
__host__ __device__ __forceinline__ void split3_bf16(float x, uint16_t &hi, uint16_t &mid, uint16_t &lo) {
    hi = f32_to_bf16_rne(x);
    float r1 = x - bf16_to_f32(hi);
    mid = f32_to_bf16_rne(r1);
    float r2 = r1 - bf16_to_f32(mid);
    lo = f32_to_bf16_rne(r2);
}

// ---------------------------------------------------------------------------
// mixed-radix plan: n = 4^a 2^b 3^c
// ---------------------------------------------------------------------------
struct FftPlan {
    int n;
    int nst;
    int rad[16];
    int span[16];   // block length after stage s (= current length / radix)
    // x / d = umulhi(x, ceil(2^32 / d)) for the stage divisors d = n / rad and
    // d = span, exact for x < 2^20 and 2 <= d <= 2^11; d = 1 is stored as 0
    // (ceil(2^32 / 1) does not fit) and handled by fft_div
    unsigned mag_seq[16], mag_span[16];
};

__host__ __device__ inline unsigned fft_magic(unsigned d) {
    return d <= 1 ? 0u : (unsigned)((((unsigned long long)1 << 32) + d - 1) / d);
}
__device__ __forceinline__ int fft_div(int x, unsigned magic) {
    return magic ? (int)__umulhi((unsigned)x, magic) : x;
}

__host__ __device__ inline bool fft_size_ok(int n) {
    if (n < 2) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// fills p in place (p may live in LDS: no private-memory copy)
__host__ __device__ inline void fft_init_plan(FftPlan &p, int n) {
    p.n = n;
    p.nst = 0;
    int m = n;
    while (m % 8 == 0) { p.rad[p.nst++] = 8; m /= 8; }
    while (m % 4 == 0) { p.rad[p.nst++] = 4; m /= 4; }
    while (m % 2 == 0) { p.rad[p.nst++] = 2; m /= 2; }
    while (m % 3 == 0) { p.rad[p.nst++] = 3; m /= 3; }
    int L = n;
    for (int s = 0; s < p.nst; ++s) {
        L /= p.rad[s];
        p.span[s] = L;
        p.mag_seq[s] = fft_magic((unsigned)(n / p.rad[s]));
        p.mag_span[s] = fft_magic((unsigned)L);
    }
}

__host__ __device__ inline FftPlan fft_make_plan(int n) {
    FftPlan p;
    fft_init_plan(p, n);
    return p;
}

// position of frequency f in the DIF output: f = p0 + R0 (p1 + R1 (p2 + ...)),
// pos = sum_s p_s span_s.
__host__ __device__ inline int fft_pos(int f, const FftPlan &p) {
    int pos = 0;
    for (int s = 0; s < p.nst; ++s) {
        int d = f % p.rad[s];
        f /= p.rad[s];
        pos += d * p.span[s];
    }
    return pos;
}

template <typename R>
__device__ __forceinline__ void dft4(cx<R> *v) {
    cx<R> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    cx<R> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, cmul_mi(t3));
    v[3] = csub(t1, cmul_mi(t3));
}

// Forward DFT of radix 2/3/4/8 on v[0..R): y_p = sum_r v_r exp(-2 pi i r p / R).
template <typename R>
__device__ __forceinline__ void dft_small(int rad, cx<R> *v) {
    if (rad == 8) {
        // two length-4 DFTs (even, odd samples) joined by W_8^p, W_8 = (1 - i) / sqrt 2
        cx<R> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        dft4(e);
        dft4(o);
        const R s = (R)0.7071067811865475244008443621048490;
        const cx<R> o1 = {s * (o[1].re + o[1].im), s * (o[1].im - o[1].re)};    // W_8 o[1]
        const cx<R> o2 = cmul_mi(o[2]);                                         // W_8^2 = -i
        const cx<R> o3 = {s * (o[3].im - o[3].re), -s * (o[3].re + o[3].im)};   // W_8^3 = -(1 + i) / sqrt 2
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    } else if (rad == 2) {
        cx<R> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (rad == 4) {
        dft4(v);
    } else {  // 3
        const R h = (R)0.8660254037844386467637231707529362;   // sqrt(3)/2
        cx<R> a = v[0];
        cx<R> t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
        cx<R> m = {a.re - (R)0.5 * t1.re, a.im - (R)0.5 * t1.im};
        cx<R> u = {h * t2.im, -h * t2.re};                       // -i (sqrt3/2) t2
        v[0] = cadd(a, t1);
        v[1] = cadd(m, u);
        v[2] = csub(m, u);
    }
}

template <int RAD, typename R>
__device__ __forceinline__ void fft_butterfly(cx<R> *x, int span, int k, int tstep, int, const cx<R> *tw) {
    cx<R> v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = x[r * span];
    dft_small(RAD, v);
    x[0] = v[0];
#pragma unroll
    for (int p = 1; p < RAD; ++p) x[p * span] = cmul(v[p], tw[k * p * tstep]);   // k p tstep < n
}

// In-place forward FFT (exp(-2 pi i f j / n)) of `cnt` sequences of length n
// stored at buf + s*seq_stride; tw[i] = exp(-2 pi i i / n) for i < n.
// All threads of the block cooperate; ends with a barrier.
template <typename R>
__device__ void lds_fft_dif(cx<R> *buf, int cnt, int seq_stride, const FftPlan &pl,
                            const cx<R> *tw) {
    const int n = pl.n;
    int L = n;
    for (int s = 0; s < pl.nst; ++s) {
        const int rad = pl.rad[s];
        const int span = L / rad;
        const int per_seq = n / rad;
        const int nbf = cnt * per_seq;
        const int tstep = n / L;
        const unsigned ms = pl.mag_seq[s], mp = pl.mag_span[s];
        for (int i = threadIdx.x; i < nbf; i += blockDim.x) {
            const int sq = fft_div(i, ms);
            const int bi = i - sq * per_seq;
            const int blk = fft_div(bi, mp);
            const int k = bi - blk * span;
            cx<R> *x = buf + (size_t)sq * seq_stride + blk * L + k;
            // one butterfly per radix with a fixed-size register array
            if (rad == 8) fft_butterfly<8>(x, span, k, tstep, n, tw);
            else if (rad == 4) fft_butterfly<4>(x, span, k, tstep, n, tw);
            else if (rad == 2) fft_butterfly<2>(x, span, k, tstep, n, tw);
            else fft_butterfly<3>(x, span, k, tstep, n, tw);
        }
        __syncthreads();
        L = span;
    }
}

}  // namespace radsvd
