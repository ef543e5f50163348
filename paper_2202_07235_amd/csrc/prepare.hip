// Precompute kernels: grid factors, translation phases, U*eta, and the
// principal rings of every image and translated target, transformed to
// angular frequency (paper section 3.2, principal image rings; section 2.3,
// angular Fourier coefficients; section 3.5, precompute items).
//
// The recombination K -> H is applied in psi-space before the angular FFT:
// both maps are linear and commute, and transforming H principal rings
// instead of K rings cuts the FFT work by K/H.
#include <math.h>

#include <type_traits>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace radsvd {

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// grid factors and translation phases, computed in FP64
//   eta_r = sqrt(w_r dpsi)                      (section 2.6, ring rescaling)
//   phi_t[r][j] = exp(-i k_r (dx cos psi_j + dy sin psi_j))
//                 (transform of B(x - delta), section 2.1)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_setup(GridArgs g, double *d_k, double *d_eta, double *d_delta, cx<R> *phase) {
    const int K = g.K, Q = g.Q, T = g.T;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < K) {
        d_k[gid] = g.k[gid];
        d_eta[gid] = sqrt(g.w[gid] * (2.0 * M_PI / (double)Q));
    }
    if (gid < 2 * T) d_delta[gid] = (&g.delta[0][0])[gid];
    const int total = T * K * Q;
    for (int i = gid; i < total; i += gridDim.x * blockDim.x) {
        const int j = i % Q;
        const int r = (i / Q) % K;
        const int t = i / (Q * K);
        double s, c;
        sincospi(2.0 * (double)j / (double)Q, &s, &c);
        const double arg = g.k[r] * (g.delta[t][0] * c + g.delta[t][1] * s);
        double ps, pc;
        sincos(arg, &ps, &pc);
        phase[i] = cx<R>{(R)pc, (R)(-ps)};
    }
}

template <typename R>
__global__ void k_ueta(const double *U, int ld, const double *eta, int K, int H, R *Ueta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K * H) {
        const int r = i / H, h = i - r * H;
        Ueta[i] = (R)(U[(size_t)r * ld + h] * eta[r]);
    }
}

// ---------------------------------------------------------------------------
// principal rings + angular FFT
//
// One workgroup per (item n, translation t).  Phase 1: thread j owns the
// angles psi_j, psi_{j+256} and accumulates, for every h of the current pass,
//   Y[h][j] = sum_r Ueta[r][h] * phi_t[r][j] * X[n][r][j]
// (Ueta[r][h] is uniform across the workgroup and is read as a scalar
// operand; no barrier inside the ring loop).  Phase 2 transforms rows of Y
// in LDS:  y[h][q] = Q^{-1/2} sum_j Y[h][j] exp(-2 pi i q j / Q)  and writes
// q in [0, Qc) to
//   generic layout  G[n][t][q][h]                      (cx<R>)
//   fast layout     F[t][tile][q] operand blocks in MFMA fragment order
//                   (FP32 or bf16 planes), zero-filled beforehand, so that
//                   padding items and ranks h in [H, H8) stay zero.
// ---------------------------------------------------------------------------
// Output of one item's principal rings: rows y[0..nrows) of ybuf (row
// stride Q, psi order) are transformed in LDS, scaled by Q^{-1/2}, and
// frequencies q < Qc of rows h0 + i are written to the generic layout and,
// for the fast path, to the fragment-ordered operand block of (t, tile, q).
// Called by all threads; starts with the FFT's barriers.
template <typename R>
__device__ void emit_rows(cx<R> *ybuf, int nrows, int h0, int n, int t, int T, int Q, int H, int Qc,
                          const FftPlan &pl, const cx<R> *tw, cx<R> *__restrict__ G, void *__restrict__ F,
                          int f_kind, int f_tile, int f_ntiles, int H8, int nplanes, int is_img) {
    const bool fbf = f_kind == kFragBF16;   // bf16 planes; otherwise FP32 values
    const int planeB = frag_plane_bytes(f_kind, H8);
    const size_t blockB = (size_t)nplanes * planeB;
    const int f_q = (Qc == Q) ? Q : Q / 2 + 1;
    const int tile = n / f_tile, n_in = n - tile * f_tile;
    const R scale = (R)(1.0 / sqrt((double)Q));
    lds_fft_dif(ybuf, nrows, Q, pl, tw);
    for (int i = threadIdx.x; i < Qc * nrows; i += blockDim.x) {
        const int q = i / nrows, hh = i - q * nrows;
        const int h = h0 + hh;
        cx<R> v = ybuf[hh * Q + fft_pos(q, pl)];
        v.re *= scale;
        v.im *= scale;
        if (G) G[(((size_t)n * T + t) * H + h) * Qc + q] = v;
        if (F) {
            // image n_in: Re row 2 n_in = [ar | ai], Im row 2 n_in + 1 = [-ai | ar];
            // target n_in: column [br | bi]
            char *blk = reinterpret_cast<char *>(F) + (((size_t)t * f_ntiles + tile) * f_q + q) * blockB;
            const int r0 = is_img ? 2 * n_in : n_in;
            const int o_re = frag_elem_offset(f_kind, H8, r0, 0, h);
            const int o_im = frag_elem_offset(f_kind, H8, r0, 1, h);
            const int o_nim = is_img ? frag_elem_offset(f_kind, H8, r0 + 1, 0, h) : 0;
            const int o_re2 = is_img ? frag_elem_offset(f_kind, H8, r0 + 1, 1, h) : 0;
            if (!fbf) {
                *reinterpret_cast<float *>(blk + o_re) = (float)v.re;
                *reinterpret_cast<float *>(blk + o_im) = (float)v.im;
                if (is_img) {
                    *reinterpret_cast<float *>(blk + o_nim) = -(float)v.im;
                    *reinterpret_cast<float *>(blk + o_re2) = (float)v.re;
                }
            } else {
                uint16_t hr[3], hi_[3];
                split3_bf16((float)v.re, hr[0], hr[1], hr[2]);
                split3_bf16((float)v.im, hi_[0], hi_[1], hi_[2]);
#pragma unroll
                for (int pl_i = 0; pl_i < 3; ++pl_i) {
                    if (pl_i >= nplanes) break;
                    char *pb = blk + (size_t)pl_i * planeB;
                    *reinterpret_cast<uint16_t *>(pb + o_re) = hr[pl_i];
                    *reinterpret_cast<uint16_t *>(pb + o_im) = hi_[pl_i];
                    if (is_img) {
                        *reinterpret_cast<uint16_t *>(pb + o_nim) = hi_[pl_i] ^ 0x8000u;
                        *reinterpret_cast<uint16_t *>(pb + o_re2) = hr[pl_i];
                    }
                }
            }
        }
    }
}

template <typename R, int HP>
__global__ __launch_bounds__(256) void k_rings(
    const cx<R> *__restrict__ X, int n_real, int T, const cx<R> *__restrict__ phase,
    const R *__restrict__ Ueta, int K, int Q, int H, int Qc, int FC,
    cx<R> *__restrict__ G,                                       // may be null
    void *__restrict__ F, int f_kind, int f_tile, int f_ntiles, int H8, int nplanes, int is_img) {
    extern __shared__ unsigned char smem_raw[];
    const int n = blockIdx.x / T;
    const int t = blockIdx.x - n * T;
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    cx<R> *tw = reinterpret_cast<cx<R> *>(smem_raw);             // [Q]
    cx<R> *ybuf = tw + Q;                                         // [FC][Q]
    if (n >= n_real) return;

    for (int i = tid; i < Q; i += nthreads) {
        double s, c;
        sincospi(-2.0 * (double)i / (double)Q, &s, &c);
        tw[i] = cx<R>{(R)c, (R)s};
    }
    __shared__ FftPlan spl;   // in LDS: the stage loops index it at run time
    if (threadIdx.x == 0) fft_init_plan(spl, Q);
    __syncthreads();
    const FftPlan &pl = spl;
    const cx<R> *Xn = X + (size_t)n * K * Q;
    const cx<R> *ph = phase ? phase + (size_t)t * K * Q : nullptr;
    const int j0 = tid, j1 = tid + nthreads;
    const bool v0 = j0 < Q, v1 = j1 < Q;

    for (int h0 = 0; h0 < H; h0 += HP) {
        const int hc = min(HP, H - h0);
        cx<R> acc0[HP], acc1[HP];
#pragma unroll
        for (int h = 0; h < HP; ++h) acc0[h] = acc1[h] = cx<R>{(R)0, (R)0};
        for (int r = 0; r < K; ++r) {
            cx<R> z0 = {(R)0, (R)0}, z1 = {(R)0, (R)0};
            if (v0) {
                z0 = Xn[(size_t)r * Q + j0];
                if (ph) z0 = cmul(z0, ph[(size_t)r * Q + j0]);
            }
            if (v1) {
                z1 = Xn[(size_t)r * Q + j1];
                if (ph) z1 = cmul(z1, ph[(size_t)r * Q + j1]);
            }
            const R *ur = Ueta + (size_t)r * H + h0;
#pragma unroll
            for (int h = 0; h < HP; ++h) {
                if (h < hc) {
                    const R u = ur[h];
                    acc0[h].re += u * z0.re;
                    acc0[h].im += u * z0.im;
                    acc1[h].re += u * z1.re;
                    acc1[h].im += u * z1.im;
                }
            }
        }
        // phase 2: FFT rows in chunks of FC rows
        for (int f0 = 0; f0 < hc; f0 += FC) {
            const int fc = min(FC, hc - f0);
            __syncthreads();
#pragma unroll
            for (int h = 0; h < HP; ++h) {
                if (h >= f0 && h < f0 + fc) {
                    if (v0) ybuf[(h - f0) * Q + j0] = acc0[h];
                    if (v1) ybuf[(h - f0) * Q + j1] = acc1[h];
                }
            }
            __syncthreads();
            emit_rows<R>(ybuf, fc, h0 + f0, n, t, T, Q, H, Qc, pl, tw, G, F, f_kind, f_tile, f_ntiles, H8, nplanes,
                         is_img);
        }
    }
}

// Output of one block of rank rows h0 .. h0 + nr - 1 of a ring (nr <= 16; h0 a
// multiple of 16), transformed in place in yb[0 .. nr).  Generic layout: one
// complex per (q, h).  Fast layout (buffers zero-filled beforehand, so rows at
// or beyond H are not written): a bf16 fragment slot gathers 8 (4 for a half
// chunk) rank values, splits them into the plane format and writes 16 (8)
// bytes per plane and row; an FP32 slot half holds depth k = 8 hc + 4 j + g,
// j = 0, 1, of one re or im half-chunk hc (8 bytes).
// Row layout of the FP32 ring kernel's transform buffer: two padding values
// after every 32, so that the FFT's strided radix passes and the emission's
// reads of digit-reversed positions spread over the LDS banks (pairs j, j + 1
// with j even stay adjacent and 16-byte aligned), and a row stride of 2 more
// than a multiple of 32, so that rank rows a few apart fall on other banks.
__host__ __device__ __forceinline__ int ring_pad(int i) { return i + 2 * (i >> 5); }
__host__ __device__ __forceinline__ int ring_row_stride(int Q) {
    const int base = ring_pad(Q - 1) + 1;
    return base + ((2 - base % 32) + 32) % 32;
}

// one radix-RAD decimation-in-frequency butterfly of the padded row
template <int RAD>
__device__ __forceinline__ void fft_butterfly_pad(cx<float> *row, int base, int span, int k, int tstep,
                                                  const cx<float> *tw) {
    cx<float> v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = row[ring_pad(base + r * span)];
    dft_small(RAD, v);
    row[ring_pad(base)] = v[0];
#pragma unroll
    for (int p = 1; p < RAD; ++p) row[ring_pad(base + p * span)] = cmul(v[p], tw[k * p * tstep]);   // k p tstep < n
}

// lds_fft_dif on rows in the padded layout (row stride rs): the same passes,
// the same output order fft_pos
__device__ void lds_fft_dif_pad(cx<float> *buf, int cnt, int rs, const FftPlan &pl, const cx<float> *tw) {
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
            cx<float> *row = buf + (size_t)sq * rs;
            const int base = blk * L + k;
            if (rad == 8) fft_butterfly_pad<8>(row, base, span, k, tstep, tw);
            else if (rad == 4) fft_butterfly_pad<4>(row, base, span, k, tstep, tw);
            else if (rad == 2) fft_butterfly_pad<2>(row, base, span, k, tstep, tw);
            else fft_butterfly_pad<3>(row, base, span, k, tstep, tw);
        }
        __syncthreads();
        L = span;
    }
}

__device__ void emit_block(const cx<float> *yb, int rs, int h0, int nr, const int *pos_tab, int n, int t, int T,
                           int Q, int H, int Qc, float scale, cx<float> *__restrict__ G, void *__restrict__ F,
                           int f_kind, int f_tile, int f_ntiles, int H8, int nplanes, int is_img) {
    typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
    typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
    const int tid = threadIdx.x, nt = blockDim.x;
    if (G) {
        cx<float> *Gn = G + ((size_t)n * T + t) * H * Qc;   // [H][Qc]: q fastest
        for (int i = tid; i < Qc * nr; i += nt) {
            const int hh = i / Qc, q = i - hh * Qc;
            const cx<float> v = yb[hh * rs + ring_pad(pos_tab[q])];
            Gn[(size_t)(h0 + hh) * Qc + q] = cx<float>{v.re * scale, v.im * scale};
        }
    }
    if (!F) return;
    const bool fbf = f_kind != kFragF32;
    const bool f32b = f_kind == kFragF32B;
    const int planeB = frag_plane_bytes(f_kind, H8);
    const size_t blockB = (size_t)nplanes * planeB;
    const int f_q = (Qc == Q) ? Q : Q / 2 + 1;
    const int tile = n / f_tile, n_in = n - tile * f_tile;
    const int row0 = is_img ? 2 * n_in : n_in;
    auto val = [&](int h, int pos, int c) -> float {   // c: 0 re, 1 im; zero past the block's rows
        const int hh = h - h0;
        if (hh < 0 || hh >= nr) return 0.f;
        const cx<float> v = yb[hh * rs + ring_pad(pos)];
        return (c ? v.im : v.re) * scale;
    };
    if (f_kind == kFragBF16D || f_kind == kFragF32P) {
        // paired slot order: lane group g of a full chunk holds h = 16 chunk + 4 g
        // + 0..3 (half chunk: 16 NF + 2 g + 0..1); fragment lane 16 g + row
        const int NF = H8 / 16;
        const int chunk = h0 / 16;
        const bool full = chunk < NF;
        const int nv = full ? 4 : 2;
        for (int i = tid; i < Qc * 4; i += nt) {
            const int q = i >> 2, g = i & 3;
            const int hb = full ? 16 * chunk + 4 * g : 16 * NF + 2 * g;
            const int pos = pos_tab[q];
            char *blk = reinterpret_cast<char *>(F) + (((size_t)t * f_ntiles + tile) * f_q + q) * blockB;
            if (f_kind == kFragF32P) {   // target column n_in: [br ..., bi ...]
                float re[4] = {0.f, 0.f, 0.f, 0.f}, im[4] = {0.f, 0.f, 0.f, 0.f};
                for (int e = 0; e < nv; ++e) {
                    re[e] = val(hb + e, pos, 0);
                    im[e] = val(hb + e, pos, 1);
                }
                const int ln = 16 * g + n_in;
                if (full) {
                    u32x4_t w0, w1;
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        w0[d] = __float_as_uint(re[d]);
                        w1[d] = __float_as_uint(im[d]);
                    }
                    *reinterpret_cast<u32x4_t *>(blk + chunk * 2048 + ln * 16) = w0;
                    *reinterpret_cast<u32x4_t *>(blk + chunk * 2048 + 1024 + ln * 16) = w1;
                } else {
                    const u32x4_t w0 = {__float_as_uint(re[0]), __float_as_uint(re[1]), __float_as_uint(im[0]),
                                        __float_as_uint(im[1])};
                    *reinterpret_cast<u32x4_t *>(blk + NF * 2048 + ln * 16) = w0;
                }
                continue;
            }
            // image n_in: row 2 n_in keeps its re values, row 2 n_in + 1 its im
            // values, each split into the three bf16 planes
            for (int part = 0; part < 2; ++part) {
                uint16_t pk[3][4] = {};
                for (int e = 0; e < nv; ++e) split3_bf16(val(hb + e, pos, part), pk[0][e], pk[1][e], pk[2][e]);
                const int ln = 16 * g + 2 * n_in + part;
#pragma unroll
                for (int pl_i = 0; pl_i < 3; ++pl_i) {
                    if (pl_i >= nplanes) break;
                    char *pb = blk + (size_t)pl_i * planeB;
                    if (full) {
                        const u32x2_t wv = {(unsigned)pk[pl_i][0] | ((unsigned)pk[pl_i][1] << 16),
                                            (unsigned)pk[pl_i][2] | ((unsigned)pk[pl_i][3] << 16)};
                        *reinterpret_cast<u32x2_t *>(pb + chunk * 512 + ln * 8) = wv;
                    } else {
                        *reinterpret_cast<unsigned *>(pb + NF * 512 + ln * 4) =
                            (unsigned)pk[pl_i][0] | ((unsigned)pk[pl_i][1] << 16);
                    }
                }
            }
        }
        return;
    }
    if (fbf) {
        const int NF = H8 / 16;
        const int chunk = h0 / 16;
        const bool full = chunk < NF;
        const int nv = full ? 8 : 4;
        for (int i = tid; i < Qc * 4; i += nt) {
            const int q = i >> 2, g = i & 3, c = g >> 1, hsub = g & 1;
            const int hb = full ? 16 * chunk + 8 * hsub : 16 * NF + 4 * hsub;
            const int pos = pos_tab[q];
            char *blk = reinterpret_cast<char *>(F) + (((size_t)t * f_ntiles + tile) * f_q + q) * blockB;
            // Re row / target column: c = 0 -> re, 1 -> im; image Im row: c = 0 -> -im, 1 -> re
            for (int rr = 0; rr < (is_img ? 2 : 1); ++rr) {
                uint16_t pk[3][8];
                float xs[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    float x = 0.f;
                    if (e < nv) x = rr == 0 ? val(hb + e, pos, c) : (c ? val(hb + e, pos, 0) : -val(hb + e, pos, 1));
                    xs[e] = x;
                    if (!f32b) split3_bf16(x, pk[0][e], pk[1][e], pk[2][e]);
                }
                const int row = row0 + rr;
                if (f32b) {   // FP32 values in bf16 fragment order: 16-byte halves 1 KB apart
                    u32x4_t w0, w1;
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        w0[d] = __float_as_uint(xs[d]);
                        w1[d] = __float_as_uint(xs[4 + d]);
                    }
                    if (full) {
                        *reinterpret_cast<u32x4_t *>(blk + chunk * 2048 + (16 * g + row) * 16) = w0;
                        *reinterpret_cast<u32x4_t *>(blk + chunk * 2048 + 1024 + (16 * g + row) * 16) = w1;
                    } else {
                        *reinterpret_cast<u32x4_t *>(blk + NF * 2048 + (16 * g + row) * 16) = w0;
                    }
                    continue;
                }
#pragma unroll
                for (int pl_i = 0; pl_i < 3; ++pl_i) {
                    if (pl_i >= nplanes) break;
                    char *pb = blk + (size_t)pl_i * planeB;
                    if (full) {
                        u32x4_t wv;
#pragma unroll
                        for (int d = 0; d < 4; ++d) wv[d] = (unsigned)pk[pl_i][2 * d] | ((unsigned)pk[pl_i][2 * d + 1] << 16);
                        *reinterpret_cast<u32x4_t *>(pb + chunk * 1024 + (16 * g + row) * 16) = wv;
                    } else {
                        u32x2_t wv;
#pragma unroll
                        for (int d = 0; d < 2; ++d) wv[d] = (unsigned)pk[pl_i][2 * d] | ((unsigned)pk[pl_i][2 * d + 1] << 16);
                        *reinterpret_cast<u32x2_t *>(pb + NF * 1024 + (16 * g + row) * 8) = wv;
                    }
                }
            }
        }
    } else {
        // FP32 chunks of 16 depth values (re rows 0 .. H8 - 1, then im): slot g of
        // chunk k / 16 holds k = 16 chunk + 4 j + g, j = 0..3; half-chunk hc =
        // k / 8 is the slot's bytes 8 (hc & 1) .. + 8
        const int nh = H8 / 8;
        for (int i = tid; i < Qc * 16; i += nt) {
            const int q = i >> 4, sel = (i >> 2) & 3, g = i & 3;
            const int c = sel >> 1, hcr = h0 / 8 + (sel & 1);
            if (8 * hcr >= h0 + nr) continue;   // rows past H: left zero
            const int hc = c * nh + hcr;
            const int pos = pos_tab[q];
            char *blk = reinterpret_cast<char *>(F) + (((size_t)t * f_ntiles + tile) * f_q + q) * blockB;
            for (int rr = 0; rr < (is_img ? 2 : 1); ++rr) {
                u32x2_t wv;
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) {
                    const int h = 8 * hcr + 4 * jj + g;
                    const float x = rr == 0 ? val(h, pos, c) : (c ? val(h, pos, 0) : -val(h, pos, 1));
                    wv[jj] = __float_as_uint(x);
                }
                *reinterpret_cast<u32x2_t *>(blk + (hc >> 1) * 1024 + (16 * g + row0 + rr) * 16 + 8 * (hc & 1)) = wv;
            }
        }
    }
}

// FP32 principal rings on the matrix cores.  Per ring (item n, translation t)
// the recombination is the real GEMM
//   Y[h][(j, re|im)] = sum_r Ueta[r][h] (phi_t[r][j] X[n][r][j])_{re|im}
// with M = H (one or two 16-row blocks), N = 2 Q and depth K, on
// v_mfma_f32_16x16x4_f32.  Lane (r16 = l % 16, rg = l / 16) takes depth
// r = 4 ks + rg; one 16-byte load gives it angles j = 32 grp + 2 r16 and j + 1,
// whose re and im parts feed four column blocks, so no sample is loaded twice
// (weights Ueta come from global memory; lane r16 is rank row h).  Wave w
// takes the angle groups w, w + 4, ...  Y is then transformed and written in
// blocks of 16 rank rows, which keeps LDS small enough for two workgroups per
// CU; the rows are held in the padded layout of ring_pad.  Workgroups loop
// over rings; each XCD runs one contiguous range of rings, so the T
// translations of an item share its samples in one L2.
template <int NG, bool PHASE, bool TWO>
__global__ __launch_bounds__(256, 2) void k_rings_mfma(
    const cx<float> *__restrict__ X, int n_real, int T, const cx<float> *__restrict__ phase,
    const float *__restrict__ Ueta, int K, int Q, int H, int Qc, cx<float> *__restrict__ G,
    void *__restrict__ F, int f_kind, int f_tile, int f_ntiles, int H8, int nplanes, int is_img) {
    typedef float f32x4_t __attribute__((ext_vector_type(4)));
    extern __shared__ unsigned char smem_raw[];
    __shared__ FftPlan spl;           // in LDS: the stage loops index it at run time
    __shared__ int pos_tab[kMaxQ];    // FFT output position of each frequency
    cx<float> *tw = reinterpret_cast<cx<float> *>(smem_raw);   // [Q]
    cx<float> *ybuf = tw + Q;                                   // [16][RS], padded rows
    const int RS = ring_row_stride(Q);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    for (int i = tid; i < Q; i += blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)i / (double)Q, &s, &c);
        tw[i] = cx<float>{(float)c, (float)s};
    }
    if (tid == 0) fft_init_plan(spl, Q);
    __syncthreads();
    const FftPlan &pl = spl;
    for (int q = tid; q < Q; q += blockDim.x) pos_tab[q] = fft_pos(q, pl);   // read after the ring loop's barriers
    const float scale = (float)(1.0 / sqrt((double)Q));
    const int KS = (K + 3) >> 2;
    const int r16 = l & 15, rg = l >> 4;
    const int R = n_real * T, nwg = gridDim.x, wg = blockIdx.x;
    int first, last, step;
    if (nwg >= 8) {   // XCD x = wg % 8 owns rings [R x / 8, R (x + 1) / 8)
        const int x = wg & 7;
        first = (int)(((long long)R * x) >> 3) + (wg >> 3);
        last = (int)(((long long)R * (x + 1)) >> 3);
        step = (nwg - x + 7) >> 3;
    } else {
        first = wg;
        last = R;
        step = nwg;
    }
    for (int ring = first; ring < last; ring += step) {
        const int n = ring / T, t = ring - n * T;
        const cx<float> *Xn = X + (size_t)n * K * Q;
        const cx<float> *ph = PHASE ? phase + (size_t)t * K * Q : nullptr;
        f32x4_t acc0[NG][4], acc1[NG][4];
#pragma unroll
        for (int gi = 0; gi < NG; ++gi)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                acc0[gi][s4] = f32x4_t{0.f, 0.f, 0.f, 0.f};
                acc1[gi][s4] = f32x4_t{0.f, 0.f, 0.f, 0.f};
            }
        // depth step ks: 16 bytes per angle group (clamped in range: rows >= K
        // meet zero weights, angles >= Q are not written), one step ahead
        auto fetch = [&](int ks, f32x4_t (&xv)[NG], f32x4_t (&pv)[NG], float &u0, float &u1)
                         __attribute__((always_inline)) {
            const int r = 4 * ks + rg;
            const size_t rb = (size_t)min(r, K - 1) * Q;
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                const int j = min(32 * (w + 4 * gi) + 2 * r16, Q - 2);
                xv[gi] = *reinterpret_cast<const f32x4_t *>(Xn + rb + j);
                if constexpr (PHASE) pv[gi] = *reinterpret_cast<const f32x4_t *>(ph + rb + j);
            }
            u0 = (r < K && r16 < H) ? Ueta[(size_t)r * H + r16] : 0.f;
            u1 = (TWO && r < K && r16 + 16 < H) ? Ueta[(size_t)r * H + r16 + 16] : 0.f;
        };
        f32x4_t xc[NG], pc[NG];
        float uc0, uc1;
        fetch(0, xc, pc, uc0, uc1);
        for (int ks = 0; ks < KS; ++ks) {
            f32x4_t xn[NG], pn[NG];
            float un0, un1;
            fetch(min(ks + 1, KS - 1), xn, pn, un0, un1);
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                f32x4_t v = xc[gi];
                if constexpr (PHASE) {
                    const f32x4_t p = pc[gi];
                    v = f32x4_t{p[0] * xc[gi][0] - p[1] * xc[gi][1], p[0] * xc[gi][1] + p[1] * xc[gi][0],
                                p[2] * xc[gi][2] - p[3] * xc[gi][3], p[2] * xc[gi][3] + p[3] * xc[gi][2]};
                }
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    acc0[gi][s4] = __builtin_amdgcn_mfma_f32_16x16x4f32(uc0, v[s4], acc0[gi][s4], 0, 0, 0);
                    if constexpr (TWO)
                        acc1[gi][s4] = __builtin_amdgcn_mfma_f32_16x16x4f32(uc1, v[s4], acc1[gi][s4], 0, 0, 0);
                }
            }
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                xc[gi] = xn[gi];
                if constexpr (PHASE) pc[gi] = pn[gi];
            }
            uc0 = un0;
            uc1 = un1;
        }
        // output lane layout: rows 4 rg + v, column r16 of each column block;
        // column blocks (re j, im j, re j+1, im j+1) are two adjacent complex
        auto put = [&](f32x4_t (&acc)[NG][4], int nr) __attribute__((always_inline)) {
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                const int j = 32 * (w + 4 * gi) + 2 * r16;
                if (j < Q) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 4 * rg + v;
                        if (row < nr)
                            *reinterpret_cast<f32x4_t *>(ybuf + (size_t)row * RS + ring_pad(j)) =
                                f32x4_t{acc[gi][0][v], acc[gi][1][v], acc[gi][2][v], acc[gi][3][v]};
                    }
                }
            }
        };
#pragma unroll
        for (int bi = 0; bi < (TWO ? 2 : 1); ++bi) {
            const int h0 = 16 * bi, nr = min(16, H - h0);
            __syncthreads();   // earlier readers of ybuf are done
            if (bi == 0) put(acc0, nr);
            else put(acc1, nr);
            __syncthreads();
            lds_fft_dif_pad(ybuf, nr, RS, pl, tw);
            emit_block(ybuf, RS, h0, nr, pos_tab, n, t, T, Q, H, Qc, scale, G, F, f_kind, f_tile, f_ntiles, H8, nplanes,
                       is_img);
        }
    }
}

// zero fill of the fast operand buffers (a kernel rather than a memset, so
// that the prepare sequence stays capturable in a graph)
__global__ void k_zero16(u32x4_t *p, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = u32x4_t{0u, 0u, 0u, 0u};
}

// caller-supplied U [K][H]: copied into columns 0..H-1 of the plan's U,
// other columns zero, eigenvalues NaN (C is not formed).
__global__ void k_user_U(const double *U_in, int K, int H, double *U, double *lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K * K) {
        const int r = i / K, h = i - r * K;
        U[i] = h < H ? U_in[(size_t)r * H + h] : 0.0;
    }
    if (i < K) lam[i] = __builtin_nan("");
}

hipError_t launch_user_U(radsvd_plan *p, const double *U_in, hipStream_t s) {
    const int n = p->K * p->K;
    hipLaunchKernelGGL(k_user_U, dim3((n + 255) / 256), dim3(256), 0, s, U_in, p->K, p->H, p->U, p->lam);
    return hipGetLastError();
}

hipError_t launch_setup(radsvd_plan *p, const GridArgs &g, hipStream_t s) {
    const int total = p->T * p->K * p->Q;
    int blocks = (total + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    if (p->prec == RADSVD_FP64)
        hipLaunchKernelGGL(k_setup<double>, dim3(blocks), dim3(256), 0, s, g, p->d_k, p->d_eta,
                           p->d_delta, reinterpret_cast<cx<double> *>(p->phase));
    else
        hipLaunchKernelGGL(k_setup<float>, dim3(blocks), dim3(256), 0, s, g, p->d_k, p->d_eta,
                           p->d_delta, reinterpret_cast<cx<float> *>(p->phase));
    return hipGetLastError();
}

hipError_t launch_ueta(radsvd_plan *p, const double *U_src, int ld, hipStream_t s) {
    const int n = p->K * p->H;
    const int blocks = (n + 255) / 256;
    if (p->prec == RADSVD_FP64)
        hipLaunchKernelGGL(k_ueta<double>, dim3(blocks), dim3(256), 0, s, U_src, ld, p->d_eta, p->K,
                           p->H, reinterpret_cast<double *>(p->Ueta));
    else
        hipLaunchKernelGGL(k_ueta<float>, dim3(blocks), dim3(256), 0, s, U_src, ld, p->d_eta, p->K,
                           p->H, reinterpret_cast<float *>(p->Ueta));
    return hipGetLastError();
}

static hipError_t rings_side_mfma(radsvd_plan *p, const void *X, int n_real, int n_pad, int T, bool use_phase,
                                  void *G, void *F, int f_tile, int is_img, hipStream_t s) {
    const int Q = p->Q;
    const size_t shmem = (size_t)(Q + 16 * ring_row_stride(Q)) * sizeof(cx<float>);   // twiddles + 16 padded rows
    const int f_kind = is_img ? p->ffmt_a : p->ffmt_b;
    const int nplanes = is_img ? p->nplanes_a : p->nplanes_b;
    const int ng = ((Q + 31) / 32 + 3) / 4;                     // angle groups per wave
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int rings = n_real * T;
    const int grid = std::max(1, std::min(rings, 2 * cus));
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), shmem, s, reinterpret_cast<const cx<float> *>(X), n_real, T,
                           reinterpret_cast<const cx<float> *>(p->phase), reinterpret_cast<const float *>(p->Ueta),
                           p->K, Q, p->H, p->Qc, reinterpret_cast<cx<float> *>(G), F, f_kind, f_tile,
                           n_pad / f_tile, p->H8, nplanes, is_img);
        return hipGetLastError();
    };
    auto pick2 = [&](auto phase_tag, auto two_tag) -> hipError_t {
        constexpr bool PH = decltype(phase_tag)::value, TW = decltype(two_tag)::value;
        if (ng <= 1) return go(k_rings_mfma<1, PH, TW>);
        if (ng <= 2) return go(k_rings_mfma<2, PH, TW>);
        if (ng <= 3) return go(k_rings_mfma<3, PH, TW>);
        return go(k_rings_mfma<4, PH, TW>);
    };
    auto pick = [&](auto phase_tag) -> hipError_t {
        return p->H > 16 ? pick2(phase_tag, std::true_type{}) : pick2(phase_tag, std::false_type{});
    };
    return use_phase ? pick(std::true_type{}) : pick(std::false_type{});
}

template <typename R, int HP>
static hipError_t rings_side(radsvd_plan *p, const void *X, int n_real, int n_pad, int T,
                             bool use_phase, void *G, void *F, int f_tile, int is_img, hipStream_t s) {
    const int Q = p->Q, K = p->K, H = p->H;
    const size_t cxb = sizeof(cx<R>);
    int FC = (int)(32768 / ((size_t)Q * cxb));
    if (FC < 1) FC = 1;
    if (FC > HP) FC = HP;
    const size_t shmem = (size_t)Q * cxb + (size_t)FC * Q * cxb;
    const int f_kind = p->prec == RADSVD_FP64 ? kFragF32 : (is_img ? p->ffmt_a : p->ffmt_b);
    const int nplanes = is_img ? p->nplanes_a : p->nplanes_b;
    const int f_ntiles = n_pad / f_tile;
    const int items = n_real * T;   // padding items of the fast layout stay zero
    hipLaunchKernelGGL((k_rings<R, HP>), dim3(items), dim3(256), shmem, s,
                       reinterpret_cast<const cx<R> *>(X), n_real, T,
                       use_phase ? reinterpret_cast<const cx<R> *>(p->phase) : nullptr,
                       reinterpret_cast<const R *>(p->Ueta), K, Q, H, p->Qc, FC,
                       reinterpret_cast<cx<R> *>(G), F, f_kind, f_tile, f_ntiles, p->H8, nplanes, is_img);
    return hipGetLastError();
}

hipError_t launch_principal_rings(radsvd_plan *p, hipStream_t s) {
    hipError_t e;
    if (p->prec == RADSVD_FP64) {
        p->g_ready = 1;
        e = rings_side<double, 16>(p, p->A_polar, p->n_img, p->na_pad, 1, false, p->Ag, nullptr,
                                   kFastTA, 1, s);
        if (e != hipSuccess) return e;
        return rings_side<double, 16>(p, p->B_polar, p->n_tgt, p->nb_pad, p->T, true, p->Bg, nullptr,
                                      kFastTB, 0, s);
    }
    if (p->Af) {   // both fast buffers are contiguous multiples of 256 bytes
        // The ring kernel writes every byte of a real item's blocks (zeros for ranks
        // at or past H) except in the FP32 format, which leaves ranks past H alone;
        // padding items of the last tile are never written.  Fill only then.
        const bool zero_a = (p->n_img % kFastTA) != 0 || (p->ffmt_a == kFragF32 && p->H != p->H8);
        const bool zero_b = (p->n_tgt % kFastTB) != 0 || (p->ffmt_b == kFragF32 && p->H != p->H8);
        if (zero_a)
            hipLaunchKernelGGL(k_zero16, dim3(2048), dim3(256), 0, s, reinterpret_cast<u32x4_t *>(p->Af),
                               p->Af_bytes / 16);
        if (zero_b)
            hipLaunchKernelGGL(k_zero16, dim3(2048), dim3(256), 0, s, reinterpret_cast<u32x4_t *>(p->Bf),
                               p->Bf_bytes / 16);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // Plans the fused kernel serves for every output (BEST, LSE, FULL) get only
    // the fast layout here; their generic one is written when the backward pass
    // first needs it.
    const bool generic = !fast_path_supported(p, RADSVD_OUT_BEST | RADSVD_OUT_LSE | RADSVD_OUT_FULL);
    p->g_ready = generic ? 1 : 0;
    e = rings_side_mfma(p, p->A_polar, p->n_img, p->na_pad, 1, false, generic ? p->Ag : nullptr, p->Af, kFastTA,
                        1, s);
    if (e != hipSuccess) return e;
    return rings_side_mfma(p, p->B_polar, p->n_tgt, p->nb_pad, p->T, true, generic ? p->Bg : nullptr, p->Bf,
                           kFastTB, 0, s);
}

hipError_t ensure_generic_layout(const radsvd_plan *cp, hipStream_t s) {
    if (cp->g_ready) return hipSuccess;
    radsvd_plan *p = const_cast<radsvd_plan *>(cp);   // reads only; the workspace is the plan's
    hipError_t e = rings_side_mfma(p, p->A_polar, p->n_img, p->na_pad, 1, false, p->Ag, nullptr, kFastTA, 1, s);
    if (e == hipSuccess)
        e = rings_side_mfma(p, p->B_polar, p->n_tgt, p->nb_pad, p->T, true, p->Bg, nullptr, kFastTB, 0, s);
    if (e != hipSuccess) return e;
    // under stream capture the writes exist only in the graph: write again next time
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusNone) cp->g_ready = 1;
    return hipSuccess;
}

}  // namespace radsvd
