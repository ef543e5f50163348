/*
 * FP64 direct sums for the radial-SVD alignment oracle.
 *
 * TEST INFRASTRUCTURE ONLY: this file is the slow, obviously correct CPU
 * definition that the HIP path is checked against.  It shares no code with
 * the HIP library and the library never calls it.
 *
 * Everything here is a plain nested loop over the quadrature nodes in
 * psi-space, with no FFT: the rotation by an on-grid angle gamma_m is an index
 * shift of each ring (paper, section 2.2, rotation definition), so the
 * inner product <A, R_gamma T_delta B> on the polar grid is a circular
 * cross-correlation along psi, summed over principal rings (section 3.3,
 * principal image rings; section 2.4, discrete inner products).
 *
 * Complex arrays are interleaved (re, im) doubles.
 */
#include <complex.h>
#include <stddef.h>

typedef double _Complex cplx;

/*
 * X[p][t][m] = sum_{h<H} sum_{j<Q} conj(Ar[ia[p]][h][j]) * Br[ib[p]][t][h][(j - m) mod Q]
 *
 * Ar: [n_img][H][Q]   principal image rings  sum_r U[r,h] eta_r Ahat(k_r, psi_j)
 * Br: [n_tgt][T][H][Q] principal target rings sum_r U[r,h] eta_r phi_t Bhat(k_r, psi_j)
 * X : [npairs][T][Q]
 */
void oracle_landscape_pairs(int npairs, const int *ia, const int *ib, int T, int H, int Q,
                            const double *Ar_, const double *Br_, double *X_)
{
    const cplx *Ar = (const cplx *)Ar_;
    const cplx *Br = (const cplx *)Br_;
    cplx *X = (cplx *)X_;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int p = 0; p < npairs; ++p) {
        for (int t = 0; t < T; ++t) {
            const cplx *a = Ar + (size_t)ia[p] * H * Q;
            const cplx *b = Br + ((size_t)ib[p] * T + t) * H * Q;
            for (int m = 0; m < Q; ++m) {
                cplx acc = 0.0;
                for (int h = 0; h < H; ++h) {
                    const cplx *ah = a + (size_t)h * Q;
                    const cplx *bh = b + (size_t)h * Q;
                    for (int j = 0; j < Q; ++j) {
                        int jm = j - m;
                        if (jm < 0) jm += Q;
                        acc += conj(ah[j]) * bh[jm];
                    }
                }
                X[((size_t)p * T + t) * Q + m] = acc;
            }
        }
    }
}

/*
 * Gradient of a real loss L(X) with respect to the principal target rings,
 * given P[a][b][t][m] = dL/d(Re X[a][b][t][m]) (real):
 *   gBr[b][t][h][i] = sum_a sum_m P[a][b][t][m] * Ar[a][h][(i + m) mod Q]
 * (complex gradient convention dL/dRe + i dL/dIm).
 */
void oracle_grad_tgt_rings(int n_img, int n_tgt, int T, int H, int Q, const double *P,
                           const double *Ar_, double *gBr_)
{
    const cplx *Ar = (const cplx *)Ar_;
    cplx *gBr = (cplx *)gBr_;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int b = 0; b < n_tgt; ++b) {
        for (int t = 0; t < T; ++t) {
            for (int h = 0; h < H; ++h) {
                for (int i = 0; i < Q; ++i) {
                    cplx acc = 0.0;
                    for (int a = 0; a < n_img; ++a) {
                        const double *pr = P + (((size_t)a * n_tgt + b) * T + t) * Q;
                        const cplx *ah = Ar + ((size_t)a * H + h) * Q;
                        for (int m = 0; m < Q; ++m) {
                            int im = i + m;
                            if (im >= Q) im -= Q;
                            acc += pr[m] * ah[im];
                        }
                    }
                    gBr[(((size_t)b * T + t) * H + h) * Q + i] = acc;
                }
            }
        }
    }
}

/*
 * Gradient with respect to the principal image rings:
 *   gAr[a][h][j] = sum_b sum_t sum_m P[a][b][t][m] * Br[b][t][h][(j - m) mod Q]
 */
void oracle_grad_img_rings(int n_img, int n_tgt, int T, int H, int Q, const double *P,
                           const double *Br_, double *gAr_)
{
    const cplx *Br = (const cplx *)Br_;
    cplx *gAr = (cplx *)gAr_;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int a = 0; a < n_img; ++a) {
        for (int h = 0; h < H; ++h) {
            for (int j = 0; j < Q; ++j) {
                cplx acc = 0.0;
                for (int b = 0; b < n_tgt; ++b) {
                    for (int t = 0; t < T; ++t) {
                        const double *pr = P + (((size_t)a * n_tgt + b) * T + t) * Q;
                        const cplx *bh = Br + (((size_t)b * T + t) * H + h) * Q;
                        for (int m = 0; m < Q; ++m) {
                            int jm = j - m;
                            if (jm < 0) jm += Q;
                            acc += pr[m] * bh[jm];
                        }
                    }
                }
                gAr[((size_t)a * H + h) * Q + j] = acc;
            }
        }
    }
}

int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
