// FP64 symmetric eigendecomposition of the kernel C (K <= 128) in one
// workgroup: parallel cyclic Jacobi with the round-robin ("circle") pair
// schedule, so that each round applies K/2 disjoint plane rotations at once.
// Paper section 3.3: the principal vectors are the eigenvectors of C, ordered
// by eigenvalue (the Rayleigh-quotient maximisers).  Output convention:
// eigenvalues descending; each eigenvector's entry of largest magnitude is
// positive (first such entry on ties).
//
// Phase 1 rotates C (in LDS) to diagonal form and records every round's
// rotations in a global log.  A round's K/2 rotations act on disjoint index
// pairs, so the two-sided update splits into independent 2x2 blocks (pair k
// rows x pair l columns) that one pass updates in place.  Phase 2 replays the
// log on V = I (in LDS): a row of V only ever mixes with itself, so each wave
// owns a set of rows and replays every round on them with no workgroup
// barrier, fetching the next round's rotations while it applies the current.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace radsvd {

struct Rot {
    int p, q;
    double c, s;
};

__device__ inline double block_sum_1024(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// up to two independent decompositions, one workgroup each
struct EigJobs {
    const double *C[2];
    int K[2];
    Rot *log[2];
    double *U[2];
    double *lam[2];
};

__global__ __launch_bounds__(1024) void k_jacobi(EigJobs jobs, int max_sweeps) {
    const int jb = blockIdx.x;
    const double *__restrict__ C = jobs.C[jb];
    const int K = jobs.K[jb];
    const int KP = (K + 1) & ~1;
    Rot *__restrict__ log = jobs.log[jb];
    double *__restrict__ U = jobs.U[jb];
    double *__restrict__ lam = jobs.lam[jb];
    extern __shared__ double sm[];   // phase 1: A [KP][KP+1]; phase 2: V [KP][KP+1]
    __shared__ int sp[kMaxK / 2], sq[kMaxK / 2];
    __shared__ double sc[kMaxK / 2], ss[kMaxK / 2];
    __shared__ double red[16];
    __shared__ double sdiag[kMaxK];
    __shared__ int srank[kMaxK];
    __shared__ int nrounds_s;
    __shared__ int any_rot;
    const int ld = KP + 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int npair = KP / 2;
    double *A = sm;
    for (int i = tid; i < KP * KP; i += nt) {
        const int r = i / KP, c = i - r * KP;
        A[r * ld + c] = (r < K && c < K) ? C[r * K + c] : 0.0;
    }
    __syncthreads();
    double part = 0.0;
    for (int i = tid; i < KP * KP; i += nt) {
        const int r = i / KP, c = i - r * KP;
        part += A[r * ld + c] * A[r * ld + c];
    }
    const double fro = block_sum_1024(part, red);
    // A non-finite entry (a NaN or infinite target sample reaches C through the
    // Gram sums) leaves no eigendecomposition to compute: every eigenvalue and
    // every entry of U is NaN, so each landscape built from U is NaN and every
    // pair takes the NaN rule of the pair step.
    if (!isfinite(fro)) {
        for (int i = tid; i < K * K; i += nt) U[i] = __builtin_nan("");
        for (int i = tid; i < K; i += nt) lam[i] = __builtin_nan("");
        return;
    }
    int nrounds = 0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        part = 0.0;
        for (int i = tid; i < KP * KP; i += nt) {
            const int r = i / KP, c = i - r * KP;
            if (r != c) part += A[r * ld + c] * A[r * ld + c];
        }
        const double off = block_sum_1024(part, red);
        // off-diagonal mass at the rounding floor: converged
        if (!(off > 1e-28 * fro)) break;
        if (tid == 0) any_rot = 0;
        for (int round = 0; round < KP - 1; ++round) {
            if (tid < npair) {
                int p, q;
                if (tid == 0) {
                    p = KP - 1;
                    q = round;
                } else {
                    p = (round + tid) % (KP - 1);
                    q = (round - tid + (KP - 1)) % (KP - 1);
                }
                const double apq = A[p * ld + q];
                const double app = A[p * ld + p], aqq = A[q * ld + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0 && fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
                    const double theta = (aqq - app) / (2.0 * apq);
                    double t;
                    if (fabs(theta) > 1e150) t = 0.5 / theta;
                    else t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    s = t * c;
                    any_rot = 1;
                }
                sp[tid] = p;
                sq[tid] = q;
                sc[tid] = c;
                ss[tid] = s;
                log[(size_t)nrounds * npair + tid] = Rot{p, q, c, s};
            }
            __syncthreads();
            // block (k, l): rows {p_k, q_k} x columns {p_l, q_l}; rows rotate by
            // (c_k, s_k), then columns by (c_l, s_l): x' = c x - s y, y' = s x + c y
            // thread t owns column pair l = t % 64 (nt is a multiple of 64) and row
            // pairs k = t / 64, t / 64 + nt / 64, ...; the column rotation is read once
            const int l = tid & 63;
            if (l < npair) {
                const double cl = sc[l], sl = ss[l];
                const int pl = sp[l], ql = sq[l];
                for (int k = tid >> 6; k < npair; k += nt >> 6) {
                    const double ck = sc[k], sk = ss[k];
                    if (sk == 0.0 && sl == 0.0) continue;
                    const int pk = sp[k], qk = sq[k];
                    const double a00 = A[pk * ld + pl], a01 = A[pk * ld + ql];
                    const double a10 = A[qk * ld + pl], a11 = A[qk * ld + ql];
                    const double r00 = ck * a00 - sk * a10, r10 = sk * a00 + ck * a10;
                    const double r01 = ck * a01 - sk * a11, r11 = sk * a01 + ck * a11;
                    A[pk * ld + pl] = cl * r00 - sl * r01;
                    A[pk * ld + ql] = sl * r00 + cl * r01;
                    A[qk * ld + pl] = cl * r10 - sl * r11;
                    A[qk * ld + ql] = sl * r10 + cl * r11;
                }
            }
            __syncthreads();
            ++nrounds;
        }
        if (!any_rot) break;   // every off-diagonal entry negligible against its diagonal pair
    }
    for (int i = tid; i < K; i += nt) sdiag[i] = A[i * ld + i];
    if (tid == 0) nrounds_s = nrounds;
    __threadfence_block();
    __syncthreads();
    nrounds = nrounds_s;
    // phase 2: V = product of the recorded rotations, applied to the identity;
    // wave wv owns rows wv, wv + nw, ..., lane k applies rotation k of a round
    double *V = sm;
    for (int i = tid; i < KP * KP; i += nt) {
        const int r = i / KP, c = i - r * KP;
        V[r * ld + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    {
        const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
        const bool act = lane < npair;
        Rot nx = {0, 0, 1.0, 0.0};
        if (act && nrounds > 0) nx = log[lane];
        for (int rd = 0; rd < nrounds; ++rd) {
            const Rot g = nx;
            if (act && rd + 1 < nrounds) nx = log[(size_t)(rd + 1) * npair + lane];
            if (act && g.s != 0.0) {
                for (int r = wv; r < KP; r += nw) {
                    const double a = V[r * ld + g.p], b = V[r * ld + g.q];
                    V[r * ld + g.p] = g.c * a - g.s * b;
                    V[r * ld + g.q] = g.s * a + g.c * b;
                }
            }
            // the next round's lanes read what other lanes of this wave wrote
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();
    // rank by descending eigenvalue (ties: lower index first); a total order
    // even for non-finite entries, which rank last, so every rank is taken once
    for (int i = tid; i < K; i += nt) {
        const double di = sdiag[i];
        const bool ni = isnan(di);
        int rank = 0;
        for (int j = 0; j < K; ++j) {
            const double dj = sdiag[j];
            const bool nj = isnan(dj);
            const bool before = (ni != nj) ? ni : (!ni && dj != di ? dj > di : j < i);
            if (j != i && before) ++rank;
        }
        srank[i] = rank;
        lam[rank] = di;
    }
    __syncthreads();
    // sign: largest-magnitude entry of each column positive; write U
    for (int src = tid; src < K; src += nt) {
        int piv = 0;
        double best = -1.0;
        for (int r = 0; r < K; ++r) {
            const double v = fabs(V[r * ld + src]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        const double sgn = V[piv * ld + src] < 0.0 ? -1.0 : 1.0;
        const int h = srank[src];
        for (int r = 0; r < K; ++r) U[r * K + h] = sgn * V[r * ld + src];
    }
}

size_t eig_log_bytes(int K) {
    const int KP = (K + 1) & ~1;
    return (size_t)kEigMaxSweeps * (KP - 1) * (KP / 2) * sizeof(Rot);
}

hipError_t launch_eig_raw2(int n, const double *const *C, const int *K, void *const *log, double *const *U,
                           double *const *lam, hipStream_t s) {
    EigJobs jobs{};
    int KPmax = 0;
    for (int i = 0; i < n; ++i) {
        jobs.C[i] = C[i];
        jobs.K[i] = K[i];
        jobs.log[i] = reinterpret_cast<Rot *>(log[i]);
        jobs.U[i] = U[i];
        jobs.lam[i] = lam[i];
        KPmax = std::max(KPmax, (K[i] + 1) & ~1);
    }
    const size_t shmem = (size_t)KPmax * (KPmax + 1) * sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void *)k_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_jacobi, dim3(n), dim3(1024), shmem, s, jobs, kEigMaxSweeps);
    return hipGetLastError();
}

hipError_t launch_eig_raw(const double *C, int K, void *log, double *U, double *lam, hipStream_t s) {
    return launch_eig_raw2(1, &C, &K, &log, &U, &lam, s);
}

hipError_t launch_eig(radsvd_plan *p, hipStream_t s) { return launch_eig_raw(p->C, p->K, p->eig_log, p->U, p->lam, s); }

}  // namespace radsvd
