// Persistent multi-job launch of the fused Hermitian pair kernel.
//
// Many independent alignment jobs, each with its own angle count Q, rank H,
// translations and image/target counts, run in one launch per tile class
// (the four-wave tile body at two workgroups per CU and at one, and the
// eight-wave one at Q = 384 and 512 for split bf16 with six products): every
// job's tiles
// (8 images x 16 targets, all translations) make up its work items, one tile
// per item, or several consecutive ones for jobs whose tiles are cheap (so
// that the per-item queue and call overhead stays small).  Items are
// ordered by decreasing cost per item (the long ones start first) and, within
// a job, in the job's band order; the sequence is cut into chunks of kChunk
// consecutive items dealt round-robin to the 8 XCDs, one queue per XCD.  A
// fixed grid of workgroups (one per compute unit) takes items from its own
// XCD's queue with an atomic counter, so the workgroups resident on one XCD
// run neighbouring tiles that share operands in its L2; an XCD whose queue is
// empty takes items from the others.  Each item runs the tile body of its
// job's (Q, H8) specialisation.  The job table lives in the batch
// workspace; it is written by a kernel (job data passed by value), so the
// whole sequence needs no host memory at run time and can be captured in a
// HIP graph.
#pragma once
#include "pairs_fast.h"

namespace radsvd {
namespace fastk {

// angle counts and ranks of the batched kernel
constexpr int kBatchQ[5] = {128, 192, 256, 384, 512};
constexpr int kBatchH8[4] = {8, 16, 24, 32};

struct BatchJob {
    Args a;        // fast-path arguments of the job (BEST output)
    int qi, hi;    // indices into kBatchQ, kBatchH8
    int item0;     // first work item of the job
    int group;     // tiles per work item (cheap tiles are grouped)
};

constexpr int kChunk = 128;   // consecutive items per XCD chunk

// Three classes of items, each with its own persistent launch: class 0 runs the
// four-wave tile body at two workgroups per CU (Q = 128, 192, 256), class 1 at
// one, class 2 the eight-wave body of the plans wide_plan() selects (512
// threads).  A job's class follows the occupancy its plan runs at alone.  Jobs
// are ordered by class, so a class's items are the contiguous range
// [base, base + its item count).
constexpr int kBatchClasses = 3;
struct BatchHeader {
    int n_jobs;
    int total;                              // work items of all classes
    int base[kBatchClasses];                // first item of each class
    int count[kBatchClasses][8];            // items in each XCD's queue, per class
    unsigned int next[kBatchClasses][8];    // queue positions
};

constexpr int kTableChunk = 32;   // jobs per table-writer launch (kernel argument space)

struct TableChunk {
    int first, n, n_jobs, total;
    int base[kBatchClasses];
    int count[kBatchClasses][8];
    BatchJob jobs[kTableChunk];
};

// Job arguments are read through the constant address space: the table is
// not written during the launch, so the compiler may reload its fields where
// it would otherwise keep them in (and spill) registers.
typedef const __attribute__((address_space(4))) Args CArgs;
typedef const __attribute__((address_space(4))) BatchJob CJob;

// One (Q, H8) specialisation per function: each gets the register allocation
// of the single-job kernel, not the union of all of them.
// tiles lin0 .. lin0 + cnt - 1 of a job, in its band order
template <int Q, int KIND, int H8, int WPC>
__device__ __attribute__((noinline)) void tile_h(CArgs &a, int lin0, int cnt, unsigned char *sm) {
    const int nTA = __builtin_amdgcn_readfirstlane(a.nTA), nTB = __builtin_amdgcn_readfirstlane(a.nTB);
    const int band = __builtin_amdgcn_readfirstlane(a.band);
    for (int k = 0; k < cnt; ++k) {
        int ta, tb;
        band_tile(lin0 + k, nTA, nTB, band, ta, tb);
        if constexpr (KIND == 0) fast_tile<Q, 0, H8 / 8, 0, WPC>(a, ta, tb, sm);
        else fast_tile<Q, KIND, H8 / 16, (H8 % 16) ? 1 : 0, WPC>(a, ta, tb, sm);
    }
}

template <int Q, int KIND, int WPC>
__device__ __forceinline__ void tile_q(int hi, CArgs &a, int lin0, int cnt, unsigned char *sm) {
    switch (hi) {
    case 0: tile_h<Q, KIND, 8, WPC>(a, lin0, cnt, sm); break;
    case 1: tile_h<Q, KIND, 16, WPC>(a, lin0, cnt, sm); break;
    case 2: tile_h<Q, KIND, 24, WPC>(a, lin0, cnt, sm); break;
    default: tile_h<Q, KIND, 32, WPC>(a, lin0, cnt, sm); break;
    }
}

// Takes the items of class CLS from the XCD queues (its own first, then the
// others) and runs f(job, lin0, cnt) for each; every wave of the workgroup
// leaves together once all queues are empty.
template <int CLS, class F>
__device__ __forceinline__ void batch_loop(BatchHeader *hdr, CJob *jobs, unsigned char *smem_raw, F &&f) {
    // the item handoff uses the tile's staging memory; the barrier after the
    // read keeps it from being overwritten early
    int &s_item = *reinterpret_cast<int *>(smem_raw);
    const int x0 = blockIdx.x & 7;   // workgroups are dealt to the XCDs round-robin
    const int base = hdr->base[CLS], nj = hdr->n_jobs;
    for (int qn = 0; qn < 8; ++qn) {
      const int x = (x0 + qn) & 7;
      for (;;) {
        const int qcount = hdr->count[CLS][x];
        __syncthreads();   // s_item of the previous item has been read by every thread
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&hdr->next[CLS][x], 1u);
        __syncthreads();
        const int k = s_item;
        __syncthreads();
        if (k >= qcount) break;   // uniform across the workgroup: every wave leaves
        const int item = base + (x + 8 * (k / kChunk)) * kChunk + k % kChunk;
        int lo = 0, hi = nj - 1;    // last job with item0 <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const int g = jobs[lo].group;
        const int lin0 = (item - jobs[lo].item0) * g;
        const int cnt = min(g, jobs[lo].a.nTA * jobs[lo].a.nTB - lin0);
        f(jobs[lo], lin0, cnt);
      }
    }
}

// class 1: one workgroup per CU
template <int KIND>
__global__ __launch_bounds__(256, 1) void k_pairs_batched(BatchHeader *hdr, const BatchJob *__restrict__ jobs_g) {
    extern __shared__ unsigned char smem_raw[];
    batch_loop<1>(hdr, (CJob *)jobs_g, smem_raw, [&](CJob &J, int lin0, int cnt) {
        CArgs &a = J.a;
        const int qi = J.qi, hr = J.hi;
        switch (qi) {
        case 0: tile_q<128, KIND, 1>(hr, a, lin0, cnt, smem_raw); break;
        case 1: tile_q<192, KIND, 1>(hr, a, lin0, cnt, smem_raw); break;
        case 2: tile_q<256, KIND, 1>(hr, a, lin0, cnt, smem_raw); break;
        case 3: tile_q<384, KIND, 1>(hr, a, lin0, cnt, smem_raw); break;
        default: tile_q<512, KIND, 1>(hr, a, lin0, cnt, smem_raw); break;
        }
    });
}

// class 0: two workgroups per CU (the host puts only Q = 128, 192, 256 here)
template <int KIND>
__global__ __launch_bounds__(256, 2) void k_pairs_batched2(BatchHeader *hdr, const BatchJob *__restrict__ jobs_g) {
    extern __shared__ unsigned char smem_raw[];
    batch_loop<0>(hdr, (CJob *)jobs_g, smem_raw, [&](CJob &J, int lin0, int cnt) {
        CArgs &a = J.a;
        const int qi = J.qi, hr = J.hi;
        switch (qi) {
        case 0: tile_q<128, KIND, 2>(hr, a, lin0, cnt, smem_raw); break;
        case 1: tile_q<192, KIND, 2>(hr, a, lin0, cnt, smem_raw); break;
        case 2: tile_q<256, KIND, 2>(hr, a, lin0, cnt, smem_raw); break;
        default: break;
        }
    });
}

template <int KIND>
hipError_t launch_batched_kind(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s) {
    static size_t attr_bytes = 0;
    if (shmem > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)k_pairs_batched<KIND>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
        attr_bytes = shmem;
    }
    hipLaunchKernelGGL(k_pairs_batched<KIND>, dim3(grid), dim3(256), shmem, s, hdr, jobs);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_batched2_kind(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s) {
    static size_t attr_bytes = 0;
    if (shmem > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)k_pairs_batched2<KIND>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
        attr_bytes = shmem;
    }
    hipLaunchKernelGGL(k_pairs_batched2<KIND>, dim3(grid), dim3(256), shmem, s, hdr, jobs);
    return hipGetLastError();
}

// the eight-wave items (Q = 384, 512; split bf16 with 6 products): batched_wide.hip
hipError_t launch_batched_wide(BatchHeader *hdr, const BatchJob *jobs, int grid, hipStream_t s);
hipError_t launch_batched_fp32(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s);
hipError_t launch_batched_bf16(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s);
hipError_t launch_batched_bf16x3(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s);
hipError_t launch_batched_bf16x3_6(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem,
                                   hipStream_t s);
// class 0 (pairs_fast_occ_*.hip)
hipError_t launch_batched2_fp32(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s);
hipError_t launch_batched2_bf16(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s);
hipError_t launch_batched2_bf16x3(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s);
hipError_t launch_batched2_bf16x3_6(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem,
                                    hipStream_t s);

}  // namespace fastk
}  // namespace radsvd
