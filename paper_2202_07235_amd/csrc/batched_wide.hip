// Persistent launch of the eight-wave items of a batch (class 2: Q = 384 and
// 512, split bf16 with six products), one tile body per (Q, H8).
#include "batched.h"
#include "pairs_wide.h"

namespace radsvd {
namespace fastk {

template <int Q, int H8>
__device__ __attribute__((noinline)) void wide_tile_h(CArgs &a, int lin0, int cnt, unsigned char *sm) {
    const int nTA = __builtin_amdgcn_readfirstlane(a.nTA), nTB = __builtin_amdgcn_readfirstlane(a.nTB);
    const int band = __builtin_amdgcn_readfirstlane(a.band);
    for (int k = 0; k < cnt; ++k) {
        int ta, tb;
        band_tile(lin0 + k, nTA, nTB, band, ta, tb);
        wide_tile<Q, H8 / 16, (H8 % 16) ? 1 : 0>(a, ta, tb, sm);
    }
}

template <int Q>
__device__ __forceinline__ void wide_tile_q(int hi, CArgs &a, int lin0, int cnt, unsigned char *sm) {
    switch (hi) {
    case 0: wide_tile_h<Q, 8>(a, lin0, cnt, sm); break;
    case 1: wide_tile_h<Q, 16>(a, lin0, cnt, sm); break;
    case 2: wide_tile_h<Q, 24>(a, lin0, cnt, sm); break;
    default: wide_tile_h<Q, 32>(a, lin0, cnt, sm); break;
    }
}

__global__ __launch_bounds__(512, 1) void k_pairs_batched_wide(BatchHeader *hdr, const BatchJob *__restrict__ jobs_g) {
    extern __shared__ unsigned char smem_raw[];
    int tables_q = 0;   // angle count whose twiddle table is in LDS
    batch_loop<2>(hdr, (CJob *)jobs_g, smem_raw, [&](CJob &J, int lin0, int cnt) {
        CArgs &a = J.a;
        const int hr = J.hi;
        if (J.qi == 3) {
            if (tables_q != 384) { wide_tables<384>(smem_raw); tables_q = 384; }
            wide_tile_q<384>(hr, a, lin0, cnt, smem_raw);
        } else {
            if (tables_q != 512) { wide_tables<512>(smem_raw); tables_q = 512; }
            wide_tile_q<512>(hr, a, lin0, cnt, smem_raw);
        }
    });
}

hipError_t launch_batched_wide(BatchHeader *hdr, const BatchJob *jobs, int grid, hipStream_t s) {
    constexpr size_t shmem = WideGeom<512>::BYTES;
    static_assert(WideGeom<384>::BYTES <= WideGeom<512>::BYTES, "LDS");
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute((const void *)k_pairs_batched_wide,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    hipLaunchKernelGGL(k_pairs_batched_wide, dim3(grid), dim3(512), shmem, s, hdr, jobs);
    return hipGetLastError();
}

}  // namespace fastk
}  // namespace radsvd
