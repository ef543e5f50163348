// The fused Hermitian pair kernel at the occupancy other than its default
// (Q = 128, 192, 256), single-job and batched: split BF16 operands, 6 products.
#include "batched.h"

namespace radsvd {
namespace fastk {

hipError_t launch_fast_alt_bf16x3_6(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    return launch_kind_alt<3>(a, Q, nwg, H8, s);
}

hipError_t launch_batched2_bf16x3_6(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s) {
    return launch_batched2_kind<3>(hdr, jobs, grid, shmem, s);
}

}  // namespace fastk
}  // namespace radsvd
