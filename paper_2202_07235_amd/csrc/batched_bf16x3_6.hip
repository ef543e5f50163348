// Persistent multi-job kernel, split-BF16 contraction with 6 products.
#include "batched.h"

namespace radsvd {
namespace fastk {

hipError_t launch_batched_bf16x3_6(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s) {
    return launch_batched_kind<3>(hdr, jobs, grid, shmem, s);
}

}  // namespace fastk
}  // namespace radsvd
