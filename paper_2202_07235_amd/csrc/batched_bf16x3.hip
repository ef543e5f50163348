// Persistent multi-job kernel, split-BF16 contraction with 3 products.
#include "batched.h"

namespace radsvd {
namespace fastk {

hipError_t launch_batched_bf16x3(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s) {
    return launch_batched_kind<2>(hdr, jobs, grid, shmem, s);
}

}  // namespace fastk
}  // namespace radsvd
