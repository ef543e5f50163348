// Persistent multi-job kernel, BF16 contraction.
#include "batched.h"

namespace radsvd {
namespace fastk {

hipError_t launch_batched_bf16(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s) {
    return launch_batched_kind<1>(hdr, jobs, grid, shmem, s);
}

}  // namespace fastk
}  // namespace radsvd
