// Persistent multi-job kernel, FP32 contraction.
#include "batched.h"

namespace radsvd {
namespace fastk {

hipError_t launch_batched_fp32(BatchHeader *hdr, const BatchJob *jobs, int grid, size_t shmem, hipStream_t s) {
    return launch_batched_kind<0>(hdr, jobs, grid, shmem, s);
}

}  // namespace fastk
}  // namespace radsvd
