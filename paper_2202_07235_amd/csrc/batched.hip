// Batched persistent launch over many alignment jobs.  Not available yet.
#include "common.h"
#include "internal.h"

namespace radsvd {

size_t batched_bytes(int n_jobs) { return 256 + (size_t)n_jobs * 256; }
hipError_t launch_pairs_batched(const radsvd_plan *const *, int, const radsvd_job_out *, void *,
                                hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace radsvd
