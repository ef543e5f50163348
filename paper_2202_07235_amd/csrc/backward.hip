// Backward pass of the soft-alignment loss.  Not available yet: no plan has
// a backward workspace size.
#include "common.h"
#include "internal.h"

namespace radsvd {

size_t backward_bytes(const radsvd_plan *) { return 0; }
hipError_t launch_backward(const radsvd_plan *, float, const float *, const float *, void *, double *,
                           void *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace radsvd
