// Fast Hermitian pair kernel (matrix cores).  Placeholder until the MFMA
// path lands: no plan is routed here.
#include "common.h"
#include "internal.h"

namespace radsvd {

bool fast_path_supported(const radsvd_plan *, int) { return false; }
bool fast_tile_ok(int tile_b) { return tile_b == 0; }
hipError_t launch_pairs_fast(const radsvd_plan *, int, float, float *, int32_t *, int32_t *, float *,
                             hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace radsvd
