// The fused Hermitian pair kernel that also writes the whole landscape
// (RADSVD_OUT_FULL), default occupancy: FP32 operands.
#include "pairs_fast.h"

namespace radsvd {
namespace fastk {

hipError_t launch_fast_full_fp32(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    return launch_kind<0, true>(a, Q, nwg, H8, s);
}

}  // namespace fastk
}  // namespace radsvd
