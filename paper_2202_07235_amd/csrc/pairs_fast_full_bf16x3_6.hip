// The fused Hermitian pair kernel that also writes the whole landscape
// (RADSVD_OUT_FULL), default occupancy: split BF16 operands, 6 products.
#include "pairs_fast.h"

namespace radsvd {
namespace fastk {

hipError_t launch_fast_full_bf16x3_6(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    return launch_kind<3, true>(a, Q, nwg, H8, s);
}

}  // namespace fastk
}  // namespace radsvd
