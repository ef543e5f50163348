// Instantiations of the fused Hermitian pair kernel: FP32 operands.
#include "pairs_fast.h"

namespace radsvd {
namespace fastk {

hipError_t launch_fast_fp32(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    return launch_kind<0>(a, Q, nwg, H8, s);
}

}  // namespace fastk
}  // namespace radsvd
