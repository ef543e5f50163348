// Instantiations of the fused Hermitian pair kernel: split BF16 operands, 6 products.
#include "pairs_fast.h"

namespace radsvd {
namespace fastk {

hipError_t launch_fast_bf16x3_6(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    return launch_kind<3>(a, Q, nwg, H8, s);
}

}  // namespace fastk
}  // namespace radsvd
