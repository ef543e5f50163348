// Instantiations of the fused Hermitian pair kernel: BF16 operands, one product.
#include "pairs_fast.h"

namespace radsvd {
namespace fastk {

hipError_t launch_fast_bf16(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    return launch_kind<1>(a, Q, nwg, H8, s);
}

}  // namespace fastk
}  // namespace radsvd
