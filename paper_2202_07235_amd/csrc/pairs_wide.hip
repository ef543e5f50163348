// Instantiations of the eight-wave pair kernel (Q = 384, 512; split bf16, 6 products).
#include "pairs_wide.h"

namespace radsvd {
namespace fastk {

hipError_t launch_wide(const Args &a, int Q, int nwg, int H8, hipStream_t s) {
    switch (Q) {
    case 384: return launch_wide_h<384>(a, nwg, H8, s);
    case 512: return launch_wide_h<512>(a, nwg, H8, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace fastk
}  // namespace radsvd
