// dfa_served_hot.hip -- served kernels with the 16-bit LDS image (own
// translation unit so the instantiations compile in parallel).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

ServedKernel select_served_hot(bool hashed, int l2, uint32_t K, uint32_t block_bytes) {
    return select_served_for<AC_PLACE_LDS_HOT>(hashed, l2, K, block_bytes);
}

}  // namespace dfa
}  // namespace acm
