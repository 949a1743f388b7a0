// dfa_served_global.hip -- served kernels on the global table (own
// translation unit so the instantiations compile in parallel).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

ServedKernel select_served_global(bool hashed, int l2, uint32_t K, uint32_t block_bytes) {
    return select_served_for<AC_PLACE_GLOBAL>(hashed, l2, K, block_bytes);
}

}  // namespace dfa
}  // namespace acm
