// dfa_served_global.hip -- served kernels on the global table (own
// translation unit so the instantiations compile in parallel).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

ServedKernel select_served_global(bool hashed, int l2, uint32_t K, uint32_t block_bytes) {
    // the server launches one walker per lane
    return K == 1 ? select_served_for<AC_PLACE_GLOBAL, 1>(hashed, l2, 1, block_bytes) : nullptr;
}

}  // namespace dfa
}  // namespace acm
