// dfa_batch_hot.hip -- batch kernels with the 16-bit LDS image (own
// translation unit so the instantiations compile in parallel).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

BatchKernel select_batch_hot(bool hashed, int l2, uint32_t K, uint32_t block_bytes) {
    // two to four walkers are instantiated in dfa_batch_hot_k*.hip
    switch (K) {
        case 1: return select_batch_for<AC_PLACE_LDS_HOT, 1>(hashed, l2, 1, block_bytes);
        case 2: return select_batch_hot_k2(hashed, l2, block_bytes);
        case 3: return select_batch_hot_k3(hashed, l2, block_bytes);
        case 4: return select_batch_hot_k4(hashed, l2, block_bytes);
    }
    return nullptr;
}

}  // namespace dfa
}  // namespace acm
