// dfa_batch_hot_k3.hip -- the LDS_HOT batch kernels for 3 walkers per lane.
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

BatchKernel select_batch_hot_k3(bool hashed, int l2, uint32_t block_bytes) {
    return select_batch_for<AC_PLACE_LDS_HOT, 3>(hashed, l2, 3, block_bytes);
}

}  // namespace dfa
}  // namespace acm
