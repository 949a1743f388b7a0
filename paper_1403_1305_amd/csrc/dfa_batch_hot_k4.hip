// dfa_batch_hot_k4.hip -- the LDS_HOT batch kernels for 4 walkers per lane.
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

BatchKernel select_batch_hot_k4(bool hashed, int l2, uint32_t block_bytes) {
    return select_batch_for<AC_PLACE_LDS_HOT, 4>(hashed, l2, 4, block_bytes);
}

}  // namespace dfa
}  // namespace acm
