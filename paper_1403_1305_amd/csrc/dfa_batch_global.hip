// dfa_batch_global.hip -- batch kernels reading every table entry from
// global memory (own translation unit so the instantiations compile in
// parallel).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

BatchKernel select_batch_global(bool hashed, int l2, uint32_t K, uint32_t block_bytes) {
    return select_batch_for<AC_PLACE_GLOBAL>(hashed, l2, K, block_bytes);
}

}  // namespace dfa
}  // namespace acm
