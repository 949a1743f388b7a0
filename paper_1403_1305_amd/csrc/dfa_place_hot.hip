// dfa_place_hot.hip -- the DFA scan kernels for one table placement
// (a translation unit of its own so the instantiations compile in parallel).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

DfaKernel select_hot(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes) {
    return select_for<AC_PLACE_LDS_HOT>(dm, K, block_bytes);
}

}  // namespace dfa
}  // namespace acm
