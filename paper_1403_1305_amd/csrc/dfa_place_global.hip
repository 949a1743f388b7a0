// dfa_place_global.hip -- the DFA scan kernels for one table placement
// (a translation unit of its own so the instantiations compile in parallel).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

DfaKernel select_global(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes) {
    return select_for<AC_PLACE_GLOBAL>(dm, K, block_bytes);
}

}  // namespace dfa
}  // namespace acm
