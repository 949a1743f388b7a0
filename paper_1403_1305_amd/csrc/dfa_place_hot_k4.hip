// dfa_place_hot_k4.hip -- the LDS_HOT DFA scan kernels for 4 walkers per lane.
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

DfaKernel select_hot_k4(const DeviceMachine &dm, uint32_t block_bytes) {
    return select_for<AC_PLACE_LDS_HOT, 4>(dm, 4, block_bytes);
}

}  // namespace dfa
}  // namespace acm
