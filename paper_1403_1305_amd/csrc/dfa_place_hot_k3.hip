// dfa_place_hot_k3.hip -- the LDS_HOT DFA scan kernels for 3 walkers per lane.
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

DfaKernel select_hot_k3(const DeviceMachine &dm, uint32_t block_bytes) {
    return select_for<AC_PLACE_LDS_HOT, 3>(dm, 3, block_bytes);
}

}  // namespace dfa
}  // namespace acm
