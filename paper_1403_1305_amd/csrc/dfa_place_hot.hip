// dfa_place_hot.hip -- the LDS_HOT DFA scan kernels for one walker per lane,
// and the choice among walker counts (two to four walkers are instantiated in
// dfa_place_hot_k*.hip, so the translation units compile in parallel).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

DfaKernel select_hot(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes) {
    switch (K) {
        case 1: return select_for<AC_PLACE_LDS_HOT, 1>(dm, 1, block_bytes);
        case 2: return select_hot_k2(dm, block_bytes);
        case 3: return select_hot_k3(dm, block_bytes);
        case 4: return select_hot_k4(dm, block_bytes);
    }
    return nullptr;
}

}  // namespace dfa
}  // namespace acm
