// dfa_place_hot_pair.hip -- the LDS_HOT scan kernels that look up two bytes at
// once from the states outside the image (four hashed columns only).
#include "dfa_kernel.h"

namespace acm {
namespace dfa {

DfaKernel select_hot_pair(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes) {
    if (!dm.hashed || dm.log2_cols != 2 || dm.pair_states == 0 || dm.hot_states == 0) return nullptr;
    constexpr int P = AC_PLACE_LDS_HOT;
    switch (K) {
        case 1:
            return block_bytes == 128 ? dfa_kernel<P, 1, 2, true, 1024, 1, 8, true>
                                      : dfa_kernel<P, 1, 2, true, 1024, 2, 4, true>;
        case 2:
            return block_bytes == 128 ? dfa_kernel<P, 2, 2, true, 1024, 1, 8, true>
                                      : dfa_kernel<P, 2, 2, true, 1024, 2, 4, true>;
        case 3: return dfa_kernel<P, 3, 2, true, 1024, 1, 4, true>;
        case 4: return dfa_kernel<P, 4, 2, true, 768, 1, 4, true>;
    }
    return nullptr;
}

}  // namespace dfa
}  // namespace acm
