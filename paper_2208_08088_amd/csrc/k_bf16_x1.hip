// Plain bfloat16-input kernels (one term, one product, binary32 output).
#include "k_bf16.h"

namespace tsmm {
static const Bf16Entry kX1[] = {
    TSMM_BE_KC(uint16_t, 1, 1, true) TSMM_BE_KC(uint16_t, 2, 1, true) TSMM_BE_KC(uint16_t, 1, 1, false)
    TSMM_BEI_KC(1, true) TSMM_BEI_KC(2, true) TSMM_BEI_KC(1, false)
};
Bf16Fn find_bf16_x1(int KC, int NT, int RT, bool vec, bool il) {
    for (const Bf16Entry &e : kX1)
        if (e.KC == KC && e.NT == NT && e.RT == RT && e.vec == (int)vec && e.il == (int)il) return e.fn;
    return nullptr;
}
}  // namespace tsmm
