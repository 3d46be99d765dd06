// Split-bf16 kernels, three terms / six products (binary32 inputs).
#include "k_bf16.h"

namespace tsmm {
static const Bf16Entry kX6[] = {
    TSMM_BE_KC(float, 1, 6, true) TSMM_BE_KC(float, 2, 6, true) TSMM_BE_KC(float, 1, 6, false)
    TSMM_BEF_KC(1, 6, true) TSMM_BEF_KC(2, 6, true) TSMM_BEF_KC(1, 6, false)
};
Bf16Fn find_bf16_x6(int KC, int NT, int RT, bool vec, bool il) {
    for (const Bf16Entry &e : kX6)
        if (e.KC == KC && e.NT == NT && e.RT == RT && e.vec == (int)vec && e.il == (int)il) return e.fn;
    return nullptr;
}
}  // namespace tsmm
