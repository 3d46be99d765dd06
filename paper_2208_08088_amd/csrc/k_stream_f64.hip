// binary64 instantiations of the op N streaming kernel (16x16x4 f64).
#include "k_stream.h"

namespace tsmm {

static const StreamEntry kF64[] = {
    // scalar k-slot mapping (odd k): one row tile per wavefront
    TSMM_SE_RT1(double, 4, false) TSMM_SE_RT1(double, 8, false) TSMM_SE_RT1(double, 16, false)
    TSMM_SE_RT1(double, 32, false) TSMM_SE_RT1(double, 64, false) TSMM_SE_RT1(double, 128, false)
    TSMM_SE_RT1(double, 256, false)
    TSMM_SE_RT2(double, 4, false) TSMM_SE_RT4(double, 4, false)
    // vector mapping (even k)
    TSMM_SE_ALL(double, 8, true) TSMM_SE_ALL(double, 16, true) TSMM_SE_RT8(double, 8, true)
    TSMM_SE_RT8(double, 16, true) TSMM_SE_ALL(double, 32, true)
    TSMM_SE_ALL(double, 64, true) TSMM_SE_RT1(double, 128, true) TSMM_SE_RT2(double, 128, true)
    TSMM_SE_RT1(double, 256, true) TSMM_SE_RT2(double, 256, true)
};

StreamFn find_stream_f64(int KC, int NT, int RT, bool vec) {
    for (const StreamEntry &e : kF64)
        if (e.KC == KC && e.NT == NT && e.RT == RT && e.vec == (int)vec) return e.fn;
    return nullptr;
}

}  // namespace tsmm
