// binary32 instantiations of the op N streaming kernel (16x16x4 f32).
#include "k_stream.h"

namespace tsmm {

static const StreamEntry kF32[] = {
    // scalar k-slot mapping (k not a multiple of 4, or k <= 8)
    TSMM_SE_RT1(float, 4, false) TSMM_SE_RT1(float, 8, false) TSMM_SE_RT1(float, 16, false)
    TSMM_SE_RT1(float, 32, false) TSMM_SE_RT1(float, 64, false) TSMM_SE_RT1(float, 128, false)
    TSMM_SE_RT1(float, 256, false)
    TSMM_SE_RT2(float, 4, false) TSMM_SE_RT4(float, 4, false)
    TSMM_SE_RT2(float, 8, false) TSMM_SE_RT4(float, 8, false)
    // vector mapping
    TSMM_SE_ALL(float, 16, true) TSMM_SE_RT8(float, 16, true) TSMM_SE_ALL(float, 32, true) TSMM_SE_ALL(float, 64, true)
    TSMM_SE_ALL(float, 128, true) TSMM_SE_RT1(float, 256, true) TSMM_SE_RT2(float, 256, true)
    // interleaved columns (n % 4 == 0): scalar mapping
    TSMM_SIS32_RT1(4) TSMM_SIS32_RT1(8) TSMM_SIS32_RT1(16) TSMM_SIS32_RT1(32) TSMM_SIS32_RT1(64)
    TSMM_SIS32_RT1(128) TSMM_SIS32_RT1(256) TSMM_SIS(float, 4, 4, 2) TSMM_SIS(float, 4, 8, 2)
    TSMM_SIS(float, 4, 4, 4) TSMM_SIS(float, 8, 4, 2) TSMM_SIS(float, 8, 8, 2) TSMM_SIS(float, 8, 4, 4)
    // vector mapping with interleaved columns (n % 4 == 0)
    TSMM_SEI32_ALL(16) TSMM_SEI32_ALL(32) TSMM_SEI32_ALL(64) TSMM_SEI32_ALL(128) TSMM_SEI32_RT1(256)
    TSMM_SEI32_RT2(256)
};

StreamFn find_stream_f32(int KC, int NT, int RT, bool vec, int cm) {
    for (const StreamEntry &e : kF32)
        if (e.KC == KC && e.NT == NT && e.RT == RT && e.vec == (int)vec && e.cm == cm) return e.fn;
    return nullptr;
}

}  // namespace tsmm
