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
    // interleaved columns (n even): scalar mapping
    TSMM_SIS64_RT1(4) TSMM_SIS64_RT1(8) TSMM_SIS64_RT1(16) TSMM_SIS64_RT1(32) TSMM_SIS64_RT1(64)
    TSMM_SIS64_RT1(128) TSMM_SIS64_RT1(256) TSMM_SIS(double, 4, 2, 2) TSMM_SIS(double, 4, 4, 2)
    TSMM_SIS(double, 4, 2, 4)
    // vector mapping with interleaved columns (n even)
    TSMM_SEI64_ALL(8) TSMM_SEI64_ALL(16) TSMM_SI(double, 8, 2, 8) TSMM_SI(double, 16, 2, 8) TSMM_SEI64_ALL(32)
    TSMM_SEI64_ALL(64) TSMM_SEI64_RT1(128) TSMM_SEI64_RT2(128) TSMM_SEI64_RT1(256) TSMM_SEI64_RT2(256)
    // one column tile, n even: lane pairs (16-byte C vectors)
    TSMM_SP(4, 1, false) TSMM_SP(8, 1, false) TSMM_SP(16, 1, false) TSMM_SP(32, 1, false) TSMM_SP(64, 1, false)
    TSMM_SP(128, 1, false) TSMM_SP(256, 1, false) TSMM_SP(4, 2, false) TSMM_SP(4, 4, false)
    TSMM_SP(8, 1, true) TSMM_SP(8, 2, true) TSMM_SP(8, 4, true) TSMM_SP(8, 8, true)
    TSMM_SP(16, 1, true) TSMM_SP(16, 2, true) TSMM_SP(16, 4, true) TSMM_SP(16, 8, true)
    TSMM_SP(32, 1, true) TSMM_SP(32, 2, true) TSMM_SP(32, 4, true) TSMM_SP(64, 1, true) TSMM_SP(64, 2, true)
    TSMM_SP(64, 4, true) TSMM_SP(128, 1, true) TSMM_SP(128, 2, true) TSMM_SP(256, 1, true) TSMM_SP(256, 2, true)
    // default-policy C stores for beta == 0 (vector mapping, k classes up to 64)
    TSMM_SPD(8, 1) TSMM_SPD(8, 2) TSMM_SPD(8, 4) TSMM_SPD(8, 8) TSMM_SPD(16, 1) TSMM_SPD(16, 2) TSMM_SPD(16, 4)
    TSMM_SPD(16, 8) TSMM_SPD(32, 1) TSMM_SPD(32, 2) TSMM_SPD(32, 4) TSMM_SPD(64, 1) TSMM_SPD(64, 2) TSMM_SPD(64, 4)
    TSMM_SID(8, 2, 1) TSMM_SID(8, 4, 1) TSMM_SID(8, 8, 1) TSMM_SID(8, 16, 1) TSMM_SID(8, 2, 2) TSMM_SID(8, 4, 2)
    TSMM_SID(8, 8, 2) TSMM_SID(8, 2, 4) TSMM_SID(8, 4, 4) TSMM_SID(8, 2, 8)
    TSMM_SID(16, 2, 1) TSMM_SID(16, 4, 1) TSMM_SID(16, 8, 1) TSMM_SID(16, 16, 1) TSMM_SID(16, 2, 2)
    TSMM_SID(16, 4, 2) TSMM_SID(16, 8, 2) TSMM_SID(16, 2, 4) TSMM_SID(16, 4, 4) TSMM_SID(16, 2, 8)
    TSMM_SID(32, 2, 1) TSMM_SID(32, 4, 1) TSMM_SID(32, 8, 1) TSMM_SID(32, 16, 1) TSMM_SID(32, 2, 2)
    TSMM_SID(32, 4, 2) TSMM_SID(32, 8, 2) TSMM_SID(32, 2, 4) TSMM_SID(32, 4, 4)
    TSMM_SID(64, 2, 1) TSMM_SID(64, 4, 1) TSMM_SID(64, 8, 1) TSMM_SID(64, 16, 1) TSMM_SID(64, 2, 2)
    TSMM_SID(64, 4, 2) TSMM_SID(64, 8, 2) TSMM_SID(64, 2, 4) TSMM_SID(64, 4, 4)
};

StreamFn find_stream_f64(int KC, int NT, int RT, bool vec, int cm) {
    for (const StreamEntry &e : kF64)
        if (e.KC == KC && e.NT == NT && e.RT == RT && e.vec == (int)vec && e.cm == cm) return e.fn;
    return nullptr;
}

}  // namespace tsmm
