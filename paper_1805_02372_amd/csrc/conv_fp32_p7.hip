// Mixed-radix FFT length classes L = 7 * 2^k for FP32 tiles (section 3,
// step 1: the product is padded to an arbitrary length; with the classes
// 3, 5 and 7 times 2^k a tile is within 1.25x of any length instead of 2x).
// Rows n1 are a power of two: those of the class 2^k below 2^20
// (workgroup-wide Stockham row pass, 16 points per thread), else 8192 (the
// wave-level row pass of conv_v2.hpp).  Columns n2 = L / n1 carry the factor
// 7: workgroup-wide Stockham column passes with a radix-7 stage, 28 points
// per thread (conv_kernels.hpp).
#include "conv_kernels.hpp"
#include "conv_v2.hpp"

namespace pa {

#define PA_SMOOTH(K, N1, N2, RR, RC)                                                                   \
    {ClassCfg{32, smooth_id(7, K), N1, N2, 8, 16, RC}, &ClassImpl<float, N1, N2, 8, 16, RR, RC, true>::pass1, \
     &ClassImpl<float, N1, N2, 8, 16, RR, RC, true>::pass2, &ClassImpl<float, N1, N2, 8, 16, RR, RC, true>::pass3}
#define PA_SMOOTH_LONG(K, N2, RC)                                                                       \
    {ClassCfg{32, smooth_id(7, K), kN1, N2, 8, 16, RC}, &ClassImplS<float, N2, 8, 16, RC>::pass1,              \
     &ClassImplS<float, N2, 8, 16, RC>::pass2, &ClassImplS<float, N2, 8, 16, RC>::pass3}

static const ClassKernels kClasses[] = {
    PA_SMOOTH(12, 64, 448, 16, 28),  // L = 28,672
    PA_SMOOTH(13, 128, 448, 16, 28),  // L = 57,344
    PA_SMOOTH(14, 128, 896, 16, 28),  // L = 114,688
    PA_SMOOTH(15, 256, 896, 16, 28),  // L = 229,376
    PA_SMOOTH(16, 256, 1792, 16, 28),  // L = 458,752
    PA_SMOOTH(17, 512, 1792, 16, 28),  // L = 917,504
    PA_SMOOTH_LONG(18, 224, 28),  // L = 1,835,008
    PA_SMOOTH_LONG(19, 448, 28),  // L = 3,670,016
    PA_SMOOTH_LONG(20, 896, 28),  // L = 7,340,032
    PA_SMOOTH_LONG(21, 1792, 28),  // L = 14,680,064
};

const ClassKernels* class_kernels_fp32_p7(int cls) {
    for (const ClassKernels& k : kClasses)
        if (k.cfg.cls == cls) return &k;
    return nullptr;
}

}  // namespace pa
