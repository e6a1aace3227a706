// Mixed-radix FFT length classes L = 3 * 2^k for FP32 tiles (section 3,
// step 1: the product is padded to an arbitrary length; with the classes
// 3, 5 and 7 times 2^k a tile is within 1.25x of any length instead of 2x).
// Rows n1 are a power of two: those of the class 2^k below 2^20
// (workgroup-wide Stockham row pass, 16 points per thread), else 8192 (the
// wave-level row pass of conv_v2.hpp).  Columns n2 = L / n1 carry the factor
// 3: workgroup-wide Stockham column passes with a radix-3 stage, 12 points
// per thread (conv_kernels.hpp).
#include "conv_kernels.hpp"
#include "conv_v2.hpp"

namespace pa {

#define PA_SMOOTH(K, N1, N2, RR, RC)                                                                   \
    {ClassCfg{32, smooth_id(3, K), N1, N2, 8, 16, RC}, &ClassImpl<float, N1, N2, 8, 16, RR, RC, true>::pass1, \
     &ClassImpl<float, N1, N2, 8, 16, RR, RC, true>::pass2, &ClassImpl<float, N1, N2, 8, 16, RR, RC, true>::pass3}
#define PA_SMOOTH_LONG(K, N2, RC)                                                                       \
    {ClassCfg{32, smooth_id(3, K), kN1, N2, 8, 16, RC}, &ClassImplS<float, N2, 8, 16, RC>::pass1,              \
     &ClassImplS<float, N2, 8, 16, RC>::pass2, &ClassImplS<float, N2, 8, 16, RC>::pass3}

static const ClassKernels kClasses[] = {
    PA_SMOOTH(13, 128, 192, 16, 12),  // L = 24,576
    PA_SMOOTH(14, 128, 384, 16, 12),  // L = 49,152
    PA_SMOOTH(15, 256, 384, 16, 12),  // L = 98,304
    PA_SMOOTH(16, 256, 768, 16, 12),  // L = 196,608
    PA_SMOOTH(17, 512, 768, 16, 12),  // L = 393,216
    PA_SMOOTH(18, 512, 1536, 16, 12),  // L = 786,432
    PA_SMOOTH_LONG(19, 192, 12),  // L = 1,572,864
    PA_SMOOTH_LONG(20, 384, 12),  // L = 3,145,728
    PA_SMOOTH_LONG(21, 768, 12),  // L = 6,291,456
    PA_SMOOTH_LONG(22, 1536, 12),  // L = 12,582,912
};

const ClassKernels* class_kernels_fp32_p3(int cls) {
    for (const ClassKernels& k : kClasses)
        if (k.cfg.cls == cls) return &k;
    return nullptr;
}

}  // namespace pa
