// Mixed-radix FFT length classes L = 5 * 2^k for FP64 tiles (section 3,
// step 1: the product is padded to an arbitrary length; with the classes
// 3, 5 and 7 times 2^k a tile is within 1.25x of any length instead of 2x).
// Rows n1 are a power of two: those of the class 2^k below 2^20
// (workgroup-wide Stockham row pass, 16 points per thread), else 8192 (the
// wave-level row pass of conv_v2.hpp).  Columns n2 = L / n1 carry the factor
// 5: workgroup-wide Stockham column passes with a radix-5 stage, 20 points
// per thread (conv_kernels.hpp).
#include "conv_kernels.hpp"
#include "conv_v2.hpp"

namespace pa {

#define PA_SMOOTH(K, N1, N2, RR, RC)                                                                   \
    {ClassCfg{64, smooth_id(5, K), N1, N2, 4, 8, RC}, &ClassImpl<double, N1, N2, 4, 8, RR, RC, true>::pass1, \
     &ClassImpl<double, N1, N2, 4, 8, RR, RC, true>::pass2, &ClassImpl<double, N1, N2, 4, 8, RR, RC, true>::pass3}
#define PA_SMOOTH_LONG(K, N2, RC)                                                                       \
    {ClassCfg{64, smooth_id(5, K), kN1, N2, 4, 8, RC}, &ClassImplS<double, N2, 4, 8, RC>::pass1,              \
     &ClassImplS<double, N2, 4, 8, RC>::pass2, &ClassImplS<double, N2, 4, 8, RC>::pass3}

static const ClassKernels kClasses[] = {
    PA_SMOOTH(12, 64, 320, 16, 20),  // L = 20,480
    PA_SMOOTH(13, 128, 320, 16, 20),  // L = 40,960
    PA_SMOOTH(14, 128, 640, 16, 20),  // L = 81,920
    PA_SMOOTH(15, 256, 640, 16, 20),  // L = 163,840
    PA_SMOOTH(16, 256, 1280, 16, 20),  // L = 327,680
    PA_SMOOTH(17, 512, 1280, 16, 20),  // L = 655,360
    PA_SMOOTH_LONG(18, 160, 20),  // L = 1,310,720
    PA_SMOOTH_LONG(19, 320, 20),  // L = 2,621,440
    PA_SMOOTH_LONG(20, 640, 20),  // L = 5,242,880
    PA_SMOOTH_LONG(21, 1280, 20),  // L = 10,485,760
};

const ClassKernels* class_kernels_fp64_p5(int cls) {
    for (const ClassKernels& k : kClasses)
        if (k.cfg.cls == cls) return &k;
    return nullptr;
}

}  // namespace pa
