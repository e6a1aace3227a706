// FFT length classes for FP32 tiles.  2^12 .. 2^13: one kernel per tile, the
// whole length in one workgroup (tile_fused.hpp).  2^14 .. 2^19: L = n1 * n2
// with n2 = 2^max(logL-13, min(10, logL/2)), workgroup-wide Stockham stages
// (conv_kernels.hpp).  2^20 .. 2^24: n1 = 8192, n2 = L / 8192, wave-level
// transforms (conv_v2.hpp).
#include "conv_kernels.hpp"
#include "conv_v2.hpp"
#include "tile_fused.hpp"

namespace pa {

#define PA_CLASS(LOGL, N1, N2) \
    {ClassCfg{32, LOGL, N1, N2, 8, 16, 16}, &ClassImpl<float, N1, N2, 8, 16, 16, 16>::pass1, \
     &ClassImpl<float, N1, N2, 8, 16, 16, 16>::pass2, &ClassImpl<float, N1, N2, 8, 16, 16, 16>::pass3}
#define PA_CLASS2(LOGL, N2) \
    {ClassCfg{32, LOGL, kN1, N2, ClassImpl2<float, N2>::C1, ClassImpl2<float, N2>::C3, 16,        \
              ClassImpl2<float, N2>::kWsExtra},                                                      \
     &ClassImpl2<float, N2>::pass1, &ClassImpl2<float, N2>::pass2, &ClassImpl2<float, N2>::pass3}
#define PA_FUSED(LOGL) \
    {ClassCfg{32, LOGL, 1 << LOGL, 1, 1 << LOGL, 1 << LOGL, 16}, &ClassImplF<float, 1 << LOGL>::pass1, \
     &ClassImplF<float, 1 << LOGL>::pass2, &ClassImplF<float, 1 << LOGL>::pass3}

static const ClassKernels kClasses32[] = {
    PA_FUSED(12),
    PA_FUSED(13),
    PA_CLASS(14, 128, 128),
    PA_CLASS(15, 256, 128),
    PA_CLASS(16, 256, 256),
    PA_CLASS(17, 512, 256),
    PA_CLASS(18, 512, 512),
    PA_CLASS(19, 1024, 512),
    PA_CLASS2(20, 128),
    PA_CLASS2(21, 256),
    PA_CLASS2(22, 512),
    PA_CLASS2(23, 1024),
    PA_CLASS2(24, 2048),
};

const ClassKernels* class_kernels32(int cls) {
    for (const ClassKernels& k : kClasses32)
        if (k.cfg.cls == cls) return &k;
    return nullptr;
}

}  // namespace pa
