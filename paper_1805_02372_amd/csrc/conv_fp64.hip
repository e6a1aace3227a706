// FFT length classes for FP64 tiles: L = n1 * n2 = 2^logL, n2 = 2^max(logL-13, min(11, logL/2)),
// 4 columns per pass-1 workgroup (64 B stores), 8 per pass-3 workgroup (128 B loads),
// 16 points per thread.
#include "conv_kernels.hpp"

namespace pa {

#define PA_CLASS(LOGL, N1, N2) \
    {ClassCfg{64, LOGL, N1, N2, 4, 8, 16}, &ClassImpl<double, N1, N2, 4, 8, 16>::pass1, \
     &ClassImpl<double, N1, N2, 4, 8, 16>::pass2, &ClassImpl<double, N1, N2, 4, 8, 16>::pass3}

static const ClassKernels kClasses64[] = {
    PA_CLASS(12, 64, 64),
    PA_CLASS(13, 128, 64),
    PA_CLASS(14, 128, 128),
    PA_CLASS(15, 256, 128),
    PA_CLASS(16, 256, 256),
    PA_CLASS(17, 512, 256),
    PA_CLASS(18, 512, 512),
    PA_CLASS(19, 1024, 512),
    PA_CLASS(20, 1024, 1024),
    PA_CLASS(21, 2048, 1024),
    PA_CLASS(22, 2048, 2048),
    PA_CLASS(23, 4096, 2048),
    PA_CLASS(24, 8192, 2048),
};

const ClassKernels* class_kernels64(int logL) {
    for (const ClassKernels& k : kClasses64)
        if (k.cfg.logL == logL) return &k;
    return nullptr;
}

}  // namespace pa
