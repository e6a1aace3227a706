// Length-class dispatch (the per-precision tables live in conv_fp32.hip,
// conv_fp64.hip, conv_fp{32,64}_p{3,5,7}.hip and ntt.hip) and the device queries the launchers share.
#include <hip/hip_runtime.h>

#include <atomic>

#include "pa_internal.hpp"
#include "planner.hpp"

namespace pa {

// Compute units of the current device (sizes persistent grids).
int row_pass_workgroups() {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
    cached[dev].store(cu, std::memory_order_relaxed);
    return cu;
}

const ClassKernels* class_kernels32(int cls);
const ClassKernels* class_kernels64(int cls);
const ClassKernels* class_kernels_ntt(int cls);
const ClassKernels* class_kernels_fp32_p3(int cls);
const ClassKernels* class_kernels_fp32_p5(int cls);
const ClassKernels* class_kernels_fp32_p7(int cls);
const ClassKernels* class_kernels_fp64_p3(int cls);
const ClassKernels* class_kernels_fp64_p5(int cls);
const ClassKernels* class_kernels_fp64_p7(int cls);

static const ClassKernels* smooth_kernels(int prec, int cls) {
    if (!smooth_valid(cls)) return nullptr;
    const int P = smooth_P(cls);
    if (prec == 32) return P == 3 ? class_kernels_fp32_p3(cls) : P == 5 ? class_kernels_fp32_p5(cls) : class_kernels_fp32_p7(cls);
    if (prec == 64) return P == 3 ? class_kernels_fp64_p3(cls) : P == 5 ? class_kernels_fp64_p5(cls) : class_kernels_fp64_p7(cls);
    return nullptr;
}

static const ClassKernels* find_kernels(int prec, int cls) {
    const bool smooth = cls >= 32;
    if (prec == 32) return smooth ? smooth_kernels(32, cls) : class_kernels32(cls);
    if (prec == 64) return smooth ? smooth_kernels(64, cls) : class_kernels64(cls);
    if (prec == 1) return smooth ? nullptr : class_kernels_ntt(cls);
    return nullptr;
}

// Kernels of class `cls` (ids in pa_internal.hpp); the mixed-radix classes
// exist for FP32 and FP64 only.  A class whose compiled row and column
// lengths differ from the planner's geometry (from which its root tables are
// built) is refused rather than run with tables of another shape.
const ClassKernels* class_kernels(int prec, int cls) {
    const ClassKernels* k = find_kernels(prec, cls);
    if (!k) return nullptr;
    ClassGeom g;   // Prec values are the precision ids used here
    if (!class_geometry(prec, cls, &g) || g.n1 != k->cfg.n1 || g.n2 != k->cfg.n2) return nullptr;
    return k;
}

}  // namespace pa
