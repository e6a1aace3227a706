// Length-class dispatch (the per-precision tables live in conv_fp32.hip,
// conv_fp64.hip and ntt.hip) and the device queries the launchers share.
#include <hip/hip_runtime.h>

#include <atomic>

#include "pa_internal.hpp"

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

const ClassKernels* class_kernels32(int logL);
const ClassKernels* class_kernels64(int logL);
const ClassKernels* class_kernels_ntt(int logL);

const ClassKernels* class_kernels(int prec, int logL) {
    if (prec == 32) return class_kernels32(logL);
    if (prec == 64) return class_kernels64(logL);
    if (prec == 1) return class_kernels_ntt(logL);
    return nullptr;
}

}  // namespace pa
