// XOR merge of per-chunk partial hashes (paper Eq. 4-7: the final key is the
// mod-2 sum of the intermediate keys of all blocks and batches).  Job j with
// nchunks > 1 has nchunks stage rows of out_words words; out[w] = XOR over the
// rows.  The rows already hold zeros beyond m, so no masking is needed.
#include <atomic>

#include "pa_internal.hpp"
#include "conv_kernels.hpp"
#include "conv_v2.hpp"

namespace pa {

__global__ void __launch_bounds__(256) k_merge(JobTable jt) {
    const JobDesc jd = (jt.njobs == 0) ? jt.one : jt.many[blockIdx.y];
    if (jd.nchunks <= 1) return;
    const uint64_t words = jd.out_words;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
         w += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t acc = 0;
        for (uint32_t b = 0; b < jd.nchunks; ++b) acc ^= jd.stage[(uint64_t)b * words + w];
        jd.out[w] = acc;
    }
}

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

int launch_merge(const JobTable& jt, uint64_t max_words, void* stream) {
    if (max_words == 0) return 0;
    uint64_t blocks = (max_words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    dim3 grid((unsigned)blocks, jt.njobs == 0 ? 1u : jt.njobs);
    hipLaunchKernelGGL(k_merge, grid, dim3(256), 0, (hipStream_t)stream, jt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
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
