// Direct (bit-sliced) evaluation of the Toeplitz hash over GF(2), with no
// transform and no floating point: y_i = parity(popcount(AND of the seed
// window at i with the reversed key)), the definition of section 2.1 (Eq. 1)
// read word-parallel.  With xr[t] = x[n-1-t] (the key reversed),
//
//     y_i = XOR_{t<n} ( s[i+t] AND xr[t] ),
//
// so output i needs the 32-bit seed words at bit offsets i + 32k, each a
// funnel shift (v_alignbit) of two aligned words, AND-ed with reversed-key
// word k and XOR-accumulated; the output bit is the parity of the
// accumulator.  Cost: ceil(n/32) word steps per output (two VALU operations
// each), against about 24 L bytes of HBM traffic per FFT tile: the direct
// path is the faster one for short outputs, and it evaluates any chosen
// outputs exactly (a verifier of the FFT path that shares nothing with it).
//
// Seed bits past n+m-1 (and reads past the seed's last word, which return 0)
// only ever meet reversed-key bits t >= n, which are zero.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "direct.hpp"

namespace pa {

constexpr int kDirectThreads = 256;
constexpr uint32_t kDirectChunk = 4096;   // reversed-key words per workgroup (multiple of 4)

// 32 key bits starting at bit p (p may be negative: bits below 0 are 0);
// p + 31 < n, so no bit at or beyond n is read.
__device__ __forceinline__ uint32_t key_bits32(const uint64_t* __restrict__ key, int64_t p) {
    if (p <= -32) return 0u;
    if (p < 0) {
        const uint32_t cnt = (uint32_t)(32 + p);   // 1..31 bits from position 0
        return (uint32_t)(key[0] & ((1ull << cnt) - 1ull)) << (uint32_t)(-p);
    }
    const uint64_t w = (uint64_t)p >> 6;
    const uint32_t s = (uint32_t)p & 63u;
    uint64_t v = key[w] >> s;
    if (s > 32) v |= key[w + 1] << (64 - s);
    return (uint32_t)v;
}

// Reversed key kr[w] (bit b = key bit n-1-32w-b, zero for t >= n), for
// w < kw4, and zeroed output words.
__global__ void __launch_bounds__(kDirectThreads)
k_direct_prep(const uint64_t* __restrict__ key, uint64_t n, uint32_t* __restrict__ kr, uint64_t kw4,
              uint64_t* __restrict__ zero, uint64_t nzero) {
    const uint64_t g = (uint64_t)blockIdx.x * kDirectThreads + threadIdx.x;
    if (g < kw4) {
        const int64_t p = (int64_t)n - 32 - 32 * (int64_t)g;
        kr[g] = __builtin_bitreverse32(key_bits32(key, p));
    }
    if (g < nzero) zero[g] = 0ull;
}

// Outputs [i_base + 256 bx, +256) over reversed-key words [k_base + kc by,
// +kc): each thread owns one output; the workgroup stages its seed words and
// key words in LDS and XORs the parity bits of its waves into out.
__global__ void __launch_bounds__(kDirectThreads)
k_direct(const uint32_t* __restrict__ seed32, uint64_t sw32, const uint32_t* __restrict__ kr, uint64_t kw4,
         uint64_t k_base, uint32_t kc, uint64_t i_base, uint64_t m, uint64_t* __restrict__ out) {
    __shared__ uint32_t S[kDirectChunk + 12];
    __shared__ __align__(16) uint32_t K[kDirectChunk];
    const int tid = threadIdx.x;
    const uint64_t i0 = i_base + (uint64_t)blockIdx.x * kDirectThreads;
    const uint64_t k0 = k_base + (uint64_t)blockIdx.y * kc;
    const uint32_t nk = (uint32_t)(kw4 - k0 < kc ? kw4 - k0 : kc);   // multiple of 4
    const uint64_t sbase = (i0 >> 5) + k0;
    for (uint32_t q = tid; q < nk + 9; q += kDirectThreads) {
        const uint64_t gq = sbase + q;
        S[q] = gq < sw32 ? seed32[gq] : 0u;
    }
    for (uint32_t q = tid; q < nk; q += kDirectThreads) K[q] = kr[k0 + q];
    __syncthreads();

    const int b = tid >> 5, sh = tid & 31;   // output i0 + tid: word offset b, shift sh
    uint32_t lo = S[b], acc = 0u;
    for (uint32_t kk = 0; kk < nk; kk += 4) {
        const uint32_t h0 = S[b + kk + 1], h1 = S[b + kk + 2], h2 = S[b + kk + 3], h3 = S[b + kk + 4];
        const uint4 kv = *reinterpret_cast<const uint4*>(&K[kk]);
        acc ^= __builtin_amdgcn_alignbit(h0, lo, sh) & kv.x;
        acc ^= __builtin_amdgcn_alignbit(h1, h0, sh) & kv.y;
        acc ^= __builtin_amdgcn_alignbit(h2, h1, sh) & kv.z;
        acc ^= __builtin_amdgcn_alignbit(h3, h2, sh) & kv.w;
        lo = h3;
    }
    const uint64_t i = i0 + (uint64_t)tid;
    const bool bit = i < m && (__popc(acc) & 1);
    const unsigned long long bal = __ballot(bit);
    if ((tid & 63) == 0 && bal) atomicXor((unsigned long long*)&out[(i0 >> 6) + (tid >> 6)], bal);
}

// Selected outputs idx[g] (g < count), bit g of res: each thread walks the
// seed from its own offset (global reads), the key words come from LDS.
__global__ void __launch_bounds__(kDirectThreads)
k_direct_select(const uint32_t* __restrict__ seed32, uint64_t sw32, const uint32_t* __restrict__ kr, uint64_t kw4,
                uint64_t k_base, uint32_t kc, const uint64_t* __restrict__ idx, uint32_t count,
                uint64_t* __restrict__ res) {
    __shared__ __align__(16) uint32_t K[kDirectChunk];
    const int tid = threadIdx.x;
    const uint64_t k0 = k_base + (uint64_t)blockIdx.y * kc;
    const uint32_t nk = (uint32_t)(kw4 - k0 < kc ? kw4 - k0 : kc);
    for (uint32_t q = tid; q < nk; q += kDirectThreads) K[q] = kr[k0 + q];
    __syncthreads();
    const uint32_t g = blockIdx.x * kDirectThreads + (uint32_t)tid;
    const bool valid = g < count;
    const uint64_t i = valid ? idx[g] : 0ull;
    const uint64_t w0 = (i >> 5) + k0;
    const uint32_t sh = (uint32_t)i & 31u;
    auto ld = [&](uint64_t q) -> uint32_t { return q < sw32 ? seed32[q] : 0u; };
    uint32_t lo = ld(w0), acc = 0u;
    for (uint32_t kk = 0; kk < nk; kk += 4) {
        const uint32_t h0 = ld(w0 + kk + 1), h1 = ld(w0 + kk + 2), h2 = ld(w0 + kk + 3), h3 = ld(w0 + kk + 4);
        const uint4 kv = *reinterpret_cast<const uint4*>(&K[kk]);
        acc ^= __builtin_amdgcn_alignbit(h0, lo, sh) & kv.x;
        acc ^= __builtin_amdgcn_alignbit(h1, h0, sh) & kv.y;
        acc ^= __builtin_amdgcn_alignbit(h2, h1, sh) & kv.z;
        acc ^= __builtin_amdgcn_alignbit(h3, h2, sh) & kv.w;
        lo = h3;
    }
    const bool bit = valid && (__popc(acc) & 1);
    const unsigned long long bal = __ballot(bit);
    const uint32_t g0 = blockIdx.x * kDirectThreads + (uint32_t)(tid & ~63);
    if ((tid & 63) == 0 && bal) atomicXor((unsigned long long*)&res[g0 >> 6], bal);
}

__global__ void __launch_bounds__(kDirectThreads)
k_xor_words(uint64_t* dst, const uint64_t* src, uint64_t words) {   // src may be dst (clears it)
    const uint64_t g = (uint64_t)blockIdx.x * kDirectThreads + threadIdx.x;
    if (g < words) dst[g] ^= src[g];
}

static uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

int launch_xor_words(uint64_t* dst, const uint64_t* src, uint64_t words, void* stream) {
    if (words == 0) return 0;
    hipLaunchKernelGGL(k_xor_words, dim3((uint32_t)cdiv(words, kDirectThreads)), dim3(kDirectThreads), 0,
                       (hipStream_t)stream, dst, src, words);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

uint64_t direct_key_words(uint64_t n) { return cdiv(cdiv(n, 32), 4) * 4; }

// Grid slabs: at most 2^20 workgroups along x and 2^15 along y per launch.
constexpr uint64_t kSlabX = 1ull << 20, kSlabY = 1ull << 15;

int launch_direct_prep(const uint64_t* key, uint64_t n, uint64_t m, uint64_t* out, uint32_t* kr, void* stream,
                       uint64_t* launches) {
    const uint64_t kw4 = direct_key_words(n), ow = cdiv(m, 64);
    const uint64_t prep = std::max(kw4, ow);
    hipLaunchKernelGGL(k_direct_prep, dim3((uint32_t)cdiv(prep, kDirectThreads)), dim3(kDirectThreads), 0,
                       (hipStream_t)stream, key, n, kr, kw4, out, ow);
    if (hipGetLastError() != hipSuccess) return -1;
    *launches += 1;
    return 0;
}

int launch_direct_main(const uint64_t* seed, uint64_t n, uint64_t m, uint64_t* out, const uint32_t* kr,
                       void* stream, uint64_t* launches) {
    hipStream_t s = (hipStream_t)stream;
    const uint64_t kw4 = direct_key_words(n), sw32 = 2 * cdiv(n + m - 1, 64);
    // about 1024 workgroups (4 per CU), each with at least 1024 key words:
    // split the key when the outputs are few (measured on MI355X against
    // 512..8192 workgroups and 256-word chunks)
    const uint64_t bx = cdiv(m, kDirectThreads);
    const uint64_t want_y = std::max<uint64_t>(1, cdiv(1024, bx));
    uint64_t kc = std::max<uint64_t>(1024, cdiv(kw4, want_y));
    kc = std::min<uint64_t>(cdiv(kc, 4) * 4, kDirectChunk);
    const uint64_t by = cdiv(kw4, kc);
    for (uint64_t x0 = 0; x0 < bx; x0 += kSlabX)
        for (uint64_t y0 = 0; y0 < by; y0 += kSlabY) {
            const dim3 grid((uint32_t)std::min(kSlabX, bx - x0), (uint32_t)std::min(kSlabY, by - y0));
            hipLaunchKernelGGL(k_direct, grid, dim3(kDirectThreads), 0, s, (const uint32_t*)seed, sw32, kr, kw4,
                               y0 * kc, (uint32_t)kc, x0 * kDirectThreads, m, out);
            if (hipGetLastError() != hipSuccess) return -1;
            *launches += 1;
        }
    return 0;
}

int launch_direct_select(const uint64_t* seed, const uint64_t* key, uint64_t n, uint64_t m, const uint64_t* idx,
                         uint32_t count, uint64_t* res, uint32_t* kr, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const uint64_t kw4 = direct_key_words(n), rw = cdiv(count, 64), sw32 = 2 * cdiv(n + m - 1, 64);
    const uint64_t prep = std::max(kw4, rw);
    hipLaunchKernelGGL(k_direct_prep, dim3((uint32_t)cdiv(prep, kDirectThreads)), dim3(kDirectThreads), 0, s, key, n,
                       kr, kw4, res, rw);
    if (hipGetLastError() != hipSuccess) return -1;
    const uint64_t bx = cdiv(count, kDirectThreads);   // count <= 2^20
    const uint64_t want_y = std::max<uint64_t>(1, cdiv(2048, bx));
    uint64_t kc = std::max<uint64_t>(256, cdiv(kw4, want_y));
    kc = std::min<uint64_t>(cdiv(kc, 4) * 4, kDirectChunk);
    const uint64_t by = cdiv(kw4, kc);
    for (uint64_t y0 = 0; y0 < by; y0 += kSlabY) {
        const dim3 grid((uint32_t)bx, (uint32_t)std::min(kSlabY, by - y0));
        hipLaunchKernelGGL(k_direct_select, grid, dim3(kDirectThreads), 0, s, (const uint32_t*)seed, sw32,
                           (const uint32_t*)kr, kw4, y0 * kc, (uint32_t)kc, idx, count, res);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace pa
