// One-kernel tiles for the shortest FFT lengths (L <= 2^13): a whole tile
// lives in one workgroup, in registers with LDS for the exchanges
// (lds_slots<L, 1> elements: 70 KB in FP32, 139 KB in FP64), so the three
// passes of the longer classes become one launch and no workspace is written.
// (FP32 L = 2^14 would also fit, but one workgroup then takes 42 us for a
// tile that the three-pass kernels spread over the device in about 30.)
//
// A workgroup of L/16 threads takes one tile through the steps of section 3,
// steps 1-3, for its key chunk and output window:
//  1. stage the tile's key and seed bits in LDS, one 32-bit word per 32
//     positions (the chunk placed as in the longer classes, the seed slice
//     up to Bi + Bo - 1), and count the key bits (the chunk weight);
//  2. z_t = x_t + i s_t (key bit, seed +-1 inside the window, 0 after it) and
//     its L-point forward transform (Stockham stages, fft_core.hpp);
//  3. the product of the separated spectra, C_k = X_k W_k / L from Z_k and
//     Z_{-k} (exchanged through LDS);
//  4. the real inverse through one half-length transform: U_k = E_k + i O_k,
//     E_k = C_k + conj C_{L/2-k}, O_k = (C_k - conj C_{L/2-k}) w_L^{-k}, whose
//     unnormalised inverse holds z_{2t} + i z_{2t+1};
//  5. window, exact rounding and parity (bit = bit 1 of rint(z) + weight,
//     check = bit 0), the output bits gathered in an LDS bitmap and written as
//     32-bit words (XOR-ed in when the job accumulates key chunks), and the
//     tile's certificate written to meta (one workgroup per tile: no atomics).
// A launch that holds chunk-0 tiles of accumulated jobs first runs a kernel
// that clears their windows (the XORs of the other chunks' tiles, in the same
// launch, must find the words cleared).
#pragma once
#include "conv_kernels.hpp"

namespace pa {

// Lengths with a one-kernel tile: the whole tile's exchange buffer fits LDS.
template <typename T> constexpr int fused_max_logL() { return 13; }

// (T only gives each precision's object file an instantiation of its own)
template <typename T>
__global__ void __launch_bounds__(256) k_tile_clear(JobTable jt) {
    const uint32_t t = jt.tile0 + blockIdx.x;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    clear_window(g, 0, 1, threadIdx.x, 256);
}

template <typename T, int L>
__global__ void __launch_bounds__(L / 16) k_tile(JobTable jt, TileMeta* __restrict__ meta, const cx<T>* __restrict__ tw) {
    constexpr int R = 16, NTH = L / R, H = L / 2, RH = 8, NW = L / 32;
    static_assert(H / RH == NTH, "the half-length inverse keeps every thread busy");
    static_assert(2 * NW * 4 <= lds_slots<L, 1>() * (int)sizeof(cx<T>), "bit words fit the exchange buffer");
    __shared__ cx<T> lds[lds_slots<L, 1>()];
    __shared__ uint32_t s_pc, s_res, s_abs, s_bad;
    uint32_t* words = reinterpret_cast<uint32_t*>(lds);   // key words [0, NW), seed words [NW, 2 NW)

    const uint32_t t = jt.tile0 + blockIdx.x;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const int j = threadIdx.x;
    const uint32_t bi = (uint32_t)g.bi, win = (uint32_t)(g.bi + g.bo - 1);
    if (j == 0) {
        s_pc = 0;
        s_res = 0;
        s_abs = 0;
        s_bad = 0;
    }
    __syncthreads();

    // 1. the tile's bits
    uint32_t pc = 0;
    for (int w = j; w < NW; w += NTH) {
        const uint32_t s0 = 32u * (uint32_t)w;
        const uint32_t kb = (uint32_t)placed_key_bits<32>(jd.key, g.j0, bi, (uint32_t)L, s0);
        const uint32_t nv = s0 < win ? ((win - s0) < 32u ? (win - s0) : 32u) : 0u;
        words[w] = kb;
        words[NW + w] = (uint32_t)extract_bits(jd.seed, g.sigma + s0, nv);
        pc += (uint32_t)__popc(kb);
    }
    atomicAdd(&s_pc, pc);
    __syncthreads();

    // 2. z and its forward transform (register i: point j + i NTH)
    cx<T> v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t p = (uint32_t)(j + i * NTH);
        const uint32_t kw = (words[p >> 5] >> (p & 31u)) & 1u;
        const uint32_t sw = (words[NW + (p >> 5)] >> (p & 31u)) & 1u;
        v[i] = cx<T>{kw ? T(1) : T(0), p < win ? (sw ? T(1) : T(-1)) : T(0)};
    }
    const uint32_t weight = s_pc;
    fft<T, -1, L, R, 1, L>(v, lds, j, 0, tw);   // its first exchange waits for every thread

    // 3. C_k = X_k W_k / L (spectrum_product folds the 1/L)
    const T quarter = T(0.25) / T(L);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) lds[lds_slot<1>(j + i * NTH, 0)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int k = j + i * NTH;
        v[i] = spectrum_product(v[i], lds[lds_slot<1>((L - k) & (L - 1), 0)], quarter);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) lds[lds_slot<1>(j + i * NTH, 0)] = v[i];
    __syncthreads();

    // 4. U_k, k < L/2 (register i: k = j + i NTH), and its inverse
    cx<T> u[RH];
#pragma unroll
    for (int i = 0; i < RH; ++i) {
        const int k = j + i * NTH;
        const cx<T> c = lds[lds_slot<1>(k, 0)];
        const cx<T> cm = conj(lds[lds_slot<1>(H - k, 0)]);
        const cx<T> e = c + cm;
        const cx<T> o = cmulc(c - cm, tw[k]);
        u[i] = cx<T>{e.re - o.im, e.im + o.re};
    }
    fft<T, +1, H, RH, 1, L>(u, lds, j, 0, tw);

    // 5. window, rounding, parity, bits and certificate
    __syncthreads();   // the exchange buffer becomes the output bitmap
    uint32_t* bitmap = reinterpret_cast<uint32_t*>(lds);
    for (int w = j; w < NW; w += NTH) bitmap[w] = 0;
    __syncthreads();
    const uint32_t bo = (uint32_t)g.bo;
    float mres = 0.f, mabs = 0.f;
    uint32_t bad = 0;
#pragma unroll
    for (int i = 0; i < RH; ++i) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t p = 2u * (uint32_t)(j + i * NTH) + (uint32_t)e;
            if (p >= bo) continue;
            const T z = e ? u[i].im : u[i].re;
            const T r = round_even(z);
            const int64_t s2 = (int64_t)r + (int64_t)weight;   // = 2 c when exact
            // an odd sum, or a non-finite z (fmaxf below would drop a NaN)
            bad += (uint32_t)(s2 & 1) + (fabs(z - r) <= T(0.5) ? 0u : 1u);
            mres = fmaxf(mres, (float)fabs(z - r));
            mabs = fmaxf(mabs, (float)fabs(z));
            if ((s2 >> 1) & 1) atomicOr(&bitmap[p >> 5], 1u << (p & 31u));
        }
    }
    atomicMax(&s_res, __float_as_uint(mres));
    atomicMax(&s_abs, __float_as_uint(mabs));
    atomicAdd(&s_bad, bad);
    __syncthreads();
    const uint32_t nw = (uint32_t)(2 * g.dst_words);   // 32-bit words of the window
    for (uint32_t w = (uint32_t)j; w < nw; w += NTH) put_bits<32>(g, 32ull * w, bitmap[w]);
    if (j == 0) meta[t] = TileMeta{weight, s_res, s_abs, s_bad};
}

// Launchers: pass 1 clears the windows of chunk-0 tiles when the launch has
// any (no kernel otherwise), pass 2 runs the tiles, pass 3 has nothing left.
// A return of 1 means that no kernel was launched.
template <typename T, int L>
struct ClassImplF {
    static_assert(L <= (1 << fused_max_logL<T>()), "one-kernel tile length");
    static bool clears(const JobTable& jt) {
        return jt.njobs == 0 ? (jt.one.nchunks > 1 && !jt.one.no_clear) : jt.clears != 0;
    }
    static int pass1(const JobTable& jt, void*, uint32_t*, TileMeta*, const Tables&, void* stream) {
        if (!clears(jt)) return 1;
        hipLaunchKernelGGL(k_tile_clear<T>, dim3(jt.ntiles), dim3(256), 0, (hipStream_t)stream, jt);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass2(const JobTable& jt, void*, uint32_t*, TileMeta* meta, const Tables& tb, void* stream) {
        hipLaunchKernelGGL((k_tile<T, L>), dim3(jt.ntiles), dim3(L / 16), 0, (hipStream_t)stream, jt, meta,
                           (const cx<T>*)tb.tw);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass3(const JobTable&, void*, uint32_t*, TileMeta*, const Tables&, void*) { return 1; }
};

}  // namespace pa
