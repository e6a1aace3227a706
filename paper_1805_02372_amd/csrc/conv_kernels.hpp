// The Toeplitz-hash tile pipeline as three HIP kernels with workgroup-wide
// Stockham transforms (the short length classes).
//
// A tile convolves a seed slice w (bi+bo-1 bits, encoded +-1) with a key
// chunk x (bi bits, encoded 0/1) circularly over L = n1*n2 >= bi+bo-1 points
// and keeps outputs [bi-1, bi-1+bo) (paper section 3, step 3; Eq. 4-7).  The
// key chunk is placed at circular offset -(bi-1), so the kept window starts at
// index 0.  With the +-1 seed, z = w (*) x equals 2c - weight(x) on the window,
// c being the 0/1 convolution, so bit = ((rint(z) + weight) / 2) mod 2 (Eq. 7).
//
// Both sequences share one complex FFT: z_t = x_t + i w_t.  The length-L FFT
// is split four-step, t = t1 + n1 t2, k = k2 + n2 k1:
//
//   pass 1 (columns): for each t1, Y[k2][t1] = w_L^{t1 k2} sum_t2 z[t1+n1 t2] w_n2^{t2 k2}
//   pass 2 (rows)   : Z[k2 + n2 k1] = sum_t1 Y[k2][t1] w_n1^{t1 k1}; the spectra of
//                     x and w are separated from Z_k and conj Z_{-k} (rows k2 and
//                     n2-k2 pair up), multiplied, and the inverse row transform
//                     gives V[k2][t1] = w_L^{-k2 t1} sum_k1 P[k2+n2 k1] w_n1^{-k1 t1}.
//                     V is Hermitian in k2, so rows 0..n2/2 suffice; rows 0 and
//                     n2/2 are real and share row 0 (re / im).  V overwrites Y.
//   pass 3 (columns): for each t1 the real inverse over k2 is one n2/2-point
//                     complex transform giving c[t1 + n1 (2t')] and
//                     c[t1 + n1 (2t'+1)] as real and imaginary parts; round,
//                     parity, pack 64 outputs per ballot, store.
//
// HBM traffic per tile (element size e = 8 B for FP32 complex, 16 B for FP64):
// pass 1 writes e L, pass 2 reads e L and writes e L/2, pass 3 reads e L/2 —
// 3 e L bytes (24 L for FP32, 48 L for FP64), plus the bits.
#pragma once
#include "fft_core.hpp"
#include "pa_internal.hpp"

namespace pa {

__device__ __forceinline__ JobDesc find_job(const JobTable& jt, uint32_t t) {
    if (jt.njobs == 0) return jt.one;
    uint32_t lo = 0, hi = jt.njobs - 1;
    while (lo < hi) {  // last job with tile_begin <= t
        uint32_t mid = (lo + hi + 1) >> 1;
        if (jt.many[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    return jt.many[lo];
}

struct TileGeo {
    uint64_t j0, bi, i0, bo, sigma;
    uint64_t* dst;        // output words of this tile's window (bit 0 = output i0)
    uint64_t dst_words;
    bool accumulate;      // several key chunks: XOR into dst (cleared by the chunk-0 tile)
    bool clears;          // this tile is chunk 0 of an accumulated window
};

__device__ __forceinline__ TileGeo tile_geo(const JobDesc& jd, uint32_t lt) {
    TileGeo g;
    const uint32_t b = lt / jd.nouts, o = lt % jd.nouts;
    const uint64_t hi = jd.n - (uint64_t)b * jd.Bi;
    const uint64_t lo = hi > jd.Bi ? hi - jd.Bi : 0;
    g.j0 = lo;
    g.bi = hi - lo;
    g.i0 = (uint64_t)o * jd.Bo;
    const uint64_t rest = jd.m - g.i0;
    g.bo = rest < jd.Bo ? rest : jd.Bo;
    g.sigma = g.i0 + jd.n - hi;
    g.dst = jd.out + (g.i0 >> 6);
    g.dst_words = (g.bo + 63) >> 6;
    g.accumulate = jd.nchunks > 1;
    g.clears = g.accumulate && b == 0 && !jd.no_clear;
    return g;
}

// Pass 1 of a chunk-0 tile of an accumulated job clears the window's words;
// `part` of `parts` workgroups of the tile take an interleaved share.
__device__ __forceinline__ void clear_window(const TileGeo& g, uint32_t part, uint32_t parts, int tid, int nthreads) {
    if (!g.clears) return;
    for (uint64_t w = (uint64_t)part * nthreads + tid; w < g.dst_words; w += (uint64_t)parts * nthreads) g.dst[w] = 0;
}

// Write B output bits at bit offset `off` (a multiple of B) of the window:
// a plain store, or an XOR into the 32-bit word holding them when the job
// accumulates chunks (zero groups are skipped).
template <int B>
__device__ __forceinline__ void put_bits(const TileGeo& g, uint64_t off, uint32_t bits) {
    static_assert(B == 8 || B == 16 || B == 32, "bit group");
    if (g.accumulate) {
        if (bits) atomicXor(reinterpret_cast<uint32_t*>(g.dst) + (off >> 5), B == 32 ? bits : bits << (off & 31));
    } else if constexpr (B == 32) {
        reinterpret_cast<uint32_t*>(g.dst)[off >> 5] = bits;
    } else if constexpr (B == 16) {
        reinterpret_cast<uint16_t*>(g.dst)[off >> 4] = (uint16_t)bits;
    } else {
        reinterpret_cast<uint8_t*>(g.dst)[off >> 3] = (uint8_t)bits;
    }
}

// Bits [pos, pos + cnt) of a bit string (cnt <= 64), LSB first.
__device__ __forceinline__ uint64_t extract_bits(const uint64_t* __restrict__ a, uint64_t pos, uint32_t cnt) {
    if (cnt == 0) return 0;
    const uint64_t w = pos >> 6;
    const uint32_t s = (uint32_t)(pos & 63);
    uint64_t v = a[w] >> s;
    if (s + cnt > 64) v |= a[w + 1] << (64 - s);
    return cnt >= 64 ? v : (v & ((1ull << cnt) - 1));
}

// Key bits of the placed chunk for C consecutive positions t = s0 .. s0+C-1:
// position t holds key bit j0 + ((t + bi - 1) mod L) when that index is < bi.
template <int C>
__device__ __forceinline__ uint64_t placed_key_bits(const uint64_t* __restrict__ key, uint64_t j0, uint32_t bi,
                                                    uint32_t L, uint32_t s0) {
    uint32_t u0 = s0 + bi - 1;
    if (u0 >= L) u0 -= L;
    auto part = [&](uint32_t ustart, uint32_t fstart, uint32_t count) -> uint64_t {
        if (ustart >= bi || count == 0) return 0;
        const uint32_t nv = (bi - ustart) < count ? (bi - ustart) : count;
        return extract_bits(key, j0 + ustart, nv) << fstart;
    };
    if (u0 + C <= L) return part(u0, 0, C);
    const uint32_t fs = L - u0;  // positions at and after fs wrap to the start
    return part(u0, 0, fs) | part(0, fs, C - fs);
}

template <typename T>
__device__ __forceinline__ cx<T> four_step_root(const cx<T>* __restrict__ fa, const cx<T>* __restrict__ fb,
                                                int fshift, uint32_t e) {
    return cmul(fa[e >> fshift], fb[e & ((1u << fshift) - 1u)]);
}

template <int A, int B> constexpr int cmax() { return A > B ? A : B; }

// ------------------------------------------------------------------ pass 1
// NT2: length of the root table tw of the column transforms (a multiple of N2).
// FP64 column passes take the split exchange where their complex buffer
// would leave room for one workgroup per compute unit, and their registers
// are budgeted for two workgroups (the mixed-radix columns of 1280 to 1792
// points, no spills).  FP32 column workgroups of eight and more waves then
// get 128 registers or fewer and spill: measured slower.
template <typename T, int N, int F> constexpr bool column_split() {
    return split_exchange<T, N, F>() && sizeof(T) == 8;
}
template <typename T, int N, int F, int THREADS> constexpr int column_waves_per_eu() {
    return column_split<T, N, F>() ? (2 * THREADS / 64 + 3) / 4 : 1;
}
template <typename T, int N1, int N2, int B, int R, int NT2>
__global__ void __launch_bounds__(B * (N2 / R))
__attribute__((amdgpu_waves_per_eu(column_waves_per_eu<T, N2, B, B * (N2 / R)>())))
k_pass1(JobTable jt, cx<T>* __restrict__ ws, uint32_t* __restrict__ part,
        const cx<T>* __restrict__ tw, const cx<T>* __restrict__ fa, const cx<T>* __restrict__ fb, int fshift) {
    constexpr uint32_t L = (uint32_t)N1 * N2;
    constexpr int NCB = N1 / B, NR = N2 / R, NT = NT2;
    constexpr bool SPLIT = column_split<T, N2, B>();
    __shared__ cx<T> lds[SPLIT ? (lds_slots<N2, B>() + 1) / 2 : lds_slots<N2, B>()];
    __shared__ uint32_t wsum;

    const uint32_t lt = blockIdx.x / NCB;          // tile within this launch
    const uint32_t cb = blockIdx.x % NCB;
    const uint32_t t = jt.tile0 + lt;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const int tid = threadIdx.x, f = tid % B, j = tid / B;
    const uint32_t t1 = cb * B + f;
    if (tid == 0) wsum = 0;
    clear_window(g, cb, NCB, tid, B * (N2 / R));

    // Stage this workgroup's key and seed bits in LDS: per row t2 the B-bit
    // fields at positions cb B + N1 t2 .. + B - 1 (key bits low, seed bits
    // high), read as funnel-shifted words instead of one load per point.  The
    // FFT's first barrier precedes its first LDS write.
    static_assert(B <= 8 && 2 * N2 <= lds_slots<N2, B>() * (int)sizeof(T), "bit fields");
    constexpr int NTH = B * (N2 / R);
    uint16_t* fld = reinterpret_cast<uint16_t*>(lds);
    const uint32_t bi = (uint32_t)g.bi, win = (uint32_t)(g.bi + g.bo - 1);
    uint32_t pc = 0;
    for (int r = tid; r < N2; r += NTH) {
        const uint32_t s0 = cb * B + (uint32_t)N1 * (uint32_t)r;
        const uint32_t kbits = (uint32_t)placed_key_bits<B>(jd.key, g.j0, bi, L, s0);
        const uint32_t nv = s0 < win ? ((win - s0) < (uint32_t)B ? (win - s0) : (uint32_t)B) : 0u;
        const uint32_t sbits = (uint32_t)extract_bits(jd.seed, g.sigma + s0, nv);
        fld[r] = (uint16_t)(kbits | (sbits << 8));
        pc += (uint32_t)__popc(kbits);
    }
    __syncthreads();
    cx<T> v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t t2 = (uint32_t)(j + i * NR);
        const uint32_t tt = t1 + (uint32_t)N1 * t2;
        const uint32_t w = fld[t2];
        const T xb = ((w >> f) & 1u) ? T(1) : T(0);
        const T sv = ((w >> (8 + f)) & 1u) ? T(1) : T(-1);
        v[i] = cx<T>{xb, tt < win ? sv : T(0)};
    }
    atomicAdd(&wsum, pc);

    fft<T, -1, N2, R, B, NT, SPLIT>(v, lds, j, f, tw);

    cx<T>* __restrict__ Y = ws + (size_t)lt * L;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t k2 = (uint32_t)(j + i * NR);
        const cx<T> w = four_step_root(fa, fb, fshift, t1 * k2);   // t1*k2 < L
        Y[(size_t)k2 * N1 + t1] = cmul(v[i], w);
    }
    __syncthreads();
    if (tid == 0) part[(size_t)lt * NCB + cb] = wsum;
}

// ------------------------------------------------------------------ pass 2

// X_k W_k / L from Z_k = a and Z_{-k} = m:  X = (a + conj m)/2,
// W = (a - conj m)/(2i), so X W = (a + conj m)(a - conj m) / (4i).  `quarter`
// is 1/(4L) (the 1/L inverse normalisation folded in; exact for L = 2^k).
// The product form keeps the error relative to |X||W| (a difference of
// squares would make it relative to |X|^2 + |W|^2).
template <typename T> __device__ __forceinline__ cx<T> spectrum_product(cx<T> a, cx<T> m, T quarter) {
    const cx<T> mc = conj(m);
    const cx<T> p = cmul(a + mc, a - mc);
    return cx<T>{p.im * quarter, -p.re * quarter};   // -i p / (4L)
}

template <typename T, int N1, int R>
__device__ __forceinline__ void load_row(cx<T> (&v)[R], const cx<T>* __restrict__ row, int j) {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = row[j + i * (N1 / R)];
}

// Replace the thread's values b[i] (at k1 = j + i N1/R) by the value at the
// mirrored index: (N1 - k1) mod N1 when ZERO, else N1 - 1 - k1.
template <typename T, int N1, int R, bool ZERO>
__device__ __forceinline__ void mirror(cx<T> (&b)[R], cx<T>* lds, int j) {
    constexpr int NR = N1 / R;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) lds[lds_slot<1>(j + i * NR, 0)] = b[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int k1 = j + i * NR;
        const int src = ZERO ? ((N1 - k1) % N1) : (N1 - 1 - k1);
        b[i] = lds[lds_slot<1>(src, 0)];
    }
}

// NT1: length of the root table tw of the row transforms (a multiple of N1).
template <typename T, int N1, int N2, int R, int NCB1, int NT1>
__global__ void __launch_bounds__(N1 / R)
k_pass2(JobTable jt, cx<T>* __restrict__ ws, const uint32_t* __restrict__ part, TileMeta* __restrict__ meta,
        const cx<T>* __restrict__ tw, const cx<T>* __restrict__ fa, const cx<T>* __restrict__ fb, int fshift) {
    constexpr uint32_t L = (uint32_t)N1 * N2;
    constexpr int NR = N1 / R, NP = N2 / 2, NT = NT1;
    __shared__ cx<T> lds[lds_slots<N1, 1>()];
    __shared__ uint32_t wsum;

    const uint32_t lt = blockIdx.x / NP;
    const int pr = blockIdx.x % NP;
    cx<T>* __restrict__ Y = ws + (size_t)lt * L;
    const int j = threadIdx.x;
    const T scale = T(0.25) / T(L);

    if (pr == 0) {
        // key-chunk weight from the pass-1 partial sums; reset the certificate
        if (j == 0) wsum = 0;
        __syncthreads();
        uint32_t s = 0;
        for (int c = j; c < NCB1; c += NR) s += part[(size_t)lt * NCB1 + c];
        atomicAdd(&wsum, s);
        __syncthreads();
        if (j == 0) meta[jt.tile0 + lt] = TileMeta{wsum, 0u, 0u, 0u};

        // Rows 0 and n2/2 are their own mirrors and their V rows are real.  Row
        // 0's result is parked in its own (already consumed) slots of Y, read
        // back by the same thread, and joined with row n2/2's as re / im.
        {
            cx<T> a[R], b[R];
            load_row<T, N1, R>(a, Y, j);
            fft<T, -1, N1, R, 1, NT>(a, lds, j, 0, tw);
#pragma unroll
            for (int i = 0; i < R; ++i) b[i] = a[i];
            mirror<T, N1, R, true>(b, lds, j);
#pragma unroll
            for (int i = 0; i < R; ++i) a[i] = spectrum_product(a[i], b[i], scale);
            fft<T, +1, N1, R, 1, NT>(a, lds, j, 0, tw);
#pragma unroll
            for (int i = 0; i < R; ++i) Y[j + i * NR] = a[i];
        }
        {
            cx<T> a[R], b[R];
            load_row<T, N1, R>(a, Y + (size_t)NP * N1, j);
            fft<T, -1, N1, R, 1, NT>(a, lds, j, 0, tw);
#pragma unroll
            for (int i = 0; i < R; ++i) b[i] = a[i];
            mirror<T, N1, R, false>(b, lds, j);
#pragma unroll
            for (int i = 0; i < R; ++i) a[i] = spectrum_product(a[i], b[i], scale);
            fft<T, +1, N1, R, 1, NT>(a, lds, j, 0, tw);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const uint32_t t1 = (uint32_t)(j + i * NR);
                const cx<T> w = four_step_root(fa, fb, fshift, (uint32_t)NP * t1);
                const cx<T> vv = cmulc(a[i], w);
                Y[t1] = cx<T>{Y[t1].re, vv.re};
            }
        }
    } else {
        cx<T> a[R], b[R];
        load_row<T, N1, R>(a, Y + (size_t)pr * N1, j);
        fft<T, -1, N1, R, 1, NT>(a, lds, j, 0, tw);
        load_row<T, N1, R>(b, Y + (size_t)(N2 - pr) * N1, j);
        fft<T, -1, N1, R, 1, NT>(b, lds, j, 0, tw);
        mirror<T, N1, R, false>(b, lds, j);
#pragma unroll
        for (int i = 0; i < R; ++i) a[i] = spectrum_product(a[i], b[i], scale);
        fft<T, +1, N1, R, 1, NT>(a, lds, j, 0, tw);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint32_t t1 = (uint32_t)(j + i * NR);
            const cx<T> w = four_step_root(fa, fb, fshift, (uint32_t)pr * t1);
            Y[(size_t)pr * N1 + t1] = cmulc(a[i], w);
        }
    }
}

// ------------------------------------------------------------------ pass 3
template <typename T> __device__ __forceinline__ T round_even(T z);
template <> __device__ __forceinline__ float round_even<float>(float z) { return rintf(z); }
template <> __device__ __forceinline__ double round_even<double>(double z) { return rint(z); }

// NT2: length of the root table tw of the column transforms (a multiple of N2).
// SPLIT: the real rows 0 and n2/2 of V are in the real parts of rows 0 and
// n2/2 (the layout of the wave-level row pass, conv_v2.hpp) instead of sharing
// row 0 as re / im.
template <typename T, int N1, int N2, int B, int R, int NT2, bool SPLIT = false>
__global__ void __launch_bounds__(B * (N2 / 2 / R))
__attribute__((amdgpu_waves_per_eu(column_waves_per_eu<T, N2 / 2, B, B * (N2 / 2 / R)>())))
k_pass3(JobTable jt, const cx<T>* __restrict__ ws, TileMeta* __restrict__ meta, const cx<T>* __restrict__ tw) {
    constexpr uint32_t L = (uint32_t)N1 * N2;
    constexpr int N2h = N2 / 2, NR = N2h / R, NCB = N1 / B, NT = NT2;
    static_assert(64 % B == 0, "column groups must tile a wavefront");
    constexpr bool XSPLIT = column_split<T, N2h, B>();
    __shared__ cx<T> lds[XSPLIT ? (lds_slots<N2h, B>() + 1) / 2 : lds_slots<N2h, B>()];
    __shared__ uint32_t s_res, s_abs, s_bad;

    const uint32_t lt = blockIdx.x / NCB;
    const uint32_t cb = blockIdx.x % NCB;
    const uint32_t t = jt.tile0 + lt;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const cx<T>* __restrict__ V = ws + (size_t)lt * L;
    const int tid = threadIdx.x, f = tid % B, j = tid / B;
    const uint32_t t1 = cb * B + f;
    if (tid == 0) { s_res = 0; s_abs = 0; s_bad = 0; }
    const int64_t weight = (int64_t)meta[t].popcnt;

    // Hermitian column H[k] = V[k][t1] (k < n2/2), H[n2/2] in the imaginary
    // part of row 0 (SPLIT: the real part of row n2/2).  The block of B
    // columns is read once as B-element row segments into LDS, where each
    // thread pairs k with n2/2 - k.  U[k] = E[k] + i O[k] with
    // E = H[k] + conj H[n2/2-k], O = (H[k] - conj H[n2/2-k]) w_n2^{-k}.
    constexpr int NTH = B * (N2h / R);
    __shared__ T hrow[B];
    if (tid < B) hrow[tid] = SPLIT ? V[(size_t)N2h * N1 + cb * B + tid].re : V[cb * B + tid].im;
    // XSPLIT: each thread reads both rows of its pairs from global memory
    // (B-element row segments; the second read of a row comes from the L2),
    // so that the LDS holds only the exchanges of the transform
    if constexpr (!XSPLIT) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int x = tid + q * NTH, k = x / B, c = x % B;
            lds[lds_slot<B>(k, c)] = V[(size_t)k * N1 + cb * B + c];
        }
    }
    __syncthreads();
    cx<T> v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int k = j + i * NR;
        const cx<T> h = XSPLIT ? V[(size_t)k * N1 + t1] : lds[lds_slot<B>(k, f)];
        if (k == 0) {
            const T hh = hrow[f];   // H[n2/2]
            v[i] = cx<T>{h.re + hh, h.re - hh};
        } else {
            const cx<T> hm = conj(XSPLIT ? V[(size_t)(N2h - k) * N1 + t1] : lds[lds_slot<B>(N2h - k, f)]);
            const cx<T> e = h + hm;
            const cx<T> o = cmulc(h - hm, tw[k * (NT / N2)]);
            v[i] = cx<T>{e.re - o.im, e.im + o.re};
        }
    }
    fft<T, +1, N2h, R, B, NT, XSPLIT>(v, lds, j, f, tw);

    float mres = 0.f, mabs = 0.f;
    uint32_t bad = 0;
    const int lane = tid & 63;
#pragma unroll
    for (int i = 0; i < R; ++i) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t t2 = 2u * (uint32_t)(j + i * NR) + (uint32_t)e;
            const uint64_t vo = (uint64_t)t1 + (uint64_t)N1 * t2;
            const T z = e ? v[i].im : v[i].re;
            uint32_t bit = 0;
            if (vo < g.bo) {
                const T r = round_even(z);
                const int64_t s2 = (int64_t)r + weight;      // = 2c when exact
                bit = (uint32_t)(s2 >> 1) & 1u;
                // an odd sum, or a non-finite z (fmaxf would drop a NaN)
                bad += (uint32_t)(s2 & 1) + (fabs(z - r) <= T(0.5) ? 0u : 1u);
                mres = fmaxf(mres, (float)fabs(z - r));
                mabs = fmaxf(mabs, (float)fabs(z));
            }
            const uint64_t mask = __ballot(bit);
            if (f == 0) {
                const uint64_t off = (uint64_t)cb * B + (uint64_t)N1 * t2;
                if (off < g.dst_words * 64u) put_bits<B>(g, off, (uint32_t)(mask >> lane) & ((1u << B) - 1u));
            }
        }
    }
    __syncthreads();
    atomicMax(&s_res, __float_as_uint(mres));
    atomicMax(&s_abs, __float_as_uint(mabs));
    atomicAdd(&s_bad, bad);
    __syncthreads();
    if (tid == 0) {
        atomicMax(&meta[t].maxres, s_res);
        atomicMax(&meta[t].maxabs, s_abs);
        if (s_bad) atomicAdd(&meta[t].badpar, s_bad);
    }
}

// Launchers of one class.  RR / RC: points per thread of the row / column
// transforms.  SMOOTH: a mixed-radix class, whose row and column transforms
// take their roots from separate tables of exactly N1 (tw) and N2 (tw2)
// entries; a power-of-two class uses one table of max(N1, N2) roots for both.
template <typename T, int N1, int N2, int B1, int B3, int RR, int RC, bool SMOOTH = false>
struct ClassImpl {
    static constexpr uint32_t L = (uint32_t)N1 * N2;
    static constexpr int NT1 = SMOOTH ? N1 : cmax<N1, N2>(), NT2 = SMOOTH ? N2 : cmax<N1, N2>();
    static int pass1(const JobTable& jt, void* ws, uint32_t* part, TileMeta*, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (N1 / B1)), block(B1 * (N2 / RC));
        hipLaunchKernelGGL((k_pass1<T, N1, N2, B1, RC, NT2>), grid, block, 0, (hipStream_t)stream, jt,
                           (cx<T>*)ws, part, (const cx<T>*)tb.tw2, (const cx<T>*)tb.fa, (const cx<T>*)tb.fb,
                           tb.fshift);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass2(const JobTable& jt, void* ws, uint32_t* part, TileMeta* meta, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (N2 / 2)), block(N1 / RR);
        hipLaunchKernelGGL((k_pass2<T, N1, N2, RR, N1 / B1, NT1>), grid, block, 0, (hipStream_t)stream, jt,
                           (cx<T>*)ws, (const uint32_t*)part, meta, (const cx<T>*)tb.tw, (const cx<T>*)tb.fa,
                           (const cx<T>*)tb.fb, tb.fshift);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass3(const JobTable& jt, void* ws, uint32_t*, TileMeta* meta, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (N1 / B3)), block(B3 * (N2 / 2 / RC));
        hipLaunchKernelGGL((k_pass3<T, N1, N2, B3, RC, NT2>), grid, block, 0, (hipStream_t)stream, jt,
                           (const cx<T>*)ws, meta, (const cx<T>*)tb.tw2);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
};

}  // namespace pa
