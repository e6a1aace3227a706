// Tile pipeline for the long FFT length classes (L = 8192 * n2, n2 = 128..2048):
// the same three passes as conv_kernels.hpp (see there for the mathematics),
// restructured around wave-level transforms (wave_fft.hpp):
//
//  * pass 1: the workgroup stages the key/seed bits of its C columns in LDS
//    (one funnel-shifted word per row instead of one load per point), each
//    wave transforms G whole columns (n2 <= 1024) or one half of a column
//    after a radix-2 split (n2 = 2048), and an LDS transpose turns the
//    column-major results into C-element row segments for the stores.
//  * pass 2: a row of 8192 points is a radix-8 stage across the 8 waves
//    (decimation in frequency, registers only) followed by one 1024-point
//    transform per wave; the inverse runs the same steps in reverse.  Two
//    workgroup barriers per row transform.
//  * pass 3: C columns are read as C-element row segments, transposed in
//    LDS, each wave inverts G columns, output bits are OR-ed into an LDS bit
//    array and stored as C-bit groups.
#pragma once
#include "conv_kernels.hpp"
#include "wave_fft.hpp"

namespace pa {

constexpr int kN1 = 8192;  // row length of the long classes

// Occupancy request for the row pass (default: none, the compiler fits the
// pair path without spills at two waves per SIMD).
#ifndef PA_PASS2_OCCUPANCY
#define PA_PASS2_OCCUPANCY
#endif

template <typename T, int N2> struct P1Geom {
    static constexpr int W = N2 > 1024 ? N2 / 1024 : 1;    // waves per column
    static constexpr int M = N2 > 1024 ? 1024 : N2;        // wave transform size
    static constexpr int G = 1024 / M;                     // columns per wave
    static constexpr int WAVES = (sizeof(T) == 4 && W > 1) ? 16 : 8;
    static constexpr int C = WAVES * G / W;                // columns per workgroup
    static constexpr int THREADS = WAVES * 64;
    static_assert(W <= 2, "column length up to 2048");
    static_assert(C <= 64 && (C & (C - 1)) == 0, "column block");
};

template <typename T, int N2> struct P3Geom {
    static constexpr int M = N2 / 2;                       // Hermitian half
    static constexpr int G = 1024 / M;
    static constexpr int WAVES = (sizeof(T) == 4 && G == 1) ? 16 : 8;   // >= 128 B row segments
    static constexpr int C = WAVES * G;
    static constexpr int THREADS = WAVES * 64;
    static constexpr int CW = (C + 31) / 32;               // 32-bit words per output row
};

// Transposition tile: row k2 of C elements, columns XOR-swizzled by the row.
template <int C> __device__ __forceinline__ int tslot(int k, int f) { return k * C + (f ^ (k & (C - 1))); }

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

// ------------------------------------------------------------------ pass 1
template <typename T, int N2>
__global__ void __launch_bounds__((P1Geom<T, N2>::THREADS))
k2_pass1(JobTable jt, cx<T>* __restrict__ ws, uint32_t* __restrict__ part, const cx<T>* __restrict__ tw,
         const cx<T>* __restrict__ fa, const cx<T>* __restrict__ fb, int fshift, const cx<T>* __restrict__ stw) {
    using Gm = P1Geom<T, N2>;
    constexpr int C = Gm::C, G = Gm::G, W = Gm::W, M = Gm::M, NJ = M / 16;
    constexpr uint32_t L = (uint32_t)kN1 * N2;
    constexpr int NCB = kN1 / C;
    constexpr int SLOTS = (Gm::WAVES * kWaveSlots > N2 * C) ? Gm::WAVES * kWaveSlots : N2 * C;
    static_assert(2 * N2 * sizeof(uint64_t) <= SLOTS * sizeof(cx<T>), "bit rows fit the LDS union");
    __shared__ __align__(16) cx<T> lds[SLOTS];
    __shared__ uint32_t wsum;
    uint64_t* kbits = reinterpret_cast<uint64_t*>(lds);   // consumed before the wave regions are used
    uint64_t* sbits = kbits + N2;

    const uint32_t lt = blockIdx.x / NCB;
    const uint32_t cb = blockIdx.x % NCB;
    const uint32_t t = jt.tile0 + lt;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const int tid = threadIdx.x;
    const uint32_t bi = (uint32_t)g.bi, win = (uint32_t)(g.bi + g.bo - 1);
    if (tid == 0) wsum = 0;
    __syncthreads();

    // stage the bits of this workgroup's C columns: rows r = tid + q * THREADS
    constexpr int RPT = (N2 + Gm::THREADS - 1) / Gm::THREADS;
    uint32_t pc = 0;
    uint64_t kb[RPT], sb[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = tid + q * Gm::THREADS;
        kb[q] = 0;
        sb[q] = 0;
        if (r < N2) {
            const uint32_t s0 = cb * C + (uint32_t)kN1 * (uint32_t)r;
            kb[q] = placed_key_bits<C>(jd.key, g.j0, bi, L, s0);
            const uint32_t nv = s0 < win ? ((win - s0) < (uint32_t)C ? (win - s0) : (uint32_t)C) : 0u;
            sb[q] = extract_bits(jd.seed, g.sigma + s0, nv);
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = tid + q * Gm::THREADS;
        if (r < N2) {
            kbits[r] = kb[q];
            sbits[r] = sb[q];
            pc += (uint32_t)__popcll(kb[q]);
        }
    }
    atomicAdd(&wsum, pc);
    __syncthreads();

    const int wv = tid >> 6, l = tid & 63;
    cx<T> v[16];
    int f, ka = 0, j;
    if constexpr (W == 1) {
        const int gg = l / NJ;
        j = l % NJ;
        f = wv * G + gg;
    } else {
        f = wv / W;
        ka = wv % W;
        j = l;
    }
    const uint32_t t1 = cb * C + (uint32_t)f;
    auto z = [&](int r) -> cx<T> {
        const T xb = (T)((kbits[r] >> f) & 1u);
        T wb = T(0);
        if (t1 + (uint32_t)kN1 * (uint32_t)r < win) wb = ((sbits[r] >> f) & 1u) ? T(1) : T(-1);
        return cx<T>{xb, wb};
    };
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = j + i * NJ;
        if constexpr (W == 1) {
            v[i] = z(e);
        } else {
            // radix-2 split of the 2048-point column: half ka, twiddle w_2048^{e ka}
            const cx<T> a = z(e), b = z(e + 1024);
            if (ka == 0) v[i] = a + b;
            else v[i] = cmul(a - b, tw[e * (kN1 / 2048)]);
        }
    }
    __syncthreads();  // bits consumed; LDS becomes wave regions
    cx<T>* reg = lds + wv * kWaveSlots + (W == 1 ? (l / NJ) * (M + M / 16) : 0);
    wave_fft<T, -1, M>(v, reg, j, stw);

    // four-step twiddle, then transpose through LDS for row-segment stores
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = j + i * NJ;
        const uint32_t k2 = (W == 1) ? (uint32_t)e : (uint32_t)(2 * e + ka);
        v[i] = cmul(v[i], four_step_root(fa, fb, fshift, t1 * k2));
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = j + i * NJ;
        const int k2 = (W == 1) ? e : 2 * e + ka;
        lds[tslot<C>(k2, f)] = v[i];
    }
    __syncthreads();
    cx<T>* __restrict__ Y = ws + (size_t)lt * L;
    static_assert((N2 * C) % Gm::THREADS == 0, "store tile");
    constexpr int SPT = N2 * C / Gm::THREADS;
    cx<T> o[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int idx = tid + q * Gm::THREADS;
        o[q] = lds[tslot<C>(idx / C, idx % C)];
    }
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int idx = tid + q * Gm::THREADS;
        Y[(size_t)(idx / C) * kN1 + cb * C + (idx % C)] = o[q];
    }
    if (tid == 0) part[(size_t)lt * NCB + cb] = wsum;
}

// ------------------------------------------------------------------ pass 2

// Forward transform of one 8192-point row.  Thread (wave w, lane l) ends with
// X[8 k_b + w] in register i, k_b = l + 64 i.
template <typename T>
__device__ __forceinline__ void row_forward(const cx<T>* __restrict__ row, cx<T> (&X)[16], cx<T>* lds, int wv,
                                            int l, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ stw) {
    constexpr int S = kWaveSlots;
    cx<T> a[16];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int nb = wv * 64 + l + 512 * s;
#pragma unroll
        for (int na = 0; na < 8; ++na) a[s * 8 + na] = row[nb + 1024 * na];
        dft8<-1>(&a[s * 8]);
        const cx<T>* __restrict__ tws = opaque(tw);
#pragma unroll
        for (int ka = 1; ka < 8; ++ka) a[s * 8 + ka] = cmul(a[s * 8 + ka], tws[nb * ka]);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int nb = wv * 64 + l + 512 * s;
#pragma unroll
        for (int ka = 0; ka < 8; ++ka) lds[ka * S + wslot(nb)] = a[s * 8 + ka];
    }
    __syncthreads();
    cx<T>* reg = lds + wv * S;
#pragma unroll
    for (int i = 0; i < 16; ++i) X[i] = reg[wslot(l + 64 * i)];
    wave_sync();
    wave_fft<T, -1, 1024>(X, reg, l, stw);
}

// Inverse transform of a row held as P[8 k_b + w] (register i, k_b = l + 64 i);
// returns a[t_b + 1024 t_a] in a[s * 8 + t_a] for t_b = w * 64 + l + 512 s.
template <typename T>
__device__ __forceinline__ void row_inverse(cx<T> (&P)[16], cx<T> (&a)[16], cx<T>* lds, int wv, int l,
                                            const cx<T>* __restrict__ tw, const cx<T>* __restrict__ stw) {
    constexpr int S = kWaveSlots;
    cx<T>* reg = lds + wv * S;
    __syncthreads();  // every wave is done with its region
    wave_fft<T, +1, 1024>(P, reg, l, stw);
#pragma unroll
    for (int i = 0; i < 16; ++i) P[i] = cmulc(P[i], opaque(tw)[wv * (l + 64 * i)]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) reg[wslot(l + 64 * i)] = P[i];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int tb = wv * 64 + l + 512 * s;
#pragma unroll
        for (int ka = 0; ka < 8; ++ka) a[s * 8 + ka] = lds[ka * S + wslot(tb)];
        dft8<+1>(&a[s * 8]);
    }
}

// Replace X (row layout of row_forward) by the values at the mirrored
// frequency: -k mod 8192 when `zero`, else 8191 - k.
template <typename T>
__device__ __forceinline__ void row_mirror(cx<T> (&X)[16], cx<T>* lds, int wv, int l, bool zero) {
    constexpr int S = kWaveSlots;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[wv * S + wslot(l + 64 * i)] = X[i];
    __syncthreads();
    const int sw = zero ? ((8 - wv) & 7) : (7 - wv);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int kb = l + 64 * i;
        const int sb = (zero && wv == 0) ? ((1024 - kb) & 1023) : (1023 - kb);
        X[i] = lds[sw * S + wslot(sb)];
    }
}

template <typename T, int N2, int NCB1>
__global__ void __launch_bounds__(512) PA_PASS2_OCCUPANCY
k2_pass2(JobTable jt, cx<T>* __restrict__ ws, const uint32_t* __restrict__ part, TileMeta* __restrict__ meta,
         const cx<T>* __restrict__ tw, const cx<T>* __restrict__ fa, const cx<T>* __restrict__ fb, int fshift,
         const cx<T>* __restrict__ stw) {
    constexpr uint32_t L = (uint32_t)kN1 * N2;
    constexpr int NP = N2 / 2;
    __shared__ __align__(16) cx<T> lds[8 * kWaveSlots];
    __shared__ uint32_t wsum;

    const uint32_t lt = blockIdx.x / NP;
    const int pr = blockIdx.x % NP;
    cx<T>* __restrict__ Y = ws + (size_t)lt * L;
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const T quarter = T(0.25) / T(L);

    if (pr == 0) {
        // key-chunk weight from the pass-1 partial sums; reset the certificate
        if (tid == 0) wsum = 0;
        __syncthreads();
        uint32_t s = 0;
        for (int c = tid; c < NCB1; c += 512) s += part[(size_t)lt * NCB1 + c];
        atomicAdd(&wsum, s);
        __syncthreads();
        if (tid == 0) meta[jt.tile0 + lt] = TileMeta{wsum, 0u, 0u, 0u};
    }
    // Workgroup pr > 0 owns the mirror pair of rows pr and n2-pr and produces
    // V row pr.  Workgroup 0 owns rows 0 and n2/2, which are their own mirrors
    // and whose V rows are real: row 0's goes to the real parts of row 0,
    // row n2/2's to the real parts of row n2/2 (each row is read only by this
    // workgroup, so storing in place is race-free).
    if (pr != 0) {
        cx<T> A[16], B[16], a[16];
        row_forward<T>(Y + (size_t)pr * kN1, A, lds, wv, l, tw, stw);
        row_forward<T>(Y + (size_t)(N2 - pr) * kN1, B, lds, wv, l, tw, stw);
        row_mirror<T>(B, lds, wv, l, false);
#pragma unroll
        for (int i = 0; i < 16; ++i) A[i] = spectrum_product(A[i], B[i], quarter);
        row_inverse<T>(A, a, lds, wv, l, tw, stw);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int ta = 0; ta < 8; ++ta) {
                const uint32_t t1 = (uint32_t)(wv * 64 + l + 512 * s + 1024 * ta);
                Y[(size_t)pr * kN1 + t1] = cmulc(a[s * 8 + ta], four_step_root(fa, fb, fshift, (uint32_t)pr * t1));
            }
    } else {
#pragma nounroll
        for (int u = 0; u < 2; ++u) {
            const int row = u == 0 ? 0 : NP;
            cx<T> A[16], B[16], a[16];
            row_forward<T>(Y + (size_t)row * kN1, A, lds, wv, l, tw, stw);
#pragma unroll
            for (int i = 0; i < 16; ++i) B[i] = A[i];
            row_mirror<T>(B, lds, wv, l, u == 0);
#pragma unroll
            for (int i = 0; i < 16; ++i) A[i] = spectrum_product(A[i], B[i], quarter);
            row_inverse<T>(A, a, lds, wv, l, tw, stw);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int ta = 0; ta < 8; ++ta) {
                    const uint32_t t1 = (uint32_t)(wv * 64 + l + 512 * s + 1024 * ta);
                    const cx<T> vv = cmulc(a[s * 8 + ta], four_step_root(fa, fb, fshift, (uint32_t)row * t1));
                    Y[(size_t)row * kN1 + t1] = cx<T>{vv.re, T(0)};
                }
        }
    }
}

// ------------------------------------------------------------------ pass 3
template <int C> __device__ __forceinline__ void store_bits(uint64_t* dst, uint64_t off, const uint32_t* w);
template <> __device__ __forceinline__ void store_bits<8>(uint64_t* dst, uint64_t off, const uint32_t* w) {
    reinterpret_cast<uint8_t*>(dst)[off >> 3] = (uint8_t)w[0];
}
template <> __device__ __forceinline__ void store_bits<16>(uint64_t* dst, uint64_t off, const uint32_t* w) {
    reinterpret_cast<uint16_t*>(dst)[off >> 4] = (uint16_t)w[0];
}

template <typename T, int N2>
__global__ void __launch_bounds__((P3Geom<T, N2>::THREADS))
k2_pass3(JobTable jt, const cx<T>* __restrict__ ws, TileMeta* __restrict__ meta, const cx<T>* __restrict__ tw,
         const cx<T>* __restrict__ stw) {
    using Gm = P3Geom<T, N2>;
    constexpr int C = Gm::C, G = Gm::G, M = Gm::M, NJ = M / 16, CW = Gm::CW;
    constexpr uint32_t L = (uint32_t)kN1 * N2;
    constexpr int NCB = kN1 / C;
    constexpr int SLOTS = (Gm::WAVES * kWaveSlots > M * C) ? Gm::WAVES * kWaveSlots : M * C;
    __shared__ __align__(16) cx<T> lds[SLOTS];
    __shared__ uint32_t obits[N2 * CW];
    __shared__ T hrow[C];
    __shared__ uint32_t s_res, s_abs, s_bad;

    const uint32_t lt = blockIdx.x / NCB;
    const uint32_t cb = blockIdx.x % NCB;
    const uint32_t t = jt.tile0 + lt;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const cx<T>* __restrict__ V = ws + (size_t)lt * L;
    const int tid = threadIdx.x;
    if (tid == 0) { s_res = 0; s_abs = 0; s_bad = 0; }
    for (int i = tid; i < N2 * CW; i += Gm::THREADS) obits[i] = 0;
    static_assert((M * C) % Gm::THREADS == 0, "load tile");
    constexpr int LPT = M * C / Gm::THREADS;
    {
        cx<T> in[LPT];
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int idx = tid + q * Gm::THREADS;
            in[q] = V[(size_t)(idx / C) * kN1 + cb * C + (idx % C)];
        }
        if (tid < C) hrow[tid] = V[(size_t)M * kN1 + cb * C + tid].re;   // H[n2/2], real
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int idx = tid + q * Gm::THREADS;
            lds[tslot<C>(idx / C, idx % C)] = in[q];
        }
    }
    __syncthreads();

    const int wv = tid >> 6, l = tid & 63;
    const int gg = l / NJ, j = l % NJ;
    const int f = wv * G + gg;
    const uint32_t t1 = cb * C + (uint32_t)f;
    const int64_t weight = (int64_t)meta[t].popcnt;
    cx<T> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int k = j + i * NJ;
        const cx<T> h = lds[tslot<C>(k, f)];
        if (k == 0) {
            // H[0] and H[n2/2] are real; H[n2/2] sits in the real parts of row n2/2
            const T hh = hrow[f];
            v[i] = cx<T>{h.re + hh, h.re - hh};
        } else {
            const cx<T> hm = conj(lds[tslot<C>(M - k, f)]);
            const cx<T> e = h + hm;
            const cx<T> o = cmulc(h - hm, tw[k * (kN1 / N2)]);
            v[i] = cx<T>{e.re - o.im, e.im + o.re};
        }
    }
    __syncthreads();  // tile consumed; LDS becomes wave regions
    cx<T>* reg = lds + wv * kWaveSlots + gg * (M + M / 16);
    wave_fft<T, +1, M>(v, reg, j, stw);

    float mres = 0.f, mabs = 0.f;
    uint32_t bad = 0;
    const uint32_t rows = (uint32_t)((g.bo + kN1 - 1) / kN1);  // rows t2 holding outputs
#pragma unroll
    for (int i = 0; i < 16; ++i) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t t2 = 2u * (uint32_t)(j + i * NJ) + (uint32_t)e;
            if (t2 >= rows) continue;
            const uint64_t vo = (uint64_t)t1 + (uint64_t)kN1 * t2;
            if (vo >= g.bo) continue;
            const T zz = e ? v[i].im : v[i].re;
            const T r = round_even(zz);
            const int64_t s2 = (int64_t)r + weight;
            bad += (uint32_t)(s2 & 1);
            mres = fmaxf(mres, (float)fabs(zz - r));
            mabs = fmaxf(mabs, (float)fabs(zz));
            if ((s2 >> 1) & 1) atomicOr(&obits[t2 * CW + (f >> 5)], 1u << (f & 31));
        }
    }
    atomicMax(&s_res, __float_as_uint(mres));
    atomicMax(&s_abs, __float_as_uint(mabs));
    atomicAdd(&s_bad, bad);
    __syncthreads();
    const uint64_t limit = g.dst_words * 64u;
    if constexpr (C >= 32) {
        for (uint32_t idx = tid; idx < rows * CW; idx += Gm::THREADS) {
            const uint32_t t2 = idx / CW, c = idx % CW;
            const uint64_t off = (uint64_t)cb * C + 32u * c + (uint64_t)kN1 * t2;
            if (off < limit) reinterpret_cast<uint32_t*>(g.dst)[off >> 5] = obits[t2 * CW + c];
        }
    } else {
        for (uint32_t t2 = tid; t2 < rows; t2 += Gm::THREADS) {
            const uint64_t off = (uint64_t)cb * C + (uint64_t)kN1 * t2;
            if (off < limit) store_bits<C>(g.dst, off, &obits[t2 * CW]);
        }
    }
    if (tid == 0) {
        atomicMax(&meta[t].maxres, s_res);
        atomicMax(&meta[t].maxabs, s_abs);
        if (s_bad) atomicAdd(&meta[t].badpar, s_bad);
    }
}

template <typename T, int N2>
struct ClassImpl2 {
    using G1 = P1Geom<T, N2>;
    using G3 = P3Geom<T, N2>;
    static constexpr int C1 = G1::C, C3 = G3::C;
    static int pass1(const JobTable& jt, void* ws, uint32_t* part, TileMeta*, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (kN1 / C1)), block(G1::THREADS);
        hipLaunchKernelGGL((k2_pass1<T, N2>), grid, block, 0, (hipStream_t)stream, jt, (cx<T>*)ws, part,
                           (const cx<T>*)tb.tw, (const cx<T>*)tb.fa, (const cx<T>*)tb.fb, tb.fshift,
                           (const cx<T>*)tb.stw);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass2(const JobTable& jt, void* ws, uint32_t* part, TileMeta* meta, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (N2 / 2)), block(512);
        hipLaunchKernelGGL((k2_pass2<T, N2, kN1 / C1>), grid, block, 0, (hipStream_t)stream, jt, (cx<T>*)ws,
                           (const uint32_t*)part, meta, (const cx<T>*)tb.tw, (const cx<T>*)tb.fa,
                           (const cx<T>*)tb.fb, tb.fshift, (const cx<T>*)tb.stw);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass3(const JobTable& jt, void* ws, uint32_t*, TileMeta* meta, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (kN1 / C3)), block(G3::THREADS);
        hipLaunchKernelGGL((k2_pass3<T, N2>), grid, block, 0, (hipStream_t)stream, jt, (const cx<T>*)ws, meta,
                           (const cx<T>*)tb.tw, (const cx<T>*)tb.stw);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
};

}  // namespace pa
