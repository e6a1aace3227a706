// Wave-level FFTs for gfx950: one 64-lane wavefront transforms G independent
// sequences of M points (M * G = 1024, 16 points per lane) in registers,
// exchanging between Stockham stages through a wave-private LDS region.  A
// wavefront executes its LDS operations in order, so the exchanges need no
// workgroup barrier, only compiler ordering (wave_sync).
//
// Register layout: lane = g * (M/16) + j; register i holds element
// j + i * (M/16) of transform g, before and after the transform.
//
// Stage twiddles come from per-stage tables laid out lane-major: for a stage
// of radix Rs and span Ns (Ns > 1), entry [k][r] (k < Ns, r < 16) holds
// w_{Ns Rs}^{k r} (forward root; zero for r >= Rs), so a lane's twiddles for
// one butterfly are 16 consecutive entries (wide, contiguous loads).
#pragma once
#include "fft_core.hpp"

namespace pa {

// Returns p unchanged, but the compiler cannot see through it: loads through
// the result cannot be hoisted above this point (keeps each stage's twiddle
// loads next to their use instead of all of them live at once).
template <typename P> __device__ __forceinline__ P opaque(P p) {
    asm volatile("" : "+s"(p));
    return p;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- stage tables (shared by host table builder and kernels)
constexpr int wfft_first_radix(int M) {
    int k = ilog2(M);
    return (k % 4) ? (1 << (k % 4)) : 16;
}
// Entries of the stage tables of one M (all stages with Ns > 1).
constexpr int wfft_table_size(int M) {
    int total = 0;
    int ns = wfft_first_radix(M);
    while (ns < M) {
        total += ns * 16;
        ns *= 16;
    }
    return total;
}
// Offset of stage Ns of transform size M within the size-M tables.
constexpr int wfft_stage_offset(int M, int Ns) {
    int off = 0;
    int ns = wfft_first_radix(M);
    while (ns < Ns) {
        off += ns * 16;
        ns *= 16;
    }
    return off;
}
constexpr int kWfftMinLog = 4, kWfftMaxLog = 10;
// Offset of the size-M tables within the table of all sizes 16..1024.
constexpr int wfft_size_offset(int M) {
    int off = 0;
    for (int lg = kWfftMinLog; (1 << lg) < M; ++lg) off += wfft_table_size(1 << lg);
    return off;
}
constexpr int wfft_tables_total() { return wfft_size_offset(1 << (kWfftMaxLog + 1)); }

// LDS slots of one wave region (1024 points, one pad slot per 16).
constexpr int kWaveSlots = 1024 + 64;
__device__ __forceinline__ int wslot(int e) { return e + (e >> 4); }

// Stage tables of one transform size M held in LDS, transposed (r-major):
// entry (k, r) of stage Ns at wfft_stage_offset(M, Ns) + r * Ns + k, so the
// lanes of a stage read consecutive entries (no bank conflicts).
constexpr int wfft_lds_entries(int M) { return wfft_table_size(M) > 0 ? wfft_table_size(M) : 1; }

template <typename T, int M, int Ns>
__device__ __forceinline__ void wfft_load_lds_from(cx<T>* __restrict__ st, const cx<T>* __restrict__ base, int tid,
                                                   int nthreads) {
    if constexpr (Ns < M) {
        constexpr int OFF = wfft_stage_offset(M, Ns);
        for (int x = tid; x < Ns * 16; x += nthreads) st[OFF + x] = base[OFF + (x % Ns) * 16 + x / Ns];
        wfft_load_lds_from<T, M, Ns * 16>(st, base, tid, nthreads);
    }
}

template <typename T, int M>
__device__ __forceinline__ void wfft_load_lds(cx<T>* __restrict__ st, const cx<T>* __restrict__ stw, int tid,
                                              int nthreads) {
    wfft_load_lds_from<T, M, wfft_first_radix(M)>(st, stw + wfft_size_offset(M), tid, nthreads);
}

// One Stockham stage.  LT: twiddles from the LDS copy `tab` (layout above),
// else from the global tables `tab` (lane-major).
template <typename T, int DIR, int M, int Rs, int Ns, bool LT>
__device__ __forceinline__ void wfft_stage(cx<T> (&v)[16], cx<T>* __restrict__ reg, int j, const cx<T>* tab) {
    constexpr int R = 16, P = R / Rs, NR = M / R;
    constexpr bool LAST = (Ns * Rs == M);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int q = j + p * NR;
        const int k = q & (Ns - 1);
        cx<T> u[Rs];
#pragma unroll
        for (int r = 0; r < Rs; ++r) u[r] = v[p + r * P];
        if constexpr (Ns > 1) {
            constexpr int OFF = wfft_stage_offset(M, Ns);
            if constexpr (LT) {
#pragma unroll
                for (int r = 1; r < Rs; ++r) u[r] = twmul<DIR>(u[r], tab[OFF + r * Ns + k]);
            } else {
                const cx<T>* __restrict__ tk = opaque(tab) + wfft_size_offset(M) + OFF + k * 16;
#pragma unroll
                for (int r = 1; r < Rs; ++r) u[r] = twmul<DIR>(u[r], tk[r]);
            }
        }
        dft<Rs, DIR>(u);
#pragma unroll
        for (int r = 0; r < Rs; ++r) v[p + r * P] = u[r];
    }
    if constexpr (!LAST) {
        wave_sync();
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int q = j + p * NR;
            const int k = q & (Ns - 1);
            const int base = (q / Ns) * Ns * Rs + k;
#pragma unroll
            for (int r = 0; r < Rs; ++r) reg[wslot(base + r * Ns)] = v[p + r * P];
        }
        wave_sync();
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = reg[wslot(j + i * NR)];
        wave_sync();
    }
}

template <typename T, int DIR, int M, int Ns, bool LT>
__device__ __forceinline__ void wfft_stages(cx<T> (&v)[16], cx<T>* __restrict__ reg, int j, const cx<T>* tab) {
    constexpr int Rs = (Ns == 1) ? wfft_first_radix(M) : 16;
    wfft_stage<T, DIR, M, Rs, Ns, LT>(v, reg, j, tab);
    if constexpr (Ns * Rs < M) wfft_stages<T, DIR, M, Ns * Rs, LT>(v, reg, j, tab);
}

// M-point transform of the values held by the M/16 lanes of one transform
// group; `reg` is that group's private LDS region (>= M + M/16 slots), `j` the
// lane within the group, `stw` the base of the global stage tables of all sizes.
template <typename T, int DIR, int M>
__device__ __forceinline__ void wave_fft(cx<T> (&v)[16], cx<T>* __restrict__ reg, int j,
                                         const cx<T>* __restrict__ stw) {
    static_assert(M >= 16 && M <= 1024 && (M & (M - 1)) == 0, "wave transform size");
    wfft_stages<T, DIR, M, 1, false>(v, reg, j, stw);
}

// 1024-point transform whose last stage (span 64) takes its twiddles from
// registers: tr[r-1] = w_1024^{j r} (forward root) for this lane j; the
// earlier stages read the LDS copy.
template <typename T, int DIR>
__device__ __forceinline__ void wave_fft1024_lds_reg(cx<T> (&v)[16], cx<T>* __restrict__ reg, int j, const cx<T>* st,
                                                     const cx<T> (&tr)[15]) {
    wfft_stage<T, DIR, 1024, 4, 1, true>(v, reg, j, st);
    wfft_stage<T, DIR, 1024, 16, 4, true>(v, reg, j, st);
    // last stage: span 64, radix 16, k = j
    cx<T> u[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) u[r] = v[r];
#pragma unroll
    for (int r = 1; r < 16; ++r) u[r] = twmul<DIR>(u[r], tr[r - 1]);
    dft<16, DIR>(u);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = u[r];
}

// The same with the size-M stage tables in LDS (wfft_load_lds).
template <typename T, int DIR, int M>
__device__ __forceinline__ void wave_fft_lds(cx<T> (&v)[16], cx<T>* __restrict__ reg, int j, const cx<T>* st) {
    static_assert(M >= 16 && M <= 1024 && (M & (M - 1)) == 0, "wave transform size");
    wfft_stages<T, DIR, M, 1, true>(v, reg, j, st);
}

}  // namespace pa
