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
#include <type_traits>

#include "conv_kernels.hpp"
#include "wave_fft.hpp"

namespace pa {

constexpr int kN1 = 8192;  // row length of the long classes

template <typename T, int N2> struct P1Geom {
    static constexpr int W = N2 > 1024 ? N2 / 1024 : 1;    // waves per column
    static constexpr int M = N2 > 1024 ? 1024 : N2;        // wave transform size
    static constexpr int G = 1024 / M;                     // columns per wave
    static constexpr int WAVES = (sizeof(T) == 4 && W > 1) ? 16 : 8;
    static constexpr int C = WAVES * G / W;                // columns per workgroup
    static constexpr int THREADS = WAVES * 64;
    static_assert(W <= 2, "column length up to 2048");
    static constexpr bool kPlanes = sizeof(T) == 4 && C == 8;   // bits from the planes of k2_bits
    static_assert(C <= 64 && (C & (C - 1)) == 0, "column block");
};

template <typename T, int N2> struct P3Geom {
    static constexpr int M = N2 / 2;                       // Hermitian half
    static constexpr int G = 1024 / M;
    static constexpr int WAVES = (sizeof(T) == 4 && G == 1) ? 16 : 8;   // >= 128 B row segments
    static constexpr int C = WAVES * G;
    static constexpr int THREADS = WAVES * 64;
    static constexpr int CW = (C + 31) / 32;               // 32-bit words per output row
    static constexpr int SLOTS = (WAVES * kWaveSlots > M * C) ? WAVES * kWaveSlots : M * C;
    // LDS with the stage tables and Hermitian twiddles copied in (the twiddles
    // share space with the output bit array) vs without; copy them only when
    // the workgroups per CU (160 KB of LDS) stay the same.
    static constexpr size_t kBits = (size_t)WAVES * 64 * 4;   // 32 output bits per lane
    static constexpr size_t kHtw = (size_t)M * sizeof(cx<T>);
    static constexpr size_t kBase = (size_t)SLOTS * sizeof(cx<T>) + C * sizeof(T) + 64;
    static constexpr size_t kWithout = kBase + kBits;
    static constexpr size_t kWith = kBase + (kBits > kHtw ? kBits : kHtw) + wfft_lds_entries(M) * sizeof(cx<T>);
    static constexpr bool LDS_TAB = kWith <= 163840 && (163840 / kWith) >= (163840 / kWithout);
    // workgroups per CU that the LDS allows; registers are capped to match
    static constexpr int MIN_WG = (163840 / (LDS_TAB ? kWith : kWithout)) >= 2 ? 2 : 1;
};

// Transposition tile: row k2 of C elements, columns XOR-swizzled by the row.
template <int C> __device__ __forceinline__ int tslot(int k, int f) { return k * C + (f ^ (k & (C - 1))); }

// ------------------------------------------------------------------ FP64 roots
// Four-step twiddles are formed as FP64 products of two-level tables and
// rounded once to the working precision: w_L^e = fa64[e >> fshift] fb64[e & mask].
struct Root64 {
    double re, im;
};
__device__ __forceinline__ Root64 mul64(Root64 a, Root64 b) {
    return Root64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Root64 root64(const cx<double>* __restrict__ fa64, const cx<double>* __restrict__ fb64,
                                         int fshift, uint32_t e) {
    const cx<double> a = fa64[e >> fshift], b = fb64[e & ((1u << fshift) - 1u)];
    return Root64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> rounded(Root64 w) { return cx<T>{(T)w.re, (T)w.im}; }

// XCD-aware workgroup order: the hardware deals consecutive workgroups to the
// 8 XCDs in turn; remap so that each XCD gets a contiguous range of logical
// blocks (neighbouring column blocks of pass 1 share bit words in its L2).
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t b = blockIdx.x, n = gridDim.x;
    return (n & 7u) ? b : (b & 7u) * (n >> 3) + (b >> 3);
}

// ------------------------------------------------------------------ pass 1
// Bit planes.  A pass-1 workgroup of 8 columns needs one byte of key bits and
// one of seed bits from every row of the tile, rows 1 KB apart: read in place,
// each byte costs a cache line on its way to the compute unit, and staging
// them took a fifth of pass 1.  For the FP32 classes with 8 columns per
// workgroup a small kernel first transposes them, coalesced, into two planes
// per tile after the launch's tiles in the workspace: byte cb n2 + r of the
// key plane holds the placed key bits at positions 8 cb + 8192 r .. + 7 (bit
// q: position + q), the seed plane the seed bits there (zero from the window
// end on).  Pass 1 then reads n2 contiguous bytes of each.
template <int N2> struct BitPlanes {
    static constexpr size_t kPlane = (size_t)N2 * (kN1 / 8);
    static constexpr size_t kTile = 2 * kPlane;   // key plane, then seed plane
    template <typename T>
    __device__ static const uint8_t* key(const cx<T>* ws, uint32_t ntiles, uint32_t lt) {
        return reinterpret_cast<const uint8_t*>(ws + (size_t)ntiles * ((size_t)kN1 * N2)) + (size_t)lt * kTile;
    }
};

// 8 x 8 byte transpose: byte c of x[q] moves to byte q of x[c].
__device__ __forceinline__ void transpose8x8(uint64_t (&x)[8]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t a = x[q], b = x[q + 4];
        x[q] = (a & 0xFFFFFFFFull) | (b << 32);
        x[q + 4] = (a >> 32) | (b & 0xFFFFFFFF00000000ull);
    }
    constexpr uint64_t m16 = 0x0000FFFF0000FFFFull, m8 = 0x00FF00FF00FF00FFull;
#pragma unroll
    for (int q = 0; q < 8; q += (q & 1) ? 3 : 1) {   // q = 0, 1, 4, 5
        const uint64_t a = x[q], b = x[q + 2];
        x[q] = (a & m16) | ((b & m16) << 16);
        x[q + 2] = ((a >> 16) & m16) | (b & ~m16);
    }
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        const uint64_t a = x[q], b = x[q + 1];
        x[q] = (a & m8) | ((b & m8) << 8);
        x[q + 1] = ((a >> 8) & m8) | (b & ~m8);
    }
}

// 64-bit extractions for k2_bits, split into the word loads and the shifts,
// so that a thread issues all its loads back to back: both words of every
// extraction are loaded (indices clamped to the array of nw words) and both
// are used whatever the shift, so no load sits behind a branch.  Same results
// as extract_bits / placed_key_bits<64>.
struct Ext64 {
    uint64_t w;     // first word
    uint32_t s;     // bit offset in it
    uint64_t mask;  // cnt low bits
};
__device__ __forceinline__ Ext64 ext64(uint64_t pos, uint32_t cnt) {
    return Ext64{pos >> 6, (uint32_t)(pos & 63), cnt >= 64 ? ~0ull : ((1ull << (cnt & 63)) - 1ull)};
}
__device__ __forceinline__ void ext64_load(const uint64_t* __restrict__ a, uint64_t nw, const Ext64& e,
                                           uint64_t& lo, uint64_t& hi) {
    lo = a[e.w < nw ? e.w : nw - 1];
    hi = a[e.w + 1 < nw ? e.w + 1 : nw - 1];
}
__device__ __forceinline__ uint64_t ext64_value(const Ext64& e, uint64_t lo, uint64_t hi) {
    return ((lo >> e.s) | ((hi << 1) << (63 - e.s))) & e.mask;   // s = 0: hi drops out
}
// The two extractions of the placed key bits at positions s0 .. s0 + 63
// (position t holds key bit j0 + ((t + bi - 1) mod L) when that index is < bi):
// the positions before the wrap to u = 0, then those after it, shifted by fs.
struct PlacedKey64 {
    Ext64 e1, e2;
    uint32_t fs;
};
__device__ __forceinline__ PlacedKey64 placed_key64(uint64_t j0, uint32_t bi, uint32_t L, uint32_t s0) {
    uint32_t u0 = s0 + bi - 1;
    if (u0 >= L) u0 -= L;
    const uint32_t fs = u0 + 64 <= L ? 64u : L - u0;
    const uint32_t c1 = u0 < bi ? (bi - u0 < fs ? bi - u0 : fs) : 0u;
    const uint32_t c2 = fs < 64 ? (bi < 64 - fs ? bi : 64 - fs) : 0u;
    return PlacedKey64{ext64(j0 + u0, c1), ext64(j0, c2), fs & 63u};   // c2 = 0 when fs = 64
}

// Workgroup: 128 rows x 8 word columns (64 positions each) of one tile, both
// planes, 256 threads.  Loads: 8 consecutive lanes take 8 consecutive words
// of one row (64 contiguous bytes of key or seed), 4 rows per lane, every
// load of a lane issued before the first wait.  The words go to LDS; then
// each lane of one half of the workgroup (key plane, seed plane) reads the
// word column of 8 consecutive rows, transposes the 8 x 8 bytes and stores
// one 64-bit word (8 rows) per byte column, so that 16 consecutive lanes write
// one whole 128-byte line.
constexpr int kBitsRows = 128, kBitsCols = 8;
// LDS slot of (row r, word w): bits 3..4 of r permute the rows within each
// 256-byte bank span and bits 3..5 of r are XOR-ed into the word, so that both
// the row-wise writes and the column-wise reads of 64 lanes touch every bank
// pair at most twice.
__device__ __forceinline__ int bits_slot(int r, int w) {
    return (r ^ ((r >> 3) & 3)) * kBitsCols + (w ^ ((r >> 3) & 7));
}
template <int N2>
__global__ void __launch_bounds__(256) k2_bits(JobTable jt, uint8_t* __restrict__ planes) {
    constexpr int R = kBitsRows, WC = kBitsCols, RPL = R * WC / 256;   // rows per lane
    constexpr int NRB = N2 / R, NWB = kN1 / 64 / WC;
    constexpr uint32_t L = (uint32_t)kN1 * N2;
    static_assert(N2 % R == 0 && (kN1 / 64) % WC == 0 && RPL == 4 && WC * 16 * 2 == 256, "workgroup block");
    __shared__ uint64_t wbits[2][R * WC];   // key words, seed words
    const uint32_t b = blockIdx.x;
    const uint32_t lt = b / (NRB * NWB), rem = b % (NRB * NWB);
    const uint32_t rb = rem / NWB, wb = rem % NWB;
    const uint32_t t = jt.tile0 + lt;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const uint32_t bi = (uint32_t)g.bi, win = (uint32_t)(g.bi + g.bo - 1);
    const uint64_t nkw = (jd.n + 63) >> 6, nsw = (jd.n + jd.m - 1 + 63) >> 6;   // key and seed words
    const int tid = threadIdx.x;
    {
        const int wl = tid & (WC - 1);
        const uint32_t wc = wb * WC + (uint32_t)wl;
        PlacedKey64 pk[RPL];
        Ext64 se[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int rl = tid / WC + (256 / WC) * q;
            const uint32_t s0 = wc * 64 + (uint32_t)kN1 * (rb * R + (uint32_t)rl);
            pk[q] = placed_key64(g.j0, bi, L, s0);
            const uint32_t nv = s0 < win ? ((win - s0) < 64u ? (win - s0) : 64u) : 0u;
            se[q] = ext64(g.sigma + s0, nv);
        }
        uint64_t kw[RPL][4], sw[RPL][2];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            ext64_load(jd.key, nkw, pk[q].e1, kw[q][0], kw[q][1]);
            ext64_load(jd.key, nkw, pk[q].e2, kw[q][2], kw[q][3]);
            ext64_load(jd.seed, nsw, se[q], sw[q][0], sw[q][1]);
        }
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int sl = bits_slot(tid / WC + (256 / WC) * q, wl);
            wbits[0][sl] = ext64_value(pk[q].e1, kw[q][0], kw[q][1]) |
                           (ext64_value(pk[q].e2, kw[q][2], kw[q][3]) << pk[q].fs);
            wbits[1][sl] = ext64_value(se[q], sw[q][0], sw[q][1]);
        }
    }
    __syncthreads();
    const int pl = tid >> 7, p = tid & 15, wl = (tid >> 4) & (WC - 1);   // plane, rows 8 p .. 8 p + 7, word
    uint64_t x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = wbits[pl][bits_slot(8 * p + i, wl)];
    transpose8x8(x);
    uint8_t* dst = planes + (size_t)lt * BitPlanes<N2>::kTile + (size_t)pl * BitPlanes<N2>::kPlane +
                   (size_t)((wb * WC + (uint32_t)wl) * 8) * N2 + rb * R + 8 * p;
#pragma unroll
    for (int c = 0; c < 8; ++c) *reinterpret_cast<uint64_t*>(dst + (size_t)c * N2) = x[c];
}

template <typename T, int N2>
__global__ void __launch_bounds__((P1Geom<T, N2>::THREADS))
k2_pass1(JobTable jt, cx<T>* __restrict__ ws, uint32_t* __restrict__ part, const cx<T>* __restrict__ tw,
         const cx<T>* __restrict__ stw, const cx<double>* __restrict__ fa64, const cx<double>* __restrict__ fb64,
         int fshift) {
    using Gm = P1Geom<T, N2>;
    constexpr int C = Gm::C, G = Gm::G, W = Gm::W, M = Gm::M, NJ = M / 16;
    constexpr uint32_t L = (uint32_t)kN1 * N2;
    constexpr int NCB = kN1 / C;
    constexpr int SLOTS = (Gm::WAVES * kWaveSlots > N2 * C) ? Gm::WAVES * kWaveSlots : N2 * C;
    static_assert(2 * N2 * sizeof(uint64_t) <= SLOTS * sizeof(cx<T>), "bit rows fit the LDS union");
    static_assert(G * 16 * sizeof(Root64) <= kWaveSlots * sizeof(cx<T>), "twiddle factors fit a wave region");
    __shared__ __align__(16) cx<T> lds[SLOTS];
    __shared__ __align__(16) cx<T> st[wfft_lds_entries(M)];
    __shared__ uint32_t wsum;
    uint64_t* kbits = reinterpret_cast<uint64_t*>(lds);   // consumed before the wave regions are used
    uint64_t* sbits = kbits + N2;

    const uint32_t blk = xcd_block();
    const uint32_t lt = blk / NCB;
    const uint32_t cb = blk % NCB;
    const uint32_t t = jt.tile0 + lt;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const int tid = threadIdx.x;
    const uint32_t bi = (uint32_t)g.bi, win = (uint32_t)(g.bi + g.bo - 1);
    if (tid == 0) wsum = 0;
    clear_window(g, cb, NCB, tid, Gm::THREADS);
    wfft_load_lds<T, M>(st, stw, tid, Gm::THREADS);
    __syncthreads();

    // stage the bits of this workgroup's C columns: rows r = tid + q * THREADS
    constexpr int RPT = (N2 + Gm::THREADS - 1) / Gm::THREADS;
    uint32_t pc = 0;
    uint64_t kb[RPT], sb[RPT];
    constexpr bool kPlanes = Gm::kPlanes;
    const uint8_t* kp = nullptr;
    if constexpr (kPlanes) kp = BitPlanes<N2>::key(ws, jt.ntiles, lt) + (size_t)cb * N2;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = tid + q * Gm::THREADS;
        kb[q] = 0;
        sb[q] = 0;
        if (r < N2) {
            if constexpr (kPlanes) {
                kb[q] = kp[r];
                sb[q] = kp[BitPlanes<N2>::kPlane + r];
            } else {
                const uint32_t s0 = cb * C + (uint32_t)kN1 * (uint32_t)r;
                kb[q] = placed_key_bits<C>(jd.key, g.j0, bi, L, s0);
                const uint32_t nv = s0 < win ? ((win - s0) < (uint32_t)C ? (win - s0) : (uint32_t)C) : 0u;
                sb[q] = extract_bits(jd.seed, g.sigma + s0, nv);
            }
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
    int f, ka = 0, j, grp;
    if constexpr (W == 1) {
        grp = l / NJ;
        j = l % NJ;
        f = wv * G + grp;
    } else {
        f = wv / W;
        ka = wv % W;
        j = l;
        grp = 0;
    }
    const uint32_t t1 = cb * C + (uint32_t)f;
    // Four-step twiddle w_L^{t1 k2} = base * c_i with
    //   W = 1: k2 = j + NJ i,           base = w_L^{t1 j},          c_i = w_L^{NJ t1 i}
    //   W = 2: k2 = 2 (j + 64 i) + ka,  base = w_L^{t1 (2 j + ka)}, c_i = w_L^{128 t1 i}
    // Each lane fetches its share of its group's 16 factors now (latency hidden
    // behind the transform); they are exchanged through LDS afterwards.
    constexpr int LPG = W == 1 ? NJ : 64;            // lanes per transform group
    constexpr int CPL = (16 + LPG - 1) / LPG;        // factors fetched per lane
    constexpr uint32_t CSTEP = W == 1 ? (uint32_t)NJ : 128u;
    const Root64 base = root64(fa64, fb64, fshift, W == 1 ? t1 * (uint32_t)j : t1 * (uint32_t)(2 * j + ka));
    Root64 cf[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int i = j + q * LPG;
        cf[q] = root64(fa64, fb64, fshift, i < 16 ? CSTEP * t1 * (uint32_t)i : 0u);
    }
    // bit f of row r from the 32-bit half holding it (unconditional reads, selects)
    const uint32_t* __restrict__ kb32 = reinterpret_cast<const uint32_t*>(kbits) + (f >> 5);
    const uint32_t* __restrict__ sb32 = reinterpret_cast<const uint32_t*>(sbits) + (f >> 5);
    const uint32_t fs = (uint32_t)f & 31u;
    auto z = [&](int r) -> cx<T> {
        const uint32_t kw = kb32[2 * r], sw = sb32[2 * r];
        const T xb = ((kw >> fs) & 1u) ? T(1) : T(0);
        const T sv = ((sw >> fs) & 1u) ? T(1) : T(-1);
        const T wb = (t1 + (uint32_t)kN1 * (uint32_t)r < win) ? sv : T(0);
        return cx<T>{xb, wb};
    };
    cx<T> v[16];
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
    cx<T>* reg = lds + wv * kWaveSlots + (W == 1 ? grp * (M + M / 16) : 0);
    wave_fft_lds<T, -1, M>(v, reg, j, st);

    // exchange the factors through this wave's own region (its transform is done)
    Root64* cw = reinterpret_cast<Root64*>(lds + wv * kWaveSlots) + grp * 16;
    wave_sync();
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int i = j + q * LPG;
        if (i < 16) cw[i] = cf[q];
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = cmul(v[i], rounded<T>(mul64(base, cw[i])));
    __syncthreads();
    // transpose through LDS for row-segment stores.  With W = 2 the rows
    // k2 = 2 e + ka of each half go to a tile of their own (the second one 8
    // slots further, off the first's banks), so that a wave writes
    // consecutive rows e as in the W = 1 layout
    constexpr int HALF = M * C + 8;
    static_assert(W * HALF <= SLOTS, "transposition tiles fit the LDS union");
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = j + i * NJ;
        lds[ka * HALF + tslot<C>(e, f)] = v[i];
    }
    __syncthreads();
    cx<T>* __restrict__ Y = ws + (size_t)lt * L;
    static_assert((N2 * C) % Gm::THREADS == 0, "store tile");
    constexpr int SPT = N2 * C / Gm::THREADS;
    cx<T> o[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int idx = tid + q * Gm::THREADS, k2 = idx / C;
        o[q] = lds[(k2 % W) * HALF + tslot<C>(k2 / W, idx % C)];
    }
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int idx = tid + q * Gm::THREADS;
        Y[(size_t)(idx / C) * kN1 + cb * C + (idx % C)] = o[q];
    }
    if (tid == 0) part[(size_t)lt * NCB + cb] = wsum;
}

// Pass 1 for FP32 columns of 2048 points, as two halves.  Half ka (outputs
// k2 = 2 e + ka) is the 1024-point transform of z(e) + z(e + 1024) (ka = 0) or
// (z(e) - z(e + 1024)) w_2048^e (ka = 1): a radix-2 split in decimation in
// frequency.  A workgroup of eight waves takes one half of 8 columns (one
// column per wave), so it needs the LDS of one half (the block's bits, then
// the wave regions, then the transposition tile: 78 KB, two workgroups per
// CU) and the registers of one 1024-point column; the two halves of a column
// block read the same bit-plane bytes.
struct P1hArgs {
    JobDesc jd;
    TileGeo g;
    uint32_t lt, cb, ntiles;
};

template <typename T, int KA>
__device__ __forceinline__ uint32_t pass1_half_body(const P1hArgs& A, cx<T>* __restrict__ ws, cx<T>* lds,
                                                    const cx<T>* st, const cx<T>* __restrict__ tw,
                                                    const cx<double>* __restrict__ fa64,
                                                    const cx<double>* __restrict__ fb64, int fshift) {
    constexpr int N2 = 2048, M = 1024, C = 8, THREADS = 512, NJ = M / 16;
    constexpr uint32_t L = (uint32_t)kN1 * N2;
    const int tid = threadIdx.x, wv = tid >> 6, j = tid & 63;
    const TileGeo& g = A.g;
    const uint32_t bi = (uint32_t)g.bi, win = (uint32_t)(g.bi + g.bo - 1);
    const int f = wv;   // this wave's column
    const uint32_t t1 = A.cb * C + (uint32_t)f;
    uint16_t* fld = reinterpret_cast<uint16_t*>(lds);   // per row: key bits (low byte), seed bits (high byte)
    uint32_t pc = 0;
    __syncthreads();   // the previous half's stores have read the LDS
    const uint8_t* kp = BitPlanes<N2>::key(ws, A.ntiles, A.lt) + (size_t)A.cb * N2;
    for (int r = tid; r < N2; r += THREADS) {
        const uint32_t kb = kp[r];
        const uint32_t sb = kp[BitPlanes<N2>::kPlane + r];
        fld[r] = (uint16_t)(kb | (sb << 8));
        pc += (uint32_t)__popc(kb);
    }
    __syncthreads();
    // four-step twiddle w_L^{t1 k2}, k2 = 2 (j + 64 i) + KA: base w_L^{t1 (2 j + KA)}
    // times c_i = w_L^{128 t1 i} (lane i < 16 fetches c_i; exchanged after the transform)
    const Root64 base = root64(fa64, fb64, fshift, t1 * (uint32_t)(2 * j + KA));
    const Root64 cf = root64(fa64, fb64, fshift, j < 16 ? 128u * t1 * (uint32_t)j : 0u);
    auto z = [&](int r) -> cx<T> {
        const uint32_t w = fld[r];
        const T xb = ((w >> f) & 1u) ? T(1) : T(0);
        const T sv = ((w >> (8 + f)) & 1u) ? T(1) : T(-1);
        return cx<T>{xb, (t1 + (uint32_t)kN1 * (uint32_t)r < win) ? sv : T(0)};
    };
    cx<T> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = j + i * NJ;
        const cx<T> a = z(e), b = z(e + M);
        if constexpr (KA == 0) v[i] = a + b;
        else v[i] = cmul(a - b, tw[e * (kN1 / N2)]);
    }
    __syncthreads();   // bits consumed; LDS becomes wave regions
    cx<T>* reg = lds + wv * kWaveSlots;
    wave_fft_lds<T, -1, M>(v, reg, j, st);
    Root64* cw = reinterpret_cast<Root64*>(reg);
    wave_sync();
    if (j < 16) cw[j] = cf;
    wave_sync();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = cmul(v[i], rounded<T>(mul64(base, cw[i])));
    __syncthreads();
    // transpose through LDS for row-segment stores (rows k2 = 2 e + KA)
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[tslot<C>(j + i * NJ, f)] = v[i];
    __syncthreads();
    cx<T>* __restrict__ Y = ws + (size_t)A.lt * L;
    constexpr int SPT = M * C / THREADS;
    cx<T> o[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int idx = tid + q * THREADS;
        o[q] = lds[tslot<C>(idx / C, idx % C)];
    }
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int idx = tid + q * THREADS;
        Y[(size_t)(2 * (idx / C) + KA) * kN1 + A.cb * C + (idx % C)] = o[q];
    }
    return pc;
}

// Each half in a workgroup of its own: logical block 2 b + KA
// takes half KA of column block b (the two read the same bit words, through
// the L2 of one XCD).  Half 0 clears the window and reports the weight.
template <typename T>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k2_pass1s(JobTable jt, cx<T>* __restrict__ ws, uint32_t* __restrict__ part, const cx<T>* __restrict__ tw,
          const cx<T>* __restrict__ stw, const cx<double>* __restrict__ fa64, const cx<double>* __restrict__ fb64,
          int fshift) {
    constexpr int M = 1024, C = 8, THREADS = 512;
    constexpr int NCB = kN1 / C;
    constexpr int SLOTS = 8 * kWaveSlots;
    static_assert(M * C <= SLOTS && 2048 * (int)sizeof(uint16_t) <= SLOTS * (int)sizeof(cx<T>), "LDS union");
    __shared__ __align__(16) cx<T> lds[SLOTS];
    __shared__ __align__(16) cx<T> st[wfft_lds_entries(M)];
    __shared__ uint32_t wsum;
    const uint32_t blk = xcd_block();
    const uint32_t lb = blk >> 1;
    const bool second = (blk & 1u) != 0;
    P1hArgs A;
    A.lt = lb / NCB;
    A.cb = lb % NCB;
    A.ntiles = jt.ntiles;
    const uint32_t t = jt.tile0 + A.lt;
    A.jd = find_job(jt, t);
    A.g = tile_geo(A.jd, t - A.jd.tile_begin);
    const int tid = threadIdx.x;
    if (tid == 0) wsum = 0;
    if (!second) clear_window(A.g, A.cb, NCB, tid, THREADS);
    wfft_load_lds<T, M>(st, stw, tid, THREADS);
    if (second) {
        (void)pass1_half_body<T, 1>(A, ws, lds, st, tw, fa64, fb64, fshift);
        return;
    }
    const uint32_t pc = pass1_half_body<T, 0>(A, ws, lds, st, tw, fa64, fb64, fshift);
    atomicAdd(&wsum, pc);
    __syncthreads();
    if (tid == 0) part[(size_t)A.lt * NCB + A.cb] = wsum;
}

// ------------------------------------------------------------------ pass 2
// Shared memory of the row pass: the row exchange / wave regions, the stage
// tables of the 1024-point transforms, and the first-stage twiddles
// w_8192^{ka nb}, ka = 1..7: FP32 holds them all, t8[(ka-1) 1024 + nb]; FP64,
// whose row region leaves no room for that, forms them as the product of two
// short tables, w_8192^e = w8a[e >> 6] w8b[e & 63] (135.7 KB for FP32, 156 KB
// for FP64).
template <typename T> struct RowSmem {
    static constexpr bool kLds = sizeof(T) == 4;   // the full first-stage table (FP32 only)
    cx<T> data[8 * kWaveSlots];
    cx<T> st[wfft_lds_entries(1024)];
    cx<T> t8[kLds ? 7 * 1024 : 1];
    cx<T> w8a[kLds ? 1 : 128];
    cx<T> w8b[kLds ? 1 : 64];
};

// FP32: thread tid writes t8 entries e = tid (mod 512) and the forward
// transform's thread tid reads only such entries (nb = tid + 512 s), so the
// first unit needs no barrier after this load; the stage tables are first
// read after one.  FP64 reads w8a / w8b entries other threads wrote: the
// kernel waits at a barrier after this load.
template <typename T>
__device__ __forceinline__ void row_smem_load(RowSmem<T>& S, const cx<T>* __restrict__ tw,
                                              const cx<T>* __restrict__ stw, int tid) {
    wfft_load_lds<T, 1024>(S.st, stw, tid, 512);
    if constexpr (RowSmem<T>::kLds) {
        for (int e = tid; e < 7 * 1024; e += 512) S.t8[e] = tw[(1 + e / 1024) * (e % 1024)];
    } else {
        if (tid < 128) S.w8a[tid] = tw[64 * tid];
        if (tid < 64) S.w8b[tid] = tw[tid];
    }
}

// Last-stage twiddles of the 1024-point transform held in registers for the
// whole row pass (FP32): w_1024^{l r}, r = 1..15.
template <typename T> struct RowReg {
    cx<T> tr[RowSmem<T>::kLds ? 15 : 1];
};

// 1024-point wave transform of the row pass, stage tables from LDS (FP32:
// the last stage's from registers)
template <typename T, int DIR>
__device__ __forceinline__ void row_wave_fft(cx<T> (&v)[16], cx<T>* __restrict__ reg, int l, const RowSmem<T>& S,
                                             const RowReg<T>& R, const cx<T>* __restrict__ stw) {
    (void)stw;
    if constexpr (RowSmem<T>::kLds) wave_fft1024_lds_reg<T, DIR>(v, reg, l, S.st, R.tr);
    else wave_fft_lds<T, DIR, 1024>(v, reg, l, S.st);
}

// w_8192^{ka nb}, 1 <= ka < 8, nb < 1024
template <typename T>
__device__ __forceinline__ cx<T> w8192(const RowSmem<T>& S, const cx<T>* __restrict__ tw, int ka, int nb) {
    if constexpr (RowSmem<T>::kLds) {
        return S.t8[(ka - 1) * 1024 + nb];
    } else {
        const int e = ka * nb;   // < 7168
        return cmul(S.w8a[e >> 6], S.w8b[e & 63]);
    }
}

template <typename T>
__device__ __forceinline__ void row_load(cx<T> (&a)[16], const cx<T>* __restrict__ row, int wv, int l) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int nb = wv * 64 + l + 512 * s;
#pragma unroll
        for (int na = 0; na < 8; ++na) a[s * 8 + na] = row[nb + 1024 * na];
    }
}

// Forward transform of one 8192-point row loaded by row_load (a is consumed).
// Thread (wave w, lane l) ends with X[8 k_b + w] in register i, k_b = l + 64 i.
template <typename T>
__device__ __forceinline__ void row_forward(cx<T> (&a)[16], cx<T> (&X)[16], RowSmem<T>& S, const RowReg<T>& R,
                                            int wv, int l, const cx<T>* __restrict__ tw,
                                            const cx<T>* __restrict__ stw) {
    constexpr int SS = kWaveSlots;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int nb = wv * 64 + l + 512 * s;
        dft8<-1>(&a[s * 8]);
#pragma unroll
        for (int ka = 1; ka < 8; ++ka) a[s * 8 + ka] = cmul(a[s * 8 + ka], w8192<T>(S, tw, ka, nb));
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int nb = wv * 64 + l + 512 * s;
#pragma unroll
        for (int ka = 0; ka < 8; ++ka) S.data[ka * SS + wslot(nb)] = a[s * 8 + ka];
    }
    __syncthreads();
    cx<T>* reg = S.data + wv * SS;
#pragma unroll
    for (int i = 0; i < 16; ++i) X[i] = reg[wslot(l + 64 * i)];
    wave_sync();
    row_wave_fft<T, -1>(X, reg, l, S, R, stw);
}

// Inverse transform of a row held as P[8 k_b + w] (register i, k_b = l + 64 i);
// returns a[t_b + 1024 t_a] in a[s * 8 + t_a] for t_b = w * 64 + l + 512 s.
template <typename T>
__device__ __forceinline__ void row_inverse(cx<T> (&P)[16], cx<T> (&a)[16], RowSmem<T>& S, const RowReg<T>& R,
                                            int wv, int l, const cx<T>* __restrict__ tw,
                                            const cx<T>* __restrict__ stw) {
    constexpr int SS = kWaveSlots;
    cx<T>* reg = S.data + wv * SS;
    __syncthreads();  // every wave is done with its region
    row_wave_fft<T, +1>(P, reg, l, S, R, stw);
    if (wv > 0) {
#pragma unroll
        for (int i = 0; i < 16; ++i) P[i] = cmulc(P[i], w8192<T>(S, tw, wv, l + 64 * i));
    }
    wave_sync();   // the wave's own region: no other wave uses it until the barrier below
#pragma unroll
    for (int i = 0; i < 16; ++i) reg[wslot(l + 64 * i)] = P[i];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int tb = wv * 64 + l + 512 * s;
#pragma unroll
        for (int ka = 0; ka < 8; ++ka) a[s * 8 + ka] = S.data[ka * SS + wslot(tb)];
        dft8<+1>(&a[s * 8]);
    }
}

// Replace X (row layout of row_forward) by the values at the mirrored
// frequency: -k mod 8192 when `zero`, else 8191 - k.
template <typename T>
__device__ __forceinline__ void row_mirror(cx<T> (&X)[16], cx<T>* lds, int wv, int l, bool zero) {
    constexpr int S = kWaveSlots;
    wave_sync();   // X was produced in the wave's own region, which no other wave touches
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

// Store V row `row` (inverse four-step twiddle w_L^{-row t1}): t1 = x + 1024 ta
// with x = w 64 + l + 512 s, so w_L^{row t1} = w_L^{row x} w_L^{1024 row ta},
// an FP64 product rounded once.  `real`: keep the real part only.
template <typename T>
__device__ __forceinline__ void row_store(cx<T>* __restrict__ Yrow, cx<T> (&a)[16], uint32_t row, bool real,
                                          int wv, int l, const cx<double>* __restrict__ fa64,
                                          const cx<double>* __restrict__ fb64, int fshift) {
    if constexpr (sizeof(T) == 8) {
        // FP64 (register-bound): one table product per point
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int ta = 0; ta < 8; ++ta) {
                const uint32_t t1 = (uint32_t)(wv * 64 + l + 512 * s + 1024 * ta);
                cx<T> vv = cmulc(a[s * 8 + ta], rounded<T>(root64(fa64, fb64, fshift, row * t1)));
                if (real) vv.im = T(0);
                Yrow[t1] = vv;
            }
        return;
    }
    Root64 b[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) b[s] = root64(fa64, fb64, fshift, row * (uint32_t)(wv * 64 + l + 512 * s));
#pragma unroll
    for (int ta = 0; ta < 8; ++ta) {
        const Root64 c = root64(fa64, fb64, fshift, 1024u * row * (uint32_t)ta);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const uint32_t x = (uint32_t)(wv * 64 + l + 512 * s);
            cx<T> vv = cmulc(a[s * 8 + ta], rounded<T>(mul64(b[s], c)));
            if (real) vv.im = T(0);
            Yrow[x + 1024u * (uint32_t)ta] = vv;
        }
    }
}

// Row pass over units: units 0 .. ntiles (n2/2 - 1) - 1 are mirror pairs (row
// pr >= 1 with n2 - pr), the last ntiles units the self rows 0 and n2/2 of
// each tile.  The pass is persistent: workgroup b walks u = b, b + G, ...,
// G = one workgroup per CU (LDS-bound), tables loaded once.
template <typename T> constexpr bool kRowPersistent = sizeof(T) == 4;
// One unit of the row pass.
template <typename T, int N2, int NCB1>
__device__ __forceinline__ void row_unit(uint32_t u, const JobTable& jt, cx<T>* __restrict__ ws,
                                         const uint32_t* __restrict__ part, TileMeta* __restrict__ meta,
                                         RowSmem<T>& S, const RowReg<T>& R, uint32_t& wsum,
                                         const cx<T>* __restrict__ tw,
                                         const cx<T>* __restrict__ stw, const cx<double>* __restrict__ fa64,
                                         const cx<double>* __restrict__ fb64, int fshift) {
    constexpr uint32_t L = (uint32_t)kN1 * N2;
    constexpr int NP = N2 / 2;
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const T quarter = T(0.25) / T(L);
    const uint32_t npairs = jt.ntiles * (uint32_t)(NP - 1);
    const bool pair = u < npairs;
    const uint32_t lt = pair ? u / (uint32_t)(NP - 1) : u - npairs;
    const uint32_t pr = pair ? 1u + u % (uint32_t)(NP - 1) : 0u;
    cx<T>* __restrict__ Y = ws + (size_t)lt * L;
    if (pair) {
        // FP32 issues the second row's loads before the first transform;
        // FP64 has no registers to spare for that
        constexpr bool kHoist = sizeof(T) == 4;
        cx<T> ra[16], rb[16], A[16], B[16], a[16];
        row_load<T>(ra, Y + (size_t)pr * kN1, wv, l);
        if constexpr (kHoist) row_load<T>(rb, Y + (size_t)(N2 - pr) * kN1, wv, l);
        row_forward<T>(ra, A, S, R, wv, l, tw, stw);
        if constexpr (!kHoist) row_load<T>(rb, Y + (size_t)(N2 - pr) * kN1, wv, l);
        row_forward<T>(rb, B, S, R, wv, l, tw, stw);
        row_mirror<T>(B, S.data, wv, l, false);
#pragma unroll
        for (int i = 0; i < 16; ++i) A[i] = spectrum_product(A[i], B[i], quarter);
        row_inverse<T>(A, a, S, R, wv, l, tw, stw);
        row_store<T>(Y + (size_t)pr * kN1, a, pr, false, wv, l, fa64, fb64, fshift);
    } else {
        // key-chunk weight from the pass-1 partial sums; reset the certificate
        __syncthreads();
        if (tid == 0) wsum = 0;
        __syncthreads();
        uint32_t sum = 0;
        for (int c = tid; c < NCB1; c += 512) sum += part[(size_t)lt * NCB1 + c];
        atomicAdd(&wsum, sum);
        __syncthreads();
        if (tid == 0) meta[jt.tile0 + lt] = TileMeta{wsum, 0u, 0u, 0u};
        // rows 0 and n2/2 are their own mirrors and their V rows are real:
        // each goes to the real parts of its own row
#pragma nounroll
        for (int v = 0; v < 2; ++v) {
            const uint32_t row = v == 0 ? 0u : (uint32_t)NP;
            cx<T> ra[16], A[16], B[16], a[16];
            row_load<T>(ra, Y + (size_t)row * kN1, wv, l);
            row_forward<T>(ra, A, S, R, wv, l, tw, stw);
#pragma unroll
            for (int i = 0; i < 16; ++i) B[i] = A[i];
            row_mirror<T>(B, S.data, wv, l, v == 0);
#pragma unroll
            for (int i = 0; i < 16; ++i) A[i] = spectrum_product(A[i], B[i], quarter);
            row_inverse<T>(A, a, S, R, wv, l, tw, stw);
            row_store<T>(Y + (size_t)row * kN1, a, row, true, wv, l, fa64, fb64, fshift);
        }
    }
}

template <typename T, int N2, int NCB1>
__global__ void __launch_bounds__(512)
k2_pass2(JobTable jt, cx<T>* __restrict__ ws, const uint32_t* __restrict__ part, TileMeta* __restrict__ meta,
         const cx<T>* __restrict__ tw, const cx<T>* __restrict__ stw, const cx<double>* __restrict__ fa64,
         const cx<double>* __restrict__ fb64, int fshift) {
    __shared__ __align__(16) RowSmem<T> S;
    __shared__ uint32_t wsum;
    const uint32_t units = jt.ntiles * (uint32_t)(N2 / 2);
    row_smem_load<T>(S, tw, stw, threadIdx.x);
    if constexpr (!RowSmem<T>::kLds) __syncthreads();
    RowReg<T> R;
    if constexpr (RowSmem<T>::kLds) {
        // w_1024^{l r} = w_8192^{8 l r}, l r < 1024
        const int l = threadIdx.x & 63;
#pragma unroll
        for (int r = 1; r < 16; ++r) R.tr[r - 1] = tw[8 * l * r];
    }
    if constexpr (kRowPersistent<T>) {
        for (uint32_t u = blockIdx.x; u < units; u += gridDim.x)
            row_unit<T, N2, NCB1>(u, jt, ws, part, meta, S, R, wsum, tw, stw, fa64, fb64, fshift);
    } else {
        if (blockIdx.x < units)
            row_unit<T, N2, NCB1>(blockIdx.x, jt, ws, part, meta, S, R, wsum, tw, stw, fa64, fb64, fshift);
    }
}

// ------------------------------------------------------------------ pass 3
// rint(z) mod 4 for an integral r (FP32: |r| < 2^31; FP64: |r| < 2^51)
__device__ __forceinline__ uint32_t low2(float r) { return (uint32_t)(int)r & 3u; }
__device__ __forceinline__ uint32_t low2(double r) {
    const double q = r * 0.25;
    return (uint32_t)(int)((q - floor(q)) * 4.0) & 3u;
}

template <typename T, int N2>
__global__ void __launch_bounds__((P3Geom<T, N2>::THREADS))
__attribute__((amdgpu_waves_per_eu(P3Geom<T, N2>::MIN_WG * P3Geom<T, N2>::WAVES / 4)))
k2_pass3(JobTable jt, const cx<T>* __restrict__ ws, TileMeta* __restrict__ meta, const cx<T>* __restrict__ tw,
         const cx<T>* __restrict__ stw) {
    using Gm = P3Geom<T, N2>;
    constexpr int C = Gm::C, G = Gm::G, M = Gm::M, NJ = M / 16, CW = Gm::CW;
    constexpr uint32_t L = (uint32_t)kN1 * N2;
    constexpr int NCB = kN1 / C;
    constexpr bool LT = Gm::LDS_TAB;
    constexpr int NHT = LT ? M : 1;
    constexpr int NLB = Gm::WAVES * 64;
    __shared__ __align__(16) cx<T> lds[Gm::SLOTS];
    __shared__ __align__(16) cx<T> st[LT ? wfft_lds_entries(M) : 1];
    // Hermitian twiddles w_n2^k (k < n2/2) until the transform, then the
    // output bits of each lane: bit 2 i + e of lbits[w * 64 + g NJ + j] is the
    // output of column w G + g, row 2 (j + NJ i) + e
    __shared__ __align__(16) union {
        cx<T> htw[NHT];
        uint32_t lbits[NLB];
    } U;
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
        if constexpr (LT) {
            wfft_load_lds<T, M>(st, stw, tid, Gm::THREADS);
            for (int k = tid; k < M; k += Gm::THREADS) U.htw[k] = tw[k * (kN1 / N2)];
        }
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
            const cx<T> wk = LT ? U.htw[k] : tw[k * (kN1 / N2)];
            const cx<T> o = cmulc(h - hm, wk);
            v[i] = cx<T>{e.re - o.im, e.im + o.re};
        }
    }
    __syncthreads();  // tile (and twiddles) consumed; LDS becomes wave regions
    cx<T>* reg = lds + wv * kWaveSlots + gg * (M + M / 16);
    if constexpr (LT) wave_fft_lds<T, +1, M>(v, reg, j, st);
    else wave_fft<T, +1, M>(v, reg, j, stw);

    // window, exact rounding and parity (branch-free): only the low two bits
    // of rint(z) + weight matter, bit = bit 1, parity check = bit 0
    const uint32_t wlow = meta[t].popcnt & 3u;
    const uint32_t bo = (uint32_t)g.bo;
    const uint32_t rows = (bo + (uint32_t)kN1 - 1u) / (uint32_t)kN1;  // rows t2 holding outputs
    float mres = 0.f, mabs = 0.f;
    uint32_t bad = 0;
    uint32_t mybits = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (2u * (uint32_t)(i * NJ) >= rows) continue;   // register i holds no output row (uniform)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t t2 = 2u * (uint32_t)(j + i * NJ) + (uint32_t)e;
            const bool valid = t1 + (uint32_t)kN1 * t2 < bo;
            const T zz = e ? v[i].im : v[i].re;
            const T r = round_even(zz);
            const uint32_t s2 = low2(r) + wlow;
            // an odd sum, or a non-finite z (fmaxf below would drop a NaN)
            bad += (valid && ((s2 & 1u) || !(fabs(zz - r) <= T(0.5)))) ? 1u : 0u;
            mres = fmaxf(mres, valid ? (float)fabs(zz - r) : 0.f);
            mabs = fmaxf(mabs, valid ? (float)fabs(zz) : 0.f);
            mybits |= (valid ? ((s2 >> 1) & 1u) : 0u) << (2 * i + e);
        }
    }
    U.lbits[wv * 64 + l] = mybits;
    atomicMax(&s_res, __float_as_uint(mres));
    atomicMax(&s_abs, __float_as_uint(mabs));
    atomicAdd(&s_bad, bad);
    __syncthreads();
    // assemble and store each output row's C bits (32 per word, C < 32: one C-bit group)
    constexpr int WB = C < 32 ? C : 32;    // bits per stored word
    const uint64_t limit = g.dst_words * 64u;
    for (uint32_t idx = tid; idx < rows * CW; idx += Gm::THREADS) {
        const uint32_t t2 = idx / CW, c = idx % CW;
        const uint32_t k = t2 >> 1, sh = 2u * (k / NJ) + (t2 & 1u), jj = k % NJ;
        uint32_t word = 0;
#pragma unroll
        for (int q = 0; q < WB; ++q) {
            const int col = 32 * (int)c + q;
            word |= ((U.lbits[(col / G) * 64 + (col % G) * NJ + jj] >> sh) & 1u) << q;
        }
        const uint64_t off = (uint64_t)cb * C + 32u * c + (uint64_t)kN1 * t2;
        if (off >= limit) continue;
        put_bits<WB>(g, off, word);
    }
    if (tid == 0) {
        atomicMax(&meta[t].maxres, s_res);
        atomicMax(&meta[t].maxabs, s_abs);
        if (s_bad) atomicAdd(&meta[t].badpar, s_bad);
    }
}

// Workgroups of the persistent row pass: one per compute unit (LDS-bound).
int row_pass_workgroups();

template <typename T, int N2>
struct ClassImpl2 {
    using G1 = P1Geom<T, N2>;
    using G3 = P3Geom<T, N2>;
    static constexpr int C1 = G1::C, C3 = G3::C;
    // workspace bytes per tile beyond its points: the bit planes
    static constexpr size_t kWsExtra = G1::kPlanes ? BitPlanes<N2>::kTile : 0;
    static int pass1(const JobTable& jt, void* ws, uint32_t* part, TileMeta*, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (kN1 / C1)), block(G1::THREADS);
        if constexpr (G1::kPlanes) {
            uint8_t* planes = reinterpret_cast<uint8_t*>((cx<T>*)ws + (size_t)jt.ntiles * ((size_t)kN1 * N2));
            hipLaunchKernelGGL((k2_bits<N2>), dim3(jt.ntiles * (N2 / kBitsRows) * (kN1 / 64 / kBitsCols)), dim3(256), 0,
                               (hipStream_t)stream, jt, planes);
        }
        if constexpr (sizeof(T) == 4 && N2 == 2048) {
            static_assert(C1 == 8, "eight columns per workgroup");
            hipLaunchKernelGGL((k2_pass1s<T>), dim3(2 * grid.x), dim3(512), 0, (hipStream_t)stream, jt, (cx<T>*)ws, part,
                               (const cx<T>*)tb.tw, (const cx<T>*)tb.stw, (const cx<double>*)tb.fa64,
                               (const cx<double>*)tb.fb64, tb.fshift);
        } else {
            hipLaunchKernelGGL((k2_pass1<T, N2>), grid, block, 0, (hipStream_t)stream, jt, (cx<T>*)ws, part,
                               (const cx<T>*)tb.tw, (const cx<T>*)tb.stw, (const cx<double>*)tb.fa64,
                               (const cx<double>*)tb.fb64, tb.fshift);
        }
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass2(const JobTable& jt, void* ws, uint32_t* part, TileMeta* meta, const Tables& tb, void* stream) {
        const uint32_t units = jt.ntiles * (N2 / 2);
        const uint32_t wgs = kRowPersistent<T> ? (uint32_t)row_pass_workgroups() : units;
        dim3 grid(units < wgs ? units : wgs), block(512);
        hipLaunchKernelGGL((k2_pass2<T, N2, kN1 / C1>), grid, block, 0, (hipStream_t)stream, jt, (cx<T>*)ws,
                           (const uint32_t*)part, meta, (const cx<T>*)tb.tw, (const cx<T>*)tb.stw,
                           (const cx<double>*)tb.fa64, (const cx<double>*)tb.fb64, tb.fshift);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass3(const JobTable& jt, void* ws, uint32_t*, TileMeta* meta, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (kN1 / C3)), block(G3::THREADS);
        hipLaunchKernelGGL((k2_pass3<T, N2>), grid, block, 0, (hipStream_t)stream, jt, (const cx<T>*)ws, meta,
                           (const cx<T>*)tb.tw, (const cx<T>*)tb.stw);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
};

// Mixed-radix classes with rows of 8192 (L = 8192 n2, n2 = P 2^b): the
// wave-level row pass above (it does not depend on how n2 factors) between
// the workgroup-wide Stockham column passes of conv_kernels.hpp, whose columns
// carry the radix-P stage (RC points per thread).
template <typename T, int N2, int B1, int B3, int RC>
struct ClassImplS {
    static constexpr int NCB1 = kN1 / B1;
    static int pass1(const JobTable& jt, void* ws, uint32_t* part, TileMeta*, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * NCB1), block(B1 * (N2 / RC));
        hipLaunchKernelGGL((k_pass1<T, kN1, N2, B1, RC, N2>), grid, block, 0, (hipStream_t)stream, jt, (cx<T>*)ws,
                           part, (const cx<T>*)tb.tw2, (const cx<T>*)tb.fa, (const cx<T>*)tb.fb, tb.fshift);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass2(const JobTable& jt, void* ws, uint32_t* part, TileMeta* meta, const Tables& tb, void* stream) {
        const uint32_t units = jt.ntiles * (N2 / 2);
        const uint32_t wgs = kRowPersistent<T> ? (uint32_t)row_pass_workgroups() : units;
        dim3 grid(units < wgs ? units : wgs), block(512);
        hipLaunchKernelGGL((k2_pass2<T, N2, NCB1>), grid, block, 0, (hipStream_t)stream, jt, (cx<T>*)ws,
                           (const uint32_t*)part, meta, (const cx<T>*)tb.tw, (const cx<T>*)tb.stw,
                           (const cx<double>*)tb.fa64, (const cx<double>*)tb.fb64, tb.fshift);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass3(const JobTable& jt, void* ws, uint32_t*, TileMeta* meta, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (kN1 / B3)), block(B3 * (N2 / 2 / RC));
        hipLaunchKernelGGL((k_pass3<T, kN1, N2, B3, RC, N2, true>), grid, block, 0, (hipStream_t)stream, jt,
                           (const cx<T>*)ws, meta, (const cx<T>*)tb.tw2);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
};

}  // namespace pa
