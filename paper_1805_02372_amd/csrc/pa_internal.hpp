// Shared host/device declarations of libpa (not part of the public ABI).
#pragma once
#include <stdint.h>
#include <stddef.h>

namespace pa {

// One hash job as the kernels see it.  A job is cut into `nchunks` key chunks
// (taken from the top of the key: chunk b covers key bits
// [max(0, n-(b+1)Bi), n-b*Bi)) and `nouts` output windows (window o covers
// outputs [o*Bo, min(m, (o+1)*Bo))); tile (b, o) is local tile b*nouts + o.
// With several chunks the tiles' partial hashes are XOR-accumulated into
// `out` (Eq. 7): pass 1 of the chunk-0 tile clears its window's words, pass 3
// of every tile XORs its bits in.
// Tile (b, o) with chunk start j0, length bi, window start i0, length bo uses
// seed bits [sigma, sigma+bi+bo-1) with sigma = i0 - j0 + n - bi: by the
// constant diagonals of T its outputs are the window [bi-1, bi-1+bo) of the
// convolution of that seed slice with the key chunk (Eq. 4-7, Fig. 1-2).
struct JobDesc {
    const uint64_t* key;
    const uint64_t* seed;
    uint64_t* out;        // m bits
    uint64_t n, m;
    uint64_t Bi, Bo;      // nominal chunk and window lengths (Bo % 64 == 0 if nouts > 1)
    uint32_t nchunks, nouts;
    uint32_t tile_begin;  // first tile of this job in the launch's tile numbering
    uint32_t out_words;   // ceil(m / 64)
    uint32_t no_clear;    // 1: chunk-0 tiles do not clear their window (a tile
                          // re-run that XORs into an accumulated window)
};

// Where the tiles of one launch come from: either one job passed by value or
// an array of jobs (sorted by tile_begin) in device memory.
struct JobTable {
    JobDesc one;
    const JobDesc* many;
    uint32_t njobs;       // 0: use `one`
    uint32_t tile0;       // first tile of this launch (groups of tiles)
    uint32_t ntiles;      // tiles in this launch
    uint32_t clears;      // some job of `many` has a chunk-0 tile that clears its window
};

// Per-tile results of pass 2/3.
struct TileMeta {
    uint32_t popcnt;      // weight of the key chunk
    uint32_t maxres;      // float bits of max |z - rint z|
    uint32_t maxabs;      // float bits of max |z|
    uint32_t badpar;      // outputs whose rounded value had the wrong parity
};

// FFT length classes.  A class is named by an id: log2 L for the power-of-two
// classes (ids 12 .. 24, every precision), and 32 + 3 (k - 12) + (P - 3) / 2
// for the mixed-radix classes L = P 2^k, P = 3, 5, 7, 2^14 < L < 2^24 (FP32
// and FP64 only; radix-P transform stages, section 3 step 1 pads the product
// to an arbitrary length).
constexpr int kMinClassId = 12;
constexpr int kMaxClassId = 63;
constexpr int smooth_id(int P, int k) { return 32 + 3 * (k - 12) + (P - 3) / 2; }
constexpr int smooth_P(int id) { return 3 + 2 * ((id - 32) % 3); }
constexpr int smooth_k(int id) { return 12 + (id - 32) / 3; }
constexpr bool smooth_valid(int id) {
    return id >= 32 && id <= kMaxClassId && ((uint64_t)smooth_P(id) << smooth_k(id)) > (1ull << 14) &&
           ((uint64_t)smooth_P(id) << smooth_k(id)) < (1ull << 24);
}
constexpr bool class_id_valid(int id) { return (id >= 12 && id <= 24) || smooth_valid(id); }
// FFT length of a class id (0 if none).
constexpr uint64_t class_len(int id) {
    return (id >= 12 && id <= 24) ? (1ull << id) : smooth_valid(id) ? ((uint64_t)smooth_P(id) << smooth_k(id)) : 0;
}

// One FFT length class: L = n1 * n2.
struct ClassCfg {
    int prec;             // 32 or 64 (1: NTT)
    int cls;              // class id (above)
    int n1, n2;           // row length (pass 2), column length (pass 1/3)
    int b1, b3;           // columns per workgroup in pass 1 / pass 3
    int r;                // points per thread
    size_t ws_extra = 0;  // workspace bytes per tile beyond its points (pass 1's bit planes)
};

// Device pointers of a class's twiddle tables (element type matches prec).
struct Tables {
    const void* tw;       // w_NT^e, e < NT = max(n1, n2) (mixed-radix classes: NT = n1)
    const void* tw2;      // roots of the column transforms: tw itself, or (mixed-radix
                          // classes) w_n2^e, e < n2
    const void* fa;       // w_L^{h << fshift}, h < ceil(L / 2^fshift)
    const void* fb;       // w_L^l, l < 1 << fshift
    int fshift;
    const void* stw;      // wave-transform stage tables, sizes 16..1024
    const double* fa64;   // fa, fb in FP64 (for FP64 classes the same arrays as fa, fb)
    const double* fb64;
};

// Enqueues one pass of a class on `stream`: 0 when a kernel was launched, 1
// when the pass has no kernel for this launch (one-kernel tiles), -1 on a
// launch error.
typedef int (*launch_fn)(const JobTable& jt, void* ws, uint32_t* part, TileMeta* meta,
                         const Tables& tb, void* stream);

struct ClassKernels {
    ClassCfg cfg;
    launch_fn pass1, pass2, pass3;
};

// Registered by the per-precision kernel objects.
const ClassKernels* class_kernels(int prec, int cls);

constexpr int kMinLogL = 12;
constexpr int kMaxLogL32 = 24;
constexpr int kMaxLogL64 = 24;

}  // namespace pa
