// Exact Toeplitz hash by number-theoretic transform (the paper's section 1
// cites NTT acceleration of privacy amplification as prior art): the tile
// convolution of a 0/1 seed slice with a 0/1 key chunk is computed modulo the
// prime p = 15 * 2^27 + 1.  Every coefficient of the kept window is at most
// bi < p, so the residue is the integer itself and bit = residue & 1 with no
// rounding step.  This path cross-checks the floating-point paths.
//
// Same tile geometry and four-step split as the FFT passes (t = t1 + n1 t2,
// k = k2 + n2 k1), but the two sequences are transformed separately (no
// conjugate symmetry in a prime field):
//   pass 1: column transforms of x and w  -> X[k2][t1], W[k2][t1] (twiddled)
//   pass 2: row transforms, P = X * W, inverse row transform (in place in X)
//   pass 3: inverse column transforms, scale by 1/L, window, parity, pack.
// Arithmetic: 32-bit Montgomery form (R = 2^32); data values are kept fully
// reduced in [0, p).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_internal.hpp"
#include "conv_kernels.hpp"

namespace pa {
namespace ntt {

constexpr uint32_t P = 2013265921u;       // 15 * 2^27 + 1
constexpr uint32_t PINV_NEG = []() {      // -p^{-1} mod 2^32
    uint32_t inv = 1;
    for (int i = 0; i < 5; ++i) inv *= 2u - P * inv;   // Newton iteration mod 2^32
    return (uint32_t)(0u - inv);
}();

__device__ __forceinline__ uint32_t mmul(uint32_t a, uint32_t b) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * PINV_NEG;
    const uint64_t u = (t + (uint64_t)m * P) >> 32;
    return u >= P ? (uint32_t)(u - P) : (uint32_t)u;
}
__device__ __forceinline__ uint32_t madd(uint32_t a, uint32_t b) {
    const uint32_t s = a + b;   // < 2^32 since a, b < 2^31
    return s >= P ? s - P : s;
}
__device__ __forceinline__ uint32_t msub(uint32_t a, uint32_t b) { return a >= b ? a - b : a + P - b; }

// Roots table layout (Montgomery form), per length class:
//   tw[e] = w_NT^e (e < NT), w_NT a primitive NT-th root; inverse uses tw[NT - e].
//   fa[h] = w_L^{h << fs}, fb[l] = w_L^l (l < 2^fs); inverse uses exponent L - e.
//   w4m = w_4 (Montgomery form); the radix-4 butterfly needs it.
struct Roots {
    const uint32_t* tw;
    const uint32_t* fa;
    const uint32_t* fb;
    int fshift;
    uint32_t NT;
    uint32_t w4;      // forward w_4
    uint32_t linv;    // plain L^{-1} mod p (mmul(Montgomery y, linv) = y L^{-1}, plain)
    uint32_t one_m;   // R mod p (Montgomery form of 1)
};

template <int DIR>
__device__ __forceinline__ uint32_t root(const Roots& r, uint32_t e /* < NT */) {
    if (DIR < 0 || e == 0) return r.tw[e];
    return r.tw[r.NT - e];
}
template <int DIR>
__device__ __forceinline__ uint32_t root_L(const Roots& r, uint32_t e, uint32_t L) {
    if (DIR > 0 && e) e = L - e;
    return mmul(r.fa[e >> r.fshift], r.fb[e & ((1u << r.fshift) - 1u)]);
}

template <int DIR>
__device__ __forceinline__ void bfly4(uint32_t& u0, uint32_t& u1, uint32_t& u2, uint32_t& u3, uint32_t w4) {
    const uint32_t a0 = madd(u0, u2), a1 = msub(u0, u2);
    const uint32_t a2 = madd(u1, u3);
    uint32_t a3 = mmul(msub(u1, u3), w4);          // w4 for DIR < 0, -w4 = w4^{-1} otherwise
    if (DIR > 0) a3 = a3 ? P - a3 : 0;
    u0 = madd(a0, a2);
    u2 = msub(a0, a2);
    u1 = madd(a1, a3);
    u3 = msub(a1, a3);
}

// Workgroup Stockham transform of F interleaved sequences of N points; thread
// (f, j) holds R values x_f[j + i N/R]; on exit X_f[j + i N/R].  Radix 4 with
// one radix-2 stage first when log2 N is odd.
template <int DIR, int N, int R, int F, int Ns>
__device__ __forceinline__ void stages(uint32_t (&v)[R], uint32_t* lds, int j, int f, const Roots& rt) {
    constexpr int LOGN = ilog2(N);
    constexpr int Rs = (Ns == 1 && (LOGN & 1)) ? 2 : 4;
    constexpr int PB = R / Rs, NR = N / R;
    constexpr bool LAST = Ns * Rs == N;
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int q = j + p * NR;
        const int k = q & (Ns - 1);
        uint32_t u[4];
#pragma unroll
        for (int r = 0; r < Rs; ++r) u[r] = v[p + r * PB];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < Rs; ++r)
                u[r] = mmul(u[r], root<DIR>(rt, (uint32_t)(k * r) * (rt.NT / (uint32_t)(Ns * Rs))));
        }
        if constexpr (Rs == 2) {
            const uint32_t a = u[0], b = u[1];
            u[0] = madd(a, b);
            u[1] = msub(a, b);
        } else {
            bfly4<DIR>(u[0], u[1], u[2], u[3], rt.w4);
        }
#pragma unroll
        for (int r = 0; r < Rs; ++r) v[p + r * PB] = u[r];
    }
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int q = j + p * NR;
            const int k = q & (Ns - 1);
            const int base = (q / Ns) * Ns * Rs + k;
#pragma unroll
            for (int r = 0; r < Rs; ++r) lds[lds_slot<F>(base + r * Ns, f)] = v[p + r * PB];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = lds[lds_slot<F>(j + i * NR, f)];
        stages<DIR, N, R, F, Ns * Rs>(v, lds, j, f, rt);
    }
}

template <int DIR, int N, int R, int F>
__device__ __forceinline__ void transform(uint32_t (&v)[R], uint32_t* lds, int j, int f, const Roots& rt) {
    static_assert(R >= 4 && (R & (R - 1)) == 0 && N >= R, "points per thread");
    stages<DIR, N, R, F, 1>(v, lds, j, f, rt);
}

constexpr int kB1 = 4, kB3 = 8, kR = 16;

// ---------------------------------------------------------------- pass 1
// Workgroup: kB1 columns of x and of w (2 kB1 interleaved transforms).
template <int N1, int N2>
__global__ void __launch_bounds__(2 * kB1 * (N2 / kR))
k_ntt1(JobTable jt, uint32_t* __restrict__ ws, uint32_t* __restrict__ part, Roots rt) {
    constexpr uint32_t L = (uint32_t)N1 * N2;
    constexpr int F = 2 * kB1, NCB = N1 / kB1, NR = N2 / kR;
    __shared__ uint32_t lds[lds_slots<N2, F>()];
    __shared__ uint32_t wsum;
    const uint32_t lt = blockIdx.x / NCB, cb = blockIdx.x % NCB;
    const uint32_t t = jt.tile0 + lt;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const int tid = threadIdx.x, f = tid % F, j = tid / F;
    const int col = f % kB1;
    const bool is_w = f >= kB1;
    const uint32_t t1 = cb * kB1 + col;
    const uint32_t bi = (uint32_t)g.bi, win = (uint32_t)(g.bi + g.bo - 1);
    if (tid == 0) wsum = 0;
    clear_window(g, cb, NCB, tid, 2 * kB1 * (N2 / kR));
    __syncthreads();
    uint32_t v[kR];
    uint32_t pc = 0;
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const uint32_t tt = t1 + (uint32_t)N1 * (uint32_t)(j + i * NR);
        uint32_t bit = 0;
        if (!is_w) {
            uint32_t u = tt + bi - 1;
            if (u >= L) u -= L;
            if (u < bi) {
                const uint64_t kb = g.j0 + u;
                bit = (uint32_t)(jd.key[kb >> 6] >> (kb & 63)) & 1u;
            }
            pc += bit;
        } else if (tt < win) {
            const uint64_t sb = g.sigma + tt;
            bit = (uint32_t)(jd.seed[sb >> 6] >> (sb & 63)) & 1u;
        }
        v[i] = bit ? rt.one_m : 0u;
    }
    atomicAdd(&wsum, pc);
    transform<-1, N2, kR, F>(v, lds, j, f, rt);
    uint32_t* __restrict__ Y = ws + (size_t)lt * 2 * L + (is_w ? L : 0);
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const uint32_t k2 = (uint32_t)(j + i * NR);
        Y[(size_t)k2 * N1 + t1] = mmul(v[i], root_L<-1>(rt, t1 * k2, L));
    }
    __syncthreads();
    if (tid == 0) part[(size_t)lt * NCB + cb] = wsum;
}

// ---------------------------------------------------------------- pass 2
// Workgroup: one row k2 of X and of W; product; inverse row (in place in X).
template <int N1, int N2>
__global__ void __launch_bounds__(2 * N1 / kR)
k_ntt2(JobTable jt, uint32_t* __restrict__ ws, const uint32_t* __restrict__ part, TileMeta* __restrict__ meta,
       Roots rt) {
    constexpr uint32_t L = (uint32_t)N1 * N2;
    constexpr int T = 2 * N1 / kR, NR = N1 / kR, NCB1 = N1 / kB1;
    constexpr int RI = N1 / T;   // points per thread of the single inverse transform (8)
    __shared__ uint32_t lds[lds_slots<N1, 2>()];
    __shared__ uint32_t wsum;
    const uint32_t lt = blockIdx.x / N2;
    const uint32_t k2 = blockIdx.x % N2;
    const int tid = threadIdx.x, f = tid % 2, j = tid / 2;
    uint32_t* __restrict__ X = ws + (size_t)lt * 2 * L;
    const uint32_t* __restrict__ W = X + L;
    if (k2 == 0) {
        if (tid == 0) wsum = 0;
        __syncthreads();
        uint32_t s = 0;
        for (int c = tid; c < NCB1; c += T) s += part[(size_t)lt * NCB1 + c];
        atomicAdd(&wsum, s);
        __syncthreads();
        if (tid == 0) meta[jt.tile0 + lt] = TileMeta{wsum, 0u, 0u, 0u};
    }
    uint32_t v[kR];
    const uint32_t* row = (f ? W : X) + (size_t)k2 * N1;
#pragma unroll
    for (int i = 0; i < kR; ++i) v[i] = row[j + i * NR];
    transform<-1, N1, kR, 2>(v, lds, j, f, rt);
    // product: the X thread needs the W value at the same index
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kR; ++i) lds[lds_slot<2>(j + i * NR, f)] = v[i];
    __syncthreads();
    // inverse row transform of P = X W by all T threads, RI points each
    uint32_t pv[RI];
    constexpr int NRI = N1 / RI;
#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const int e = tid + i * NRI;
        pv[i] = mmul(lds[lds_slot<2>(e, 0)], lds[lds_slot<2>(e, 1)]);
    }
    __syncthreads();
    transform<+1, N1, RI, 1>(pv, lds, tid, 0, rt);
#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const uint32_t t1 = (uint32_t)(tid + i * NRI);
        X[(size_t)k2 * N1 + t1] = mmul(pv[i], root_L<+1>(rt, k2 * t1, L));
    }
}

// ---------------------------------------------------------------- pass 3
template <int N1, int N2>
__global__ void __launch_bounds__(kB3 * (N2 / kR))
k_ntt3(JobTable jt, const uint32_t* __restrict__ ws, TileMeta* __restrict__ meta, Roots rt) {
    constexpr uint32_t L = (uint32_t)N1 * N2;
    constexpr int NCB = N1 / kB3, NR = N2 / kR;
    __shared__ uint32_t lds[lds_slots<N2, kB3>()];
    __shared__ uint32_t s_bad;
    const uint32_t lt = blockIdx.x / NCB, cb = blockIdx.x % NCB;
    const uint32_t t = jt.tile0 + lt;
    const JobDesc jd = find_job(jt, t);
    const TileGeo g = tile_geo(jd, t - jd.tile_begin);
    const uint32_t* __restrict__ X = ws + (size_t)lt * 2 * L;
    const int tid = threadIdx.x, f = tid % kB3, j = tid / kB3;
    const uint32_t t1 = cb * kB3 + f;
    if (tid == 0) s_bad = 0;
    uint32_t v[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) v[i] = X[(size_t)(j + i * NR) * N1 + t1];
    transform<+1, N2, kR, kB3>(v, lds, j, f, rt);
    uint32_t bad = 0;
    const int lane = tid & 63;
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const uint32_t t2 = (uint32_t)(j + i * NR);
        const uint64_t vo = (uint64_t)t1 + (uint64_t)N1 * t2;
        uint32_t bit = 0;
        if (vo < g.bo) {
            const uint32_t c = mmul(v[i], rt.linv);   // plain convolution value
            bad += c > (uint32_t)g.bi;                 // a window value counts at most bi products
            bit = c & 1u;
        }
        const uint64_t mask = __ballot(bit);
        if (f == 0) {
            const uint64_t off = (uint64_t)cb * kB3 + (uint64_t)N1 * t2;
            if (off < g.dst_words * 64u) put_bits<8>(g, off, (uint32_t)((mask >> lane) & 0xFFu));
        }
    }
    __syncthreads();
    if (bad) atomicAdd(&s_bad, bad);
    __syncthreads();
    if (tid == 0 && s_bad) atomicAdd(&meta[t].badpar, s_bad);
}

template <int N1, int N2>
struct Impl {
    static Roots roots(const Tables& tb) {
        Roots r;
        const uint32_t* base = (const uint32_t*)tb.tw;
        r.tw = base;
        r.fa = (const uint32_t*)tb.fa;
        r.fb = (const uint32_t*)tb.fb;
        r.fshift = tb.fshift;
        r.NT = (uint32_t)(N1 > N2 ? N1 : N2);
        r.w4 = base[r.NT / 4];
        r.linv = ((const uint32_t*)tb.stw)[0];
        r.one_m = ((const uint32_t*)tb.stw)[1];
        return r;
    }
    static int pass1(const JobTable& jt, void* ws, uint32_t* part, TileMeta*, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (N1 / kB1)), block(2 * kB1 * (N2 / kR));
        hipLaunchKernelGGL((k_ntt1<N1, N2>), grid, block, 0, (hipStream_t)stream, jt, (uint32_t*)ws, part,
                           roots(tb));
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass2(const JobTable& jt, void* ws, uint32_t* part, TileMeta* meta, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * N2), block(2 * N1 / kR);
        hipLaunchKernelGGL((k_ntt2<N1, N2>), grid, block, 0, (hipStream_t)stream, jt, (uint32_t*)ws,
                           (const uint32_t*)part, meta, roots(tb));
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    static int pass3(const JobTable& jt, void* ws, uint32_t*, TileMeta* meta, const Tables& tb, void* stream) {
        dim3 grid(jt.ntiles * (N1 / kB3)), block(kB3 * (N2 / kR));
        hipLaunchKernelGGL((k_ntt3<N1, N2>), grid, block, 0, (hipStream_t)stream, jt, (const uint32_t*)ws, meta,
                           roots(tb));
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
};

}  // namespace ntt

// Classes (power-of-two only): L = n1 * n2 = 2^logL, n2 = 2^min(11, logL/2),
// rows up to 8192.
#define PA_NTT_CLASS(LOGL, N1, N2) \
    {ClassCfg{1, LOGL, N1, N2, ntt::kB1, ntt::kB3, ntt::kR}, &ntt::Impl<N1, N2>::pass1, \
     &ntt::Impl<N1, N2>::pass2, &ntt::Impl<N1, N2>::pass3}

static const ClassKernels kClassesNtt[] = {
    PA_NTT_CLASS(12, 64, 64),     PA_NTT_CLASS(13, 128, 64),    PA_NTT_CLASS(14, 128, 128),
    PA_NTT_CLASS(15, 256, 128),   PA_NTT_CLASS(16, 256, 256),   PA_NTT_CLASS(17, 512, 256),
    PA_NTT_CLASS(18, 512, 512),   PA_NTT_CLASS(19, 1024, 512),  PA_NTT_CLASS(20, 1024, 1024),
    PA_NTT_CLASS(21, 2048, 1024), PA_NTT_CLASS(22, 2048, 2048), PA_NTT_CLASS(23, 4096, 2048),
    PA_NTT_CLASS(24, 8192, 2048),
};

const ClassKernels* class_kernels_ntt(int cls) {
    for (const ClassKernels& k : kClassesNtt)
        if (k.cfg.cls == cls) return &k;
    return nullptr;
}

}  // namespace pa
