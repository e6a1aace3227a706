// Device-side FFT building blocks for gfx950: complex arithmetic, radix
// 2/3/4/5/7/8/16 DFT butterflies in registers, and a mixed-radix Stockham
// auto-sort FFT whose stages exchange data through LDS.
//
// Conventions.  DIR = -1 is the forward transform X_k = sum_t x_t w^{tk} with
// w = exp(-2 pi i / N); DIR = +1 the unnormalised inverse (w -> conj w).
// Twiddle tables hold the forward roots exp(-2 pi i k / NT) in the working
// precision, computed on the host in extended precision; a DIR = +1 stage uses
// their conjugates.
//
// Stockham stage (radix Rs, span Ns = product of the earlier radices, N
// points; any factorisation of N into the radices above): butterfly q reads
// x[q + r N/Rs] (r < Rs), multiplies input r by w_{Ns Rs}^{(q mod Ns) r},
// applies the Rs-point DFT and writes output s to
// x'[(q / Ns) Ns Rs + (q mod Ns) + s Ns].  After the last stage (Ns Rs = N) the
// result is in natural order.  A thread owns R points; in every stage it loads
// x[j + i N/R] (i < R) and runs R/Rs butterflies q = j + p N/R, so after the
// last stage register i holds X[j + i N/R].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

template <typename T> struct cx { T re, im; };

template <typename T> __device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
// a * b
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// multiply by DIR * i  (forward DIR=-1: -i; inverse: +i)
template <int DIR, typename T> __device__ __forceinline__ cx<T> rot90(cx<T> a) {
    return DIR < 0 ? cx<T>{a.im, -a.re} : cx<T>{-a.im, a.re};
}
// multiply by the table root w (forward) or its conjugate (inverse)
template <int DIR, typename T> __device__ __forceinline__ cx<T> twmul(cx<T> a, cx<T> w) {
    return DIR < 0 ? cmul(a, w) : cmulc(a, w);
}

// Constants in the working precision (double literals rounded once).
template <typename T> struct K {
    static constexpr T r2 = (T)0.70710678118654752440084436210485;   // cos(pi/4)
    static constexpr T c8 = (T)0.92387953251128675612818318939679;   // cos(pi/8)
    static constexpr T s8 = (T)0.38268343236508977172845998403040;   // sin(pi/8)
};

// ---------------------------------------------------------------- butterflies

template <int DIR, typename T> __device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
    cx<T> t = a - b;
    a = a + b;
    b = t;
}

template <int DIR, typename T> __device__ __forceinline__ void dft4(cx<T>& u0, cx<T>& u1, cx<T>& u2, cx<T>& u3) {
    cx<T> a0 = u0 + u2, a1 = u0 - u2;
    cx<T> a2 = u1 + u3, a3 = rot90<DIR>(u1 - u3);
    u0 = a0 + a2;
    u2 = a0 - a2;
    u1 = a1 + a3;
    u3 = a1 - a3;
}

// multiply by w8^k, w8 = exp(DIR 2 pi i / 8)
template <int DIR, int k, typename T> __device__ __forceinline__ cx<T> w8(cx<T> a) {
    constexpr T r2 = K<T>::r2;
    if constexpr (k == 0) return a;
    else if constexpr (k == 2) return rot90<DIR>(a);
    else if constexpr (k == 1) {
        // (1 + DIR i)/sqrt2 * a
        return DIR < 0 ? cx<T>{(a.re + a.im) * r2, (a.im - a.re) * r2}
                       : cx<T>{(a.re - a.im) * r2, (a.im + a.re) * r2};
    } else {  // k == 3: (-1 + DIR i)/sqrt2
        return DIR < 0 ? cx<T>{(a.im - a.re) * r2, -(a.re + a.im) * r2}
                       : cx<T>{-(a.re + a.im) * r2, (a.re - a.im) * r2};
    }
}

template <int DIR, typename T> __device__ __forceinline__ void dft8(cx<T>* u) {
    // even/odd split: E = DFT4(u0,u2,u4,u6), O = DFT4(u1,u3,u5,u7)
    dft4<DIR>(u[0], u[2], u[4], u[6]);
    dft4<DIR>(u[1], u[3], u[5], u[7]);
    cx<T> o1 = w8<DIR, 1>(u[3]), o2 = w8<DIR, 2>(u[5]), o3 = w8<DIR, 3>(u[7]);
    cx<T> e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6], o0 = u[1];
    u[0] = e0 + o0; u[4] = e0 - o0;
    u[1] = e1 + o1; u[5] = e1 - o1;
    u[2] = e2 + o2; u[6] = e2 - o2;
    u[3] = e3 + o3; u[7] = e3 - o3;
}

// multiply by w16^k, w16 = exp(DIR 2 pi i / 16), for the exponents a 4x4
// split needs (1, 2, 3, 4, 6, 9)
template <int DIR, int k, typename T> __device__ __forceinline__ cx<T> w16(cx<T> a) {
    constexpr T c = K<T>::c8, s = K<T>::s8;
    if constexpr (k == 0) return a;
    else if constexpr (k == 2) return w8<DIR, 1>(a);
    else if constexpr (k == 4) return rot90<DIR>(a);
    else if constexpr (k == 6) return w8<DIR, 3>(a);
    else {
        // cos(2 pi k/16), DIR*sin(2 pi k/16)
        constexpr T cr = (k == 1) ? c : (k == 3) ? s : -c;      // k=9: cos(9pi/8) = -cos(pi/8)
        constexpr T si0 = (k == 1) ? s : (k == 3) ? c : -s;     // sin(9pi/8) = -sin(pi/8)
        constexpr T si = DIR < 0 ? -si0 : si0;
        return cx<T>{a.re * cr - a.im * si, a.re * si + a.im * cr};
    }
}

template <int DIR, typename T> __device__ __forceinline__ void dft16(cx<T>* u) {
    // index r = 4 r1 + r2, output s = s1 + 4 s2
    dft4<DIR>(u[0], u[4], u[8], u[12]);
    dft4<DIR>(u[1], u[5], u[9], u[13]);
    dft4<DIR>(u[2], u[6], u[10], u[14]);
    dft4<DIR>(u[3], u[7], u[11], u[15]);
    // F[r2][s1] lives at u[r2 + 4 s1]; twiddle by w16^{r2 s1}
    u[5] = w16<DIR, 1>(u[5]);
    u[9] = w16<DIR, 2>(u[9]);
    u[13] = w16<DIR, 3>(u[13]);
    u[6] = w16<DIR, 2>(u[6]);
    u[10] = w16<DIR, 4>(u[10]);
    u[14] = w16<DIR, 6>(u[14]);
    u[7] = w16<DIR, 3>(u[7]);
    u[11] = w16<DIR, 6>(u[11]);
    u[15] = w16<DIR, 9>(u[15]);
    // for each s1: DFT4 over r2 -> out[s1 + 4 s2] at u[4 s1 + s2]
    dft4<DIR>(u[0], u[1], u[2], u[3]);
    dft4<DIR>(u[4], u[5], u[6], u[7]);
    dft4<DIR>(u[8], u[9], u[10], u[11]);
    dft4<DIR>(u[12], u[13], u[14], u[15]);
    // transpose u[4 s1 + s2] -> natural order u[s1 + 4 s2]
    cx<T> t;
    t = u[1]; u[1] = u[4]; u[4] = t;
    t = u[2]; u[2] = u[8]; u[8] = t;
    t = u[3]; u[3] = u[12]; u[12] = t;
    t = u[6]; u[6] = u[9]; u[9] = t;
    t = u[7]; u[7] = u[13]; u[13] = t;
    t = u[11]; u[11] = u[14]; u[14] = t;
}

// cos and sin of 2 pi e / P (0 < e <= P/2) for the odd radices P = 3, 5, 7
// (double literals; rounded once to the working precision where used).
constexpr double odd_root(int P, int e, bool sine) {
    if (P == 3) return sine ? 0.86602540378443864676372317075294 : -0.5;
    if (P == 5) {
        if (e == 1) return sine ? 0.95105651629515357211643933337938 : 0.30901699437494742410229341718282;
        return sine ? 0.58778525229247312916870595463907 : -0.80901699437494742410229341718282;
    }
    if (e == 1) return sine ? 0.78183148246802980870844452667406 : 0.62348980185873353052500488400424;
    if (e == 2) return sine ? 0.97492791218182360701813168299393 : -0.22252093395631440428890256449679;
    return sine ? 0.43388373911755812047576833284836 : -0.90096886790241912623610231950745;
}
// cos(2 pi e / P) and sin(2 pi e / P) for any 0 < e < P
constexpr double odd_cos(int P, int e) { return odd_root(P, e <= P / 2 ? e : P - e, false); }
constexpr double odd_sin(int P, int e) { return e <= P / 2 ? odd_root(P, e, true) : -odd_root(P, P - e, true); }

// P-point DFT for an odd prime P by pairing inputs s and P - s: with
// a_s = u_s + u_{P-s} and b_s = u_s - u_{P-s} (s = 1 .. (P-1)/2),
//   y_k     = u_0 + sum_s cos(2 pi s k / P) a_s + DIR i sum_s sin(2 pi s k / P) b_s,
//   y_{P-k} = the same with the sine sum negated   (k = 1 .. (P-1)/2),
// since the root of the transform is exp(DIR 2 pi i / P).  All loops unroll,
// so the roots are compile-time constants.
template <int DIR, int P, typename T> __device__ __forceinline__ void dft_odd(cx<T>* u) {
    constexpr int H = (P - 1) / 2;
    cx<T> a[H], b[H];
#pragma unroll
    for (int s = 0; s < H; ++s) {
        a[s] = u[s + 1] + u[P - 1 - s];
        b[s] = u[s + 1] - u[P - 1 - s];
    }
    const cx<T> u0 = u[0];
    cx<T> y0 = u0;
#pragma unroll
    for (int s = 0; s < H; ++s) y0 = y0 + a[s];
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        cx<T> c = u0, d = cx<T>{T(0), T(0)};
#pragma unroll
        for (int s = 1; s <= H; ++s) {
            const T cs = (T)odd_cos(P, (s * k) % P), sn = (T)odd_sin(P, (s * k) % P);
            c.re += cs * a[s - 1].re;
            c.im += cs * a[s - 1].im;
            d.re += sn * b[s - 1].re;
            d.im += sn * b[s - 1].im;
        }
        const cx<T> id = rot90<DIR>(d);   // DIR i d
        u[k] = c + id;
        u[P - k] = c - id;
    }
    u[0] = y0;
}

template <int Rs, int DIR, typename T> __device__ __forceinline__ void dft(cx<T>* u) {
    if constexpr (Rs == 1) {
    } else if constexpr (Rs == 2) dft2<DIR>(u[0], u[1]);
    else if constexpr (Rs == 3 || Rs == 5 || Rs == 7) dft_odd<DIR, Rs>(u);
    else if constexpr (Rs == 4) dft4<DIR>(u[0], u[1], u[2], u[3]);
    else if constexpr (Rs == 8) dft8<DIR>(u);
    else if constexpr (Rs == 16) dft16<DIR>(u);
    else static_assert(Rs == 2, "unsupported radix");
}

// ------------------------------------------------------------------ LDS layout
// F interleaved transforms of N points; element e of transform f lives at
// e*F + f, plus one pad slot after every 16 slots so that stride-16 stores
// (the first stages) spread over the LDS banks.
template <int F> __device__ __forceinline__ int lds_slot(int e, int f) {
    int s = e * F + f;
    return s + (s >> 4);
}
template <int N, int F> constexpr int lds_slots() { return N * F + (N * F >> 4) + 1; }

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Stage radices of an N-point transform whose threads hold R points each.
// N = P * 2^k with P in {1, 3, 5, 7} dividing R: an odd first stage of radix
// P, then power-of-two stages of radix Q (the largest power of two dividing
// R, at most 16), the first of them taking the remainder so that the rest are
// all radix Q.
constexpr int odd_part(int n) { return (n % 2 == 0 && n > 0) ? odd_part(n / 2) : n; }
constexpr int pow2_radix(int R, int q = 1) { return (R % (2 * q) == 0 && 2 * q <= 16) ? pow2_radix(R, 2 * q) : q; }
constexpr int stockham_radix(int N, int R, int Ns) {
    const int P = odd_part(N);
    if (Ns == 1 && P > 1) return P;
    const int lq = ilog2(pow2_radix(R)), lr = ilog2(N / Ns);
    return (Ns == P && lr % lq) ? (1 << (lr % lq)) : (1 << lq);
}
// Whether the FFT below supports (N, R).
constexpr bool stockham_ok(int N, int R) {
    const int P = odd_part(N);
    return N % R == 0 && (P == 1 || P == 3 || P == 5 || P == 7) && R % P == 0 && pow2_radix(R) >= 2;
}

// One Stockham stage.  v: the thread's R points (layout described above).
// tw: forward roots of unity w_NT^e at tw[e]; NT a multiple of N.
// SPLIT: the exchange moves the real parts, then the imaginary parts, through
// an LDS buffer of lds_slots<N, F>() scalars (half the bytes, two more
// barriers per stage), for transforms whose complex buffer would leave room
// for only one workgroup per compute unit.
template <typename T, int DIR, int N, int R, int Rs, int Ns, int F, int NT, bool SPLIT>
__device__ __forceinline__ void stockham_stage(cx<T> (&v)[R], cx<T>* lds, int j, int f,
                                               const cx<T>* __restrict__ tw) {
    constexpr int P = R / Rs;
    constexpr int NR = N / R;
    constexpr bool LAST = (Ns * Rs == N);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        cx<T> u[Rs];
#pragma unroll
        for (int r = 0; r < Rs; ++r) u[r] = v[p + r * P];
        if constexpr (Ns > 1) {
            const int k = (j + p * NR) % Ns;
            static_assert(NT % (Ns * Rs) == 0, "twiddle table length");
            constexpr int step = NT / (Ns * Rs);
#pragma unroll
            for (int r = 1; r < Rs; ++r) u[r] = twmul<DIR>(u[r], tw[k * r * step]);
        }
        dft<Rs, DIR>(u);
#pragma unroll
        for (int r = 0; r < Rs; ++r) v[p + r * P] = u[r];
    }
    if constexpr (!LAST && !SPLIT) {
        __syncthreads();  // everyone has finished reading the previous exchange
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int q = j + p * NR;
            const int k = q % Ns;
            const int base = (q / Ns) * Ns * Rs + k;
#pragma unroll
            for (int r = 0; r < Rs; ++r) lds[lds_slot<F>(base + r * Ns, f)] = v[p + r * P];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = lds[lds_slot<F>(j + i * NR, f)];
    } else if constexpr (!LAST) {
        // the real parts, then the imaginary parts: the writes of a half read
        // the parts of v that its reads have not replaced yet
        T* __restrict__ half = reinterpret_cast<T*>(lds);
#pragma unroll
        for (int part = 0; part < 2; ++part) {
            __syncthreads();
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int q = j + p * NR;
                const int k = q % Ns;
                const int base = (q / Ns) * Ns * Rs + k;
#pragma unroll
                for (int r = 0; r < Rs; ++r)
                    half[lds_slot<F>(base + r * Ns, f)] = part ? v[p + r * P].im : v[p + r * P].re;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const T x = half[lds_slot<F>(j + i * NR, f)];
                if (part) v[i].im = x;
                else v[i].re = x;
            }
        }
    }
}

template <typename T, int DIR, int N, int R, int F, int NT, int Ns, bool SPLIT>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[R], cx<T>* lds, int j, int f,
                                           const cx<T>* __restrict__ tw) {
    constexpr int Rs = stockham_radix(N, R, Ns);
    static_assert(R % Rs == 0, "stage radix divides the points per thread");
    stockham_stage<T, DIR, N, R, Rs, Ns, F, NT, SPLIT>(v, lds, j, f, tw);
    if constexpr (Ns * Rs < N) fft_stages<T, DIR, N, R, F, NT, Ns * Rs, SPLIT>(v, lds, j, f, tw);
}

// N-point FFT of F interleaved transforms held by N/R * F threads.  On entry
// register i of thread (f, j) holds x_f[j + i N/R]; on exit X_f[j + i N/R].
// The LDS buffer must hold lds_slots<N, F>() elements (SPLIT: that many
// scalars).  Contains barriers: every thread of the workgroup must call it.
template <typename T, int DIR, int N, int R, int F, int NT, bool SPLIT = false>
__device__ __forceinline__ void fft(cx<T> (&v)[R], cx<T>* lds, int j, int f,
                                    const cx<T>* __restrict__ tw) {
    static_assert(stockham_ok(N, R), "N = P 2^k (P = 1, 3, 5, 7), R a multiple of P and of 2");
    fft_stages<T, DIR, N, R, F, NT, 1, SPLIT>(v, lds, j, f, tw);
}

// Whether a workgroup's complex exchange buffer of N F points would leave
// room for only one workgroup per compute unit (160 KB of LDS), so that the
// split exchange lets two share it.
template <typename T, int N, int F> constexpr bool split_exchange() {
    return (size_t)lds_slots<N, F>() * sizeof(cx<T>) > 81920;
}

}  // namespace pa
