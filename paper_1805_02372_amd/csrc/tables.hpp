// Host-side twiddle tables (see tables.cpp).
#pragma once
#include <cstdint>
#include <vector>

namespace pa {

// exp(-2 pi i e / N) in long double.
void unit_root(uint64_t e, uint64_t N, long double* c, long double* s);

// Interleaved (re, im) tables of one FFT length class:
//   tw[e] = w_NT^e, e < NT = max(n1, n2);
//   fa[h] = w_L^{h << fshift}, fb[l] = w_L^l, so w_L^e = fa[e >> fshift] fb[e & mask].
//   stw: stage tables of the wave transforms of every size 16..1024 (layout
//        in wave_fft.hpp).
//   fa64, fb64: fa and fb in FP64 (FP32 classes only; an FP64 class uses fa
//        and fb), for twiddles formed as FP64 products and rounded once.
template <typename T> struct TableHost {
    std::vector<T> tw, fa, fb, stw;
    std::vector<double> fa64, fb64;
    int fshift = 0;
};

template <typename T> void build_tables(int logL, int n1, int n2, TableHost<T>* th);

// Number-theoretic tables modulo p = 15 * 2^27 + 1 in Montgomery form
// (a -> a 2^32 mod p): tw[e] = w_NT^e, fa / fb the two-level w_L tables, and
// stw = {L^{-1} mod p (plain), 2^32 mod p}.  w_N = 31^((p-1)/N).
void build_ntt_tables(int logL, int n1, int n2, TableHost<uint32_t>* th);

}  // namespace pa
