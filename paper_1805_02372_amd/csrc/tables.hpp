// Host-side twiddle tables (see tables.cpp).
#pragma once
#include <cstdint>
#include <vector>

namespace pa {

// exp(-2 pi i e / N) in long double.
void unit_root(uint64_t e, uint64_t N, long double* c, long double* s);

// Interleaved (re, im) tables of one FFT length class:
//   tw[e] = w_NT^e, e < NT = max(n1, n2) (mixed-radix classes: NT = n1);
//   tw2[e] = w_n2^e, e < n2 (mixed-radix classes only: the roots of the
//        column transforms; a power-of-two class uses tw for both);
//   fa[h] = w_L^{h << fshift}, h < ceil(L / 2^fshift), fb[l] = w_L^l, so
//        w_L^e = fa[e >> fshift] fb[e & mask] for every e < L;
//   stw: stage tables of the wave transforms of every size 16..1024 (layout
//        in wave_fft.hpp);
//   fa64, fb64: fa and fb in FP64 (FP32 classes only; an FP64 class uses fa
//        and fb), for twiddles formed as FP64 products and rounded once.
template <typename T> struct TableHost {
    std::vector<T> tw, tw2, fa, fb, stw;
    std::vector<double> fa64, fb64;
    int fshift = 0;
};

// Tables of the class of FFT length L = n1 * n2; `smooth`: a mixed-radix class.
template <typename T> void build_tables(uint64_t L, int n1, int n2, bool smooth, TableHost<T>* th);

// Number-theoretic tables modulo p = 15 * 2^27 + 1 in Montgomery form
// (a -> a 2^32 mod p): tw[e] = w_NT^e, fa / fb the two-level w_L tables, and
// stw = {L^{-1} mod p (plain), 2^32 mod p}.  w_N = 31^((p-1)/N); L a power of two.
void build_ntt_tables(uint64_t L, int n1, int n2, TableHost<uint32_t>* th);

}  // namespace pa
