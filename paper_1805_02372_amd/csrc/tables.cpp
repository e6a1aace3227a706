// Twiddle tables, computed on the host in extended precision and rounded once
// to the working precision.
#include <cmath>
#include <cstdint>
#include <vector>

#include "tables.hpp"
#include "wave_fft.hpp"

namespace pa {

// exp(-2 pi i e / N) = c + i s.  The angle is reduced to the nearest quarter
// turn first, so multiples of pi/2 come out exact and the table is symmetric.
void unit_root(uint64_t e, uint64_t N, long double* c, long double* s) {
    e %= N;
    // e/N = q/4 + d/N with |d/N| <= 1/8
    const uint64_t q = (4 * e + N / 2) / N;        // nearest quarter turn
    const long double d = (long double)e - (long double)q * (long double)N / 4.0L;
    const long double th = 2.0L * 3.14159265358979323846264338327950288L * d / (long double)N;
    const long double cd = cosl(th), sd = sinl(th);
    long double cc, ss;  // cos and sin of the full angle
    switch (q & 3) {
        case 0: cc = cd; ss = sd; break;
        case 1: cc = -sd; ss = cd; break;
        case 2: cc = -cd; ss = -sd; break;
        default: cc = sd; ss = -cd; break;
    }
    *c = cc;
    *s = -ss;
}

template <typename T>
static void roots(std::vector<T>& out, uint64_t count, uint64_t N, uint64_t mult) {
    out.resize(2 * count);
    for (uint64_t e = 0; e < count; ++e) {
        long double c, s;
        unit_root(e * mult, N, &c, &s);
        out[2 * e] = (T)c;
        out[2 * e + 1] = (T)s;
    }
}

static int log2_ceil(uint64_t L) {
    int k = 0;
    while ((1ull << k) < L) ++k;
    return k;
}

template <typename T>
void build_tables(uint64_t L, int n1, int n2, bool smooth, TableHost<T>* th) {
    const uint64_t NT = smooth ? (uint64_t)n1 : (uint64_t)(n1 > n2 ? n1 : n2);
    th->fshift = (log2_ceil(L) + 1) / 2;
    const uint64_t nfa = (L + (1ull << th->fshift) - 1) >> th->fshift;
    roots(th->tw, NT, NT, 1);
    if (smooth) roots(th->tw2, (uint64_t)n2, (uint64_t)n2, 1);
    roots(th->fa, nfa, L, 1ull << th->fshift);
    roots(th->fb, 1ull << th->fshift, L, 1);
    if (sizeof(T) < sizeof(double)) {
        roots(th->fa64, nfa, L, 1ull << th->fshift);
        roots(th->fb64, 1ull << th->fshift, L, 1);
    }
    // stage tables: size M, stage span Ns (> 1), radix 16: entry [k][r] = w_{16 Ns}^{k r}
    th->stw.assign(2 * (size_t)wfft_tables_total(), T(0));
    for (int lg = kWfftMinLog; lg <= kWfftMaxLog; ++lg) {
        const int M = 1 << lg;
        for (int ns = wfft_first_radix(M); ns < M; ns *= 16) {
            const size_t base = (size_t)wfft_size_offset(M) + wfft_stage_offset(M, ns);
            for (int k = 0; k < ns; ++k)
                for (int r = 0; r < 16; ++r) {
                    long double c, sn;
                    unit_root((uint64_t)k * r, (uint64_t)ns * 16, &c, &sn);
                    th->stw[2 * (base + k * 16 + r)] = (T)c;
                    th->stw[2 * (base + k * 16 + r) + 1] = (T)sn;
                }
        }
    }
}

template void build_tables<float>(uint64_t, int, int, bool, TableHost<float>*);

namespace {
constexpr uint64_t kP = 2013265921ull;  // 15 * 2^27 + 1
uint64_t mulmod(uint64_t a, uint64_t b) { return (a * b) % kP; }
uint64_t powmod(uint64_t a, uint64_t e) {
    uint64_t r = 1;
    a %= kP;
    while (e) {
        if (e & 1) r = mulmod(r, a);
        a = mulmod(a, a);
        e >>= 1;
    }
    return r;
}
uint32_t to_mont(uint64_t a) { return (uint32_t)(((a % kP) << 32) % kP); }
}  // namespace

void build_ntt_tables(uint64_t L, int n1, int n2, TableHost<uint32_t>* th) {
    const uint64_t NT = (uint64_t)(n1 > n2 ? n1 : n2);
    th->fshift = (log2_ceil(L) + 1) / 2;
    const uint64_t wNT = powmod(31, (kP - 1) / NT), wL = powmod(31, (kP - 1) / L);
    th->tw.resize(NT);
    uint64_t a = 1;
    for (uint64_t e = 0; e < NT; ++e, a = mulmod(a, wNT)) th->tw[e] = to_mont(a);
    const uint64_t nfa = L >> th->fshift, nfb = 1ull << th->fshift;
    th->fa.resize(nfa);
    th->fb.resize(nfb);
    const uint64_t step = powmod(wL, nfb);
    a = 1;
    for (uint64_t h = 0; h < nfa; ++h, a = mulmod(a, step)) th->fa[h] = to_mont(a);
    a = 1;
    for (uint64_t l = 0; l < nfb; ++l, a = mulmod(a, wL)) th->fb[l] = to_mont(a);
    th->stw = {(uint32_t)powmod(L, kP - 2), to_mont(1)};
}
template void build_tables<double>(uint64_t, int, int, bool, TableHost<double>*);

}  // namespace pa
