/*
 * CPU oracle for the Toeplitz hash over GF(2).  TEST INFRASTRUCTURE ONLY:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * it.  It shares no code, header or table with the GPU library: no FFT and no
 * floating point appear here.
 *
 * What it computes (paper section 2.1, Eq. 1, and section 2.3, steps 1-2):
 * the m x n Toeplitz matrix T over GF(2) is fixed by n+m-1 seed bits s[.] as
 *
 *        T[i][j] = s[i - j + n - 1],      0 <= i < m, 0 <= j < n,
 *
 * Every diagonal i - j = const carries one seed bit: the first row reads
 * s[n-1], s[n-2], ..., s[0] from left to right (s[0] is the top-right
 * corner), the first column s[n-1], s[n], ..., s[n+m-2] from top to bottom.
 * The hash of an n-bit key x is
 *
 *        y_i = XOR_{j=0}^{n-1} ( T[i][j] AND x_j ),   0 <= i < m.
 *
 * This ordering is the one under which the product is a window of the
 * polynomial product s(z) x(z): y_i is the coefficient of z^(i+n-1)
 * (section 3, step 3, read 1-based: outputs n .. n+m-1), and it uses every one
 * of the n+m-1 seed bits.
 *
 * Bit format: uint64 words, LSB-first (bit k is (w[k>>6] >> (k&63)) & 1).
 * Output bits at positions >= m in the last word are written as zero.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

static inline int get_bit(const uint64_t* w, uint64_t k) {
    return (int)((w[k >> 6] >> (k & 63)) & 1u);
}

static inline void put_bit(uint64_t* w, uint64_t k, int b) {
    uint64_t mask = (uint64_t)1 << (k & 63);
    if (b) w[k >> 6] |= mask; else w[k >> 6] &= ~mask;
}

/* Output word count for m bits. */
static inline uint64_t nwords(uint64_t nbits) { return (nbits + 63) >> 6; }

/*
 * O2: the definition, one bit at a time.  Cost n*m bit operations.
 */
void oracle_hash_bits(const uint64_t* seed, uint64_t n, uint64_t m,
                      const uint64_t* key, uint64_t* out) {
    memset(out, 0, nwords(m) * sizeof(uint64_t));
    for (uint64_t i = 0; i < m; ++i) {
        int acc = 0;
        for (uint64_t j = 0; j < n; ++j)
            acc ^= get_bit(seed, i - j + n - 1) & get_bit(key, j);
        put_bit(out, i, acc);
    }
}

/*
 * One output bit from the definition, 64 key bits at a time: with the key
 * reversed, xr[t] = x[n-1-t], the sum becomes y_i = XOR_t s[i+t] AND xr[t],
 * i.e. the parity of popcount(seed bits i..i+n-1 AND xr).  Cost n/64 word
 * steps.  `sp` is the seed padded with one zero word; `xr` the reversed key.
 */
static int one_output(const uint64_t* sp, const uint64_t* xr, uint64_t nkw, uint64_t i) {
    uint64_t acc = 0;
    uint64_t q = i >> 6;
    unsigned r = (unsigned)(i & 63);
    for (uint64_t k = 0; k < nkw; ++k) {
        uint64_t lo = sp[q + k], hi = sp[q + k + 1];
        uint64_t win = r ? ((lo >> r) | (hi << (64 - r))) : lo; /* seed bits i+64k .. i+64k+63 */
        acc ^= win & xr[k];
    }
    return __builtin_parityll(acc);
}

/* Reverse the n-bit key into xr (nkw words, zero tail). */
static void reverse_key(const uint64_t* key, uint64_t n, uint64_t* xr) {
    memset(xr, 0, nwords(n) * sizeof(uint64_t));
    for (uint64_t t = 0; t < n; ++t)
        if (get_bit(key, n - 1 - t)) xr[t >> 6] |= (uint64_t)1 << (t & 63);
}

/* Seed copy with its tail (bits >= n+m-1) cleared and one extra zero word. */
static uint64_t* padded_seed(const uint64_t* seed, uint64_t sbits) {
    uint64_t sw = nwords(sbits);
    uint64_t* sp = (uint64_t*)calloc(sw + 2, sizeof(uint64_t));
    if (!sp) return NULL;
    memcpy(sp, seed, sw * sizeof(uint64_t));
    if (sbits & 63) sp[sw - 1] &= ((uint64_t)1 << (sbits & 63)) - 1;
    return sp;
}

typedef struct {
    const uint64_t* sp;
    const uint64_t* xr;
    uint64_t nkw;
    uint64_t w_begin, w_end; /* output words [w_begin, w_end) */
    uint64_t m;
    uint64_t* out;
} job_t;

static void* worker(void* arg) {
    job_t* jb = (job_t*)arg;
    for (uint64_t w = jb->w_begin; w < jb->w_end; ++w) {
        uint64_t word = 0;
        for (unsigned b = 0; b < 64; ++b) {
            uint64_t i = (w << 6) + b;
            if (i >= jb->m) break;
            word |= (uint64_t)one_output(jb->sp, jb->xr, jb->nkw, i) << b;
        }
        jb->out[w] = word;
    }
    return NULL;
}

/*
 * O3: the same definition evaluated 64 key bits per step, split over
 * `threads` host threads by output word ranges.  Cost about n*m/64 word steps.
 * Returns 0 on success, -1 on allocation failure.
 */
int oracle_hash_words(const uint64_t* seed, uint64_t n, uint64_t m,
                      const uint64_t* key, uint64_t* out, int threads) {
    uint64_t nkw = nwords(n), mw = nwords(m);
    uint64_t* sp = padded_seed(seed, n + m - 1);
    uint64_t* xr = (uint64_t*)calloc(nkw + 1, sizeof(uint64_t));
    if (!sp || !xr) { free(sp); free(xr); return -1; }
    reverse_key(key, n, xr);
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > mw) threads = (int)mw;
    pthread_t* th = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    job_t* jobs = (job_t*)calloc((size_t)threads, sizeof(job_t));
    if (!th || !jobs) { free(sp); free(xr); free(th); free(jobs); return -1; }
    for (int t = 0; t < threads; ++t) {
        jobs[t].sp = sp; jobs[t].xr = xr; jobs[t].nkw = nkw; jobs[t].m = m; jobs[t].out = out;
        jobs[t].w_begin = mw * (uint64_t)t / (uint64_t)threads;
        jobs[t].w_end = mw * (uint64_t)(t + 1) / (uint64_t)threads;
    }
    char* live = (char*)calloc((size_t)threads, 1);
    for (int t = 1; t < threads; ++t) {
        if (live && pthread_create(&th[t], NULL, worker, &jobs[t]) == 0) live[t] = 1;
        else worker(&jobs[t]);  /* no thread: do the range here */
    }
    worker(&jobs[0]);
    for (int t = 1; t < threads; ++t)
        if (live && live[t]) pthread_join(th[t], NULL);
    free(live);
    free(th); free(jobs); free(sp); free(xr);
    return 0;
}

/*
 * Selected output bits y_{idx[k]} (k < count) by the word-parallel
 * definition; for spot checks of outputs too large to hash in full.
 * Writes 0/1 bytes into bits_out.  Returns 0, or -1 on allocation failure.
 */
int oracle_hash_select(const uint64_t* seed, uint64_t n, uint64_t m,
                       const uint64_t* key, const uint64_t* idx, uint64_t count,
                       uint8_t* bits_out) {
    uint64_t nkw = nwords(n);
    uint64_t* sp = padded_seed(seed, n + m - 1);
    uint64_t* xr = (uint64_t*)calloc(nkw + 1, sizeof(uint64_t));
    if (!sp || !xr) { free(sp); free(xr); return -1; }
    reverse_key(key, n, xr);
    for (uint64_t k = 0; k < count; ++k)
        bits_out[k] = (uint8_t)(idx[k] < m ? one_output(sp, xr, nkw, idx[k]) : 0);
    free(sp); free(xr);
    return 0;
}
