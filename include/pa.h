/*
 * libpa — Toeplitz-hash privacy amplification on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper section 2.1, Eq. 1; section 2.3, steps 1-2; section 3,
 * Fig. 1-2, Eq. 4-7): for an n-bit key x and an (n+m-1)-bit seed s, the m x n
 * Toeplitz matrix over GF(2) has T[i][j] = s[i - j + n - 1], and the hash is
 *
 *     y_i = XOR_{j<n} ( s[i - j + n - 1] AND x_j ),   0 <= i < m.
 *
 * y is the window [n-1, n+m-1) of the polynomial product s(z) x(z) reduced mod
 * 2 (section 3, step 3: outputs n .. n+m-1 of the product, counted from 1;
 * Eq. 7: mod-2 addition).  The library evaluates it as an exact FFT convolution
 * (integer rounding, parity, output window), splitting long keys into chunks
 * and long outputs into windows whose partial hashes are XOR-merged (Eq. 4-7).
 *
 * Bit strings: arrays of uint64_t words, LSB-first: bit k of a string is
 * (w[k >> 6] >> (k & 63)) & 1.  A k-bit string occupies ceil(k/64) words.
 * Bits beyond n (key) or n+m-1 (seed) in the last word are ignored.  Output
 * bits beyond m in the last word are written as 0.
 *
 * Memory: unless PA_DEVICE_PTRS is given, seed/key/out are host pointers and
 * the call copies them (and the call is synchronous).  With PA_DEVICE_PTRS they
 * are device pointers on the context's device (e.g. a torch tensor's
 * data_ptr()).  The context's stream is not ordered after other streams:
 * device buffers written on another stream must be complete (synchronized,
 * or the context created on that stream) before a call uses them.  The caller owns seed, key and out and keeps them alive until the
 * call has completed; out must not overlap seed or key.  The library owns its
 * workspace, plans, twiddle tables, tuning data and copies of registered
 * seeds.
 *
 * Errors: every entry point returns a pa_status; nothing is thrown across the
 * ABI.  A context is used by one host thread at a time (calls on one context
 * are serialised by an internal mutex).
 */
#ifndef PA_H
#define PA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PA_OK = 0,
    PA_EINVAL = 1,       /* n == 0, m == 0, NULL pointer, bad flags, unknown id */
    PA_ENOMEM = 2,       /* the job cannot fit the HBM budget even when tiled    */
    PA_EDEVICE = 3,      /* a HIP runtime error (no device, launch failure, ...) */
    PA_EPRECISION = 4,   /* a floating-point certificate failed, fallback off    */
    PA_EBUSY = 5,        /* serving queue full                                   */
    PA_ENOTREADY = 6,    /* ticket not finished (pa_poll)                         */
    PA_ESCRATCH = 7      /* pa_hash_noalloc: the job exceeds its fixed scratch    */
} pa_status;

/* ---- flags ---------------------------------------------------------------- */
#define PA_DEVICE_PTRS    0x0001u  /* seed/key/out are device pointers                 */
#define PA_PREC_AUTO      0x0000u  /* fastest exact plan: the direct product where it is
                                      modeled cheaper (short outputs), else FP32 tiles
                                      with FP64 fallback                                */
#define PA_PREC_FP32_SEG  0x0010u  /* FP32 FFT tiles sized by the rounding bound        */
#define PA_PREC_FP64      0x0020u  /* FP64 FFT, one tile where it fits ("plain" path)   */
#define PA_PREC_NTT       0x0030u  /* exact number-theoretic transform mod 15*2^27+1    */
#define PA_PREC_DIRECT    0x0040u  /* exact word-parallel GF(2) product, no transform:
                                      ceil(n/32) word steps per output (short outputs) */
#define PA_PREC_MASK      0x00F0u
#define PA_NO_FALLBACK    0x0100u  /* report PA_EPRECISION instead of re-running FP64   */
#define PA_ASYNC          0x0200u  /* with PA_DEVICE_PTRS and an exact or a-priori
                                      certified plan (FP64, NTT, direct): return once
                                      enqueued                                          */
#define PA_TIMING         0x0400u  /* record per-kernel durations (pa_last_stats)       */

typedef struct pa_ctx pa_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * workspace (0 = 8 GiB).  hip_stream: a hipStream_t to run on, or NULL for a
 * stream owned by the context.  Returns PA_EDEVICE when no usable device. */
pa_status pa_create(pa_ctx** ctx, int device, uint64_t hbm_budget_bytes, void* hip_stream);

/* Destroy a context (waits for its work, frees its memory).  NULL is a no-op. */
void pa_destroy(pa_ctx* ctx);

/* y = T(seed) * key over GF(2), m output bits (see top of file).
 * seed: n+m-1 bits; key: n bits; out: m bits (ceil(m/64) words, written).
 * Synchronous unless PA_ASYNC applies.  PA_EINVAL for n == 0, m == 0, NULL
 * pointers, an unknown precision, n or m above 2^40, or m above 2^38 (a plan
 * has at most 2^14 output windows of at most 2^24 bits); PA_ENOMEM when even
 * the smallest tiling exceeds the budget; PA_EPRECISION when a certificate
 * fails and PA_NO_FALLBACK is set. */
pa_status pa_hash(pa_ctx* ctx, const uint64_t* seed, uint64_t n, uint64_t m,
                  const uint64_t* key, uint64_t* out, uint32_t flags);

/* pa_hash for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * operation, kernels and results as pa_hash with PA_DEVICE_PTRS; the call
 * itself makes no hipMalloc, hipFree or other device or pinned allocation.
 * The workspace, per-tile sums, certificates and twiddle tables live in one
 * fixed array in device memory, about 137 MiB, that every GPU the library runs
 * on holds until the process ends (its address is taken once per device when
 * a context is created there).
 * - seed, key, out: device pointers; flags must include PA_DEVICE_PTRS
 *   (PA_EINVAL otherwise).  Precision bits, PA_NO_FALLBACK and PA_ASYNC as
 *   for pa_hash; PA_TIMING is ignored.
 * - Limits: FFT tiles of at most 2^23 points (so a failed FP32 tile can be
 *   re-run in FP64 within the workspace), at most 16384 tiles per job, and
 *   keys of at most 2^30 bits on the direct path; a job beyond them returns
 *   PA_ESCRATCH before any work is queued.
 * - Every call on one GPU shares that GPU's array, which keeps the last
 *   call's contents.  Calls are serialised per device on the host, but calls
 *   whose device work overlaps (PA_ASYNC, or contexts on different streams)
 *   race on the array: order them on one stream or wait for each.
 * - The first call for a length class builds its twiddle tables on the host
 *   and copies them into the array (at most 8 classes are held; the least
 *   recently used is replaced).
 * pa_last_stats describes the call as for pa_hash. */
pa_status pa_hash_noalloc(pa_ctx* ctx, const uint64_t* seed, uint64_t n, uint64_t m,
                          const uint64_t* key, uint64_t* out, uint32_t flags);

/* One job of a batch. */
typedef struct {
    const uint64_t* seed;   /* n+m-1 bits */
    const uint64_t* key;    /* n bits     */
    uint64_t* out;          /* m bits     */
    uint64_t n, m;
} pa_job;

/* Hash `count` independent jobs (uneven n and m): the paper runs the batches
 * of a long key in parallel on the GPU and queues later work behind them
 * (section 3, Fig. 2; section 4).  Here jobs are grouped by FFT
 * length class (each job's cheapest class, groups folded together while that
 * lowers the summed cost); each group runs as one launch per pipeline pass for
 * all its tiles.  The groups run concurrently on the context's stream and on
 * PA_BATCH_LANES - 1 side streams of the context (default 2 streams in all),
 * forked from the context's stream.  Tile and segment sizes come from the cost
 * model (tuned when pa_tune ran).  Jobs that the precision bits put on the
 * direct path (PA_PREC_DIRECT, or PA_PREC_AUTO where it is modeled cheaper)
 * run on the context's stream beside the groups.  pa_last_stats then names
 * the largest class used and counts the direct jobs.
 * per_job (optional, count entries) receives each job's status; the return
 * value is PA_OK only if every job succeeded.  Pointer kind per PA_DEVICE_PTRS
 * as for pa_hash.  Synchronous. */
pa_status pa_hash_batch(pa_ctx* ctx, const pa_job* jobs, uint64_t count, uint32_t flags,
                        pa_status* per_job);

/* Output bits y[idx[k]], k < count, computed exactly by the direct GF(2)
 * product (section 2.1, Eq. 1: each bit is the parity of the seed window at
 * idx[k] AND-ed with the reversed key), which shares nothing with the FFT
 * path: an on-device check of any chosen outputs.  seed (n+m-1 bits) and key
 * (n bits) as for pa_hash (PA_DEVICE_PTRS); idx (count indices < m) and bits
 * (count bytes, each 0 or 1, written) are host arrays.  count <= 2^20; count
 * == 0 is a no-op.  Synchronous.  PA_EINVAL for an index >= m, NULL pointers
 * or count > 2^20. */
pa_status pa_hash_select(pa_ctx* ctx, const uint64_t* seed, uint64_t n, uint64_t m, const uint64_t* key,
                         const uint64_t* idx, uint64_t count, uint8_t* bits, uint32_t flags);

/* ---- block-serial hashing (section 3, Fig. 1-3, Eq. 4-7) --------------------
 * The key arrives in blocks, from host or device memory, and each block's
 * partial hash is XOR-accumulated into an m-bit accumulator kept in device
 * memory.  Key bits [lo, lo+len) meet only seed bits [n-lo-len, n-lo+m-1)
 * (len+m-1 bits): the block's partial hash is the hash of that seed slice with
 * the block (Eq. 4-6), and the hash of the key is the XOR of the partial
 * hashes of blocks that cover it once (Eq. 7).  Blocks may come in any order
 * and have any lengths.  The accumulator can be read and restored, so a job
 * can resume at any block boundary. */
typedef struct pa_stream pa_stream;

/* Open a stream for an (n, m) job.  flags: the precision bits used for every
 * block (as for pa_hash) and PA_DEVICE_PTRS when the pointers given to
 * pa_stream_feed / _state / _resume / _close are device pointers.  The
 * accumulator starts at zero.  The stream has a GPU stream and workspace of
 * its own (charged to the context's budget), so it may run beside other calls
 * on the context; calls on one stream must not overlap.  It must be closed
 * before the context is destroyed.  PA_EINVAL for
 * n == 0, m == 0 or NULL; PA_ENOMEM when the accumulator does not fit the
 * context's budget. */
pa_status pa_stream_open(pa_ctx* ctx, uint64_t n, uint64_t m, uint32_t flags, pa_stream** stream);

/* XOR the partial hash of key bits [lo, lo+len) into the accumulator.
 * key_block: len bits, bit 0 = key bit lo.  seed_block: len+m-1 bits, bit 0 =
 * seed bit n-lo-len.  The inputs may be reused on return.  Host blocks are
 * pipelined: the call copies its block to the device and returns while the
 * block's kernels may still run; the block's certificate is read (FP64
 * fallback as in pa_hash) by the next call on the stream (feed, state or
 * close).  A block that fails there (PA_EPRECISION, PA_EDEVICE) is dropped:
 * that call returns its error and does nothing else (a feed's own block is
 * not fed), and the accumulator and fed count stay without it, so the caller
 * can read the state and feed the blocks again.  Device-pointer blocks are
 * hashed and checked before the call returns.  PA_EINVAL for len == 0,
 * lo+len > n or NULL pointers; errors of pa_hash otherwise (the block is then
 * not fed). */
pa_status pa_stream_feed(pa_stream* stream, const uint64_t* key_block, uint64_t lo, uint64_t len,
                         const uint64_t* seed_block);

/* Copy the accumulator (ceil(m/64) words) to acc and the number of key bits
 * fed so far to *fed_bits (either may be NULL), after the block in flight.
 * Synchronous.  The error of a block in flight that fails (see
 * pa_stream_feed) is returned instead, with nothing written. */
pa_status pa_stream_state(pa_stream* stream, uint64_t* acc, uint64_t* fed_bits);

/* Replace the accumulator by acc (ceil(m/64) words, e.g. a saved state) and
 * the fed-bit count by fed_bits; a block in flight is completed and replaced
 * with the rest.  PA_EINVAL for fed_bits > n or NULL acc. */
pa_status pa_stream_resume(pa_stream* stream, const uint64_t* acc, uint64_t fed_bits);

/* Write the hash (m bits) to out unless out is NULL, and free the stream.
 * With out != NULL, PA_EINVAL (and nothing written) unless exactly n key bits
 * were fed; the error of a failing block in flight is returned likewise.  The
 * stream is freed in every case. */
pa_status pa_stream_close(pa_stream* stream, uint64_t* out);

/* ---- serving (continuous batching) ---------------------------------------
 * The paper has no serving passage; it motivates real-time hashing of keys
 * that are already resident on the GPU (section 3).  Requests are hashed
 * exactly as pa_hash with PA_PREC_AUTO would hash them: short outputs by the
 * direct product, the rest by FP32 tiles with FP64 fallback. */

/* Copy a seed of nbits bits (device pointer if PA_DEVICE_PTRS in flags, else
 * host) into library-owned device memory and return its id.  Requests that
 * name the id use its first n+m-1 bits. */
pa_status pa_seed_register(pa_ctx* ctx, const uint64_t* seed, uint64_t nbits, uint32_t flags,
                           uint32_t* seed_id);

/* Queue a hash request against a registered seed.  key (n bits) and out (m
 * bits) are device pointers that stay valid until the ticket completes.
 * Requests are admitted to the device as the HBM budget allows and are
 * batched with whatever else is waiting; a request that arrives while others
 * run joins the next launch.  PA_EBUSY when the queue is full, PA_EINVAL when
 * n+m-1 exceeds the seed. */
pa_status pa_submit(pa_ctx* ctx, uint32_t seed_id, uint64_t n, uint64_t m,
                    const uint64_t* key, uint64_t* out, uint64_t* ticket);

/* done = 1 when the ticket's output is complete, else 0. */
pa_status pa_poll(pa_ctx* ctx, uint64_t ticket, int* done);

/* Block until the ticket completes; returns the request's status. */
pa_status pa_wait(pa_ctx* ctx, uint64_t ticket);

/* Latency of a finished ticket in seconds (submit -> completion seen). */
pa_status pa_ticket_latency(pa_ctx* ctx, uint64_t ticket, double* seconds);

/* Forget a finished ticket: its record (status, latency) is freed and the
 * ticket becomes unknown to pa_poll / pa_wait / pa_ticket_latency.  A
 * long-running service releases every ticket once it has read it; records of
 * unreleased tickets live until pa_destroy (pa_serve_stats counts them).
 * PA_ENOTREADY while the ticket runs, PA_EINVAL for an unknown ticket. */
pa_status pa_ticket_release(pa_ctx* ctx, uint64_t ticket);

/* ---- statistics ----------------------------------------------------------- */

/* How a result is known to be exact (pa_stats.certified). */
#define PA_CERT_NONE          0u  /* no result (error, or nothing ran)              */
#define PA_CERT_EXACT         1u  /* integer arithmetic only (NTT, direct product)   */
#define PA_CERT_A_PRIORI      2u  /* every floating-point tile is within the worst-case
                                     rounding bound (rigorous_bound < 0.5): rigorously
                                     certified for any input bits                     */
#define PA_CERT_A_POSTERIORI  3u  /* some FP32 tile is not covered by the worst-case
                                     bound; each such tile passed its run-time check
                                     (max |z - rint z| <= 1/8, |z| < 2^20, even
                                     rint z + weight, finite) or was re-run in FP64   */

typedef struct {
    uint32_t prec;            /* PA_PREC_* of the plan that ran               */
    uint32_t log2_len;        /* ceil(log2 L) of the FFT length L             */
    uint32_t n1, n2;          /* L = n1 * n2 (row and column lengths)         */
    uint64_t chunk_bits;      /* key bits per tile (Bi)                       */
    uint64_t window_bits;     /* output bits per tile (Bo)                    */
    uint64_t tiles;           /* tiles run                                    */
    uint64_t fallback_tiles;  /* tiles re-run in FP64 after a failed check    */
    double max_residual;      /* max |z - rint z| over all outputs            */
    double max_abs;           /* max |z| over all outputs                     */
    double bound;             /* predicted max error of the plan              */
    double ms_pass[4];        /* PA_TIMING: summed kernel ms of pass 1, 2, 3; [3] is 0
                                 (key chunks are XOR-merged inside pass 3).
                                 Direct path: [0] key reversal, [1] product */
    uint64_t model_bytes;     /* algorithmic HBM bytes of the FFT passes (direct
                                 path: seed, key and output once)             */
    uint64_t launches;        /* kernel launches                              */
    uint64_t direct_jobs;     /* jobs that ran on the direct path (prec is
                                 PA_PREC_DIRECT when all of them did)         */
    double rigorous_bound;    /* worst-case error bound of the FP plan (for any
                                 input bits); 0 for exact paths              */
    uint32_t certified;       /* how the result is known exact: PA_CERT_*     */
    uint32_t fft_len;         /* the FFT length L: 2^k, or 3, 5 or 7 times 2^k
                                 (mixed-radix classes, FP32 and FP64)        */
    uint64_t live_requests;   /* pa_serve_stats: request records held (queued,
                                 running, or finished and not yet released)  */
} pa_stats;

/* Statistics of the last pa_hash / pa_hash_batch on this context. */
pa_status pa_last_stats(pa_ctx* ctx, pa_stats* stats);

/* Statistics summed over the serving launches finished so far: tiles,
 * fallback_tiles (FP32 tiles re-run in FP64), launches, model_bytes, and the
 * largest max_residual / max_abs.  The plan fields are not set. */
pa_status pa_serve_stats(pa_ctx* ctx, pa_stats* stats);

/* Human-readable name of a status. */
const char* pa_strerror(pa_status status);

/* ---- tuning ----------------------------------------------------------------- */

/* Measure the cost of a tile of every FFT length class 2^12..2^24 (section
 * 3, step 2: the planner picks block and batch sizes from measured costs) for
 * the precisions selected by flags (PA_PREC_AUTO: FP32 and FP64; otherwise the
 * one named), with `reps` timed runs each on synthetic bits, and use the
 * results in this context's planner.  Each class runs one launch with one tile
 * and one with four: the marginal cost per tile goes to the class and the
 * remainder (median over classes) to the per-launch cost.  With PA_PREC_AUTO
 * or PA_PREC_DIRECT it also times the direct GF(2) path at two output lengths
 * and takes the slope as its cost per output and key word (PA_PREC_DIRECT
 * times only that).  If path is not NULL the table is also written there as
 * JSON ({"launch": seconds, "direct": seconds, "fp32": {"12": seconds, ...},
 * ...}).  Synchronous; PA_EDEVICE on a HIP error, PA_EINVAL for
 * a file that cannot be written. */
pa_status pa_tune(pa_ctx* ctx, uint32_t flags, int reps, const char* path);

/* Load a table written by pa_tune into this context's planner.  A context
 * also loads the file named by the PA_TUNE_CACHE environment variable when it
 * is created.  PA_EINVAL when the file is missing or malformed. */
pa_status pa_tune_load(pa_ctx* ctx, const char* path);

/* ---- host-only planning (no device needed) --------------------------------- */

typedef struct {
    uint32_t prec;        /* PA_PREC_FP32_SEG or PA_PREC_FP64 (or NTT)  */
    uint32_t log2_len;    /* ceil(log2 L)                                */
    uint32_t n1, n2;
    uint64_t chunk_bits;  /* Bi: key bits per chunk (last chunk may be shorter) */
    uint64_t window_bits; /* Bo: output bits per window, multiple of 64 unless it is m */
    uint64_t chunks;      /* ceil(n / Bi) */
    uint64_t windows;     /* ceil(m / Bo) */
    double bound;         /* predicted max error (probabilistic model)  */
    double cost;          /* model cost used to choose the plan          */
    double direct_cost;   /* model cost of the direct path for (n, m)    */
    uint32_t direct;      /* 1: the flags run (n, m) on the direct path; the
                             fields above still describe the FFT plan   */
    uint32_t fft_len;     /* FFT length L of a tile                      */
    double rigorous_bound; /* worst-case rounding bound of one tile of the plan,
                              for any input bits (0 for NTT); below 0.5 the plan
                              is certified a priori                      */
} pa_plan;

/* The plan pa_hash would use for (n, m) under the precision bits of flags,
 * with the starting cost model of a new context (the MI355X table shipped
 * beside the library, or the built-in model when PA_TUNE_DEFAULT=0; no
 * pa_tune data, no device).  Tile k (chunk b =
 * k / windows, window o = k % windows) covers key bits [max(0, n-(b+1)Bi),
 * n-b*Bi) and outputs [o*Bo, min(m, (o+1)*Bo)). */
pa_status pa_plan_query(uint64_t n, uint64_t m, uint32_t flags, pa_plan* plan);

/* Predicted max rounding error of one FP tile (probabilistic model with the
 * calibration constant in use), for chunk Bi and FFT length 2^log2_len. */
double pa_error_model(uint32_t prec, uint32_t log2_len, uint64_t chunk_bits);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
