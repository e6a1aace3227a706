// Block-serial hashing (paper section 3, Fig. 1-3): the key is processed in
// blocks whose partial hashes are XOR-merged (Eq. 4-7), with the accumulator
// resident in device memory.  Each block is an ordinary job on the context
// (pa_hash on the block and its seed slice); its output lands in a scratch
// word array that a small kernel XORs into the accumulator.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "direct.hpp"
#include "engine.hpp"

using namespace pa;

struct pa_stream {
    Ctx* c = nullptr;
    uint64_t n = 0, m = 0;
    uint32_t flags = 0;
    uint64_t fed = 0;
    DevBuf acc, part, in;   // accumulator, block output, staged block inputs
};

static uint64_t nwords(uint64_t bits) { return (bits + 63) >> 6; }

extern "C" {

pa_status pa_stream_open(pa_ctx* ctx, uint64_t n, uint64_t m, uint32_t flags, pa_stream** out) {
    if (!ctx || !out || n == 0 || m == 0 || n > (1ull << 40) || m > (1ull << 40)) return PA_EINVAL;
    if (policy_of(flags) < 0) return PA_EINVAL;
    *out = nullptr;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    pa_stream* s = new pa_stream();
    s->c = c;
    s->n = n;
    s->m = m;
    s->flags = flags;
    std::lock_guard<std::mutex> lk(c->mu);
    pa_status st = hipSetDevice(c->device) == hipSuccess ? PA_OK : PA_EDEVICE;
    if (st == PA_OK) st = s->acc.ensure(c, nwords(m) * 8, c->main.stream);
    if (st == PA_OK) st = s->part.ensure(c, nwords(m) * 8, c->main.stream);
    // x ^ x = 0: clear the accumulator with the XOR kernel itself
    if (st == PA_OK && launch_xor_words((uint64_t*)s->acc.ptr, (const uint64_t*)s->acc.ptr, nwords(m), c->main.stream))
        st = PA_EDEVICE;
    if (st == PA_OK && hipStreamSynchronize(c->main.stream) != hipSuccess) st = PA_EDEVICE;
    if (st != PA_OK) {
        s->acc.release(c);
        s->part.release(c);
        delete s;
        return st;
    }
    *out = s;
    return PA_OK;
}

pa_status pa_stream_feed(pa_stream* s, const uint64_t* key_block, uint64_t lo, uint64_t len,
                         const uint64_t* seed_block) {
    if (!s || !key_block || !seed_block || len == 0 || lo >= s->n || len > s->n - lo) return PA_EINVAL;
    Ctx* c = s->c;
    const uint64_t m = s->m, kw = nwords(len), sw = nwords(len + m - 1);
    const uint64_t *dseed = seed_block, *dkey = key_block;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
        if (!(s->flags & PA_DEVICE_PTRS)) {   // stage the block in device memory
            pa_status st = s->in.ensure(c, (sw + kw) * 8, c->main.stream);
            if (st != PA_OK) return st;
            uint64_t* base = (uint64_t*)s->in.ptr;
            void* dsts[2] = {base, base + sw};
            const void* srcs[2] = {seed_block, key_block};
            const size_t lens[2] = {sw * 8, kw * 8};
            st = stage_in(c, c->main, dsts, srcs, lens, 2);   // pinned staging, multi-threaded copy
            // the staging buffer is the context's: the copies land before the lock is released
            if (st == PA_OK && hipStreamSynchronize(c->main.stream) != hipSuccess) st = PA_EDEVICE;
            if (st != PA_OK) return st;
            dseed = base;
            dkey = base + sw;
        }
    }
    // the block's partial hash (Eq. 4-6) into `part`; stream order follows the copies
    const uint32_t f = (s->flags & (PA_PREC_MASK | PA_NO_FALLBACK)) | PA_DEVICE_PTRS;
    pa_status st = pa_hash(reinterpret_cast<pa_ctx*>(c), dseed, len, m, dkey, (uint64_t*)s->part.ptr, f);
    if (st != PA_OK) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    if (launch_xor_words((uint64_t*)s->acc.ptr, (const uint64_t*)s->part.ptr, nwords(m), c->main.stream) ||
        hipStreamSynchronize(c->main.stream) != hipSuccess)
        return PA_EDEVICE;
    s->fed += len;
    return PA_OK;
}

pa_status pa_stream_state(pa_stream* s, uint64_t* acc, uint64_t* fed_bits) {
    if (!s) return PA_EINVAL;
    if (fed_bits) *fed_bits = s->fed;
    if (!acc) return PA_OK;
    Ctx* c = s->c;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    const hipMemcpyKind kind = (s->flags & PA_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (hipMemcpyAsync(acc, s->acc.ptr, nwords(s->m) * 8, kind, c->main.stream) != hipSuccess ||
        hipStreamSynchronize(c->main.stream) != hipSuccess)
        return PA_EDEVICE;
    return PA_OK;
}

pa_status pa_stream_resume(pa_stream* s, const uint64_t* acc, uint64_t fed_bits) {
    if (!s || !acc || fed_bits > s->n) return PA_EINVAL;
    Ctx* c = s->c;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    const hipMemcpyKind kind = (s->flags & PA_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (hipMemcpyAsync(s->acc.ptr, acc, nwords(s->m) * 8, kind, c->main.stream) != hipSuccess ||
        hipStreamSynchronize(c->main.stream) != hipSuccess)
        return PA_EDEVICE;
    s->fed = fed_bits;
    return PA_OK;
}

pa_status pa_stream_close(pa_stream* s, uint64_t* out) {
    if (!s) return PA_EINVAL;
    pa_status st = PA_OK;
    if (out) st = s->fed == s->n ? pa_stream_state(s, out, nullptr) : PA_EINVAL;
    Ctx* c = s->c;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        (void)hipSetDevice(c->device);
        s->acc.release(c);
        s->part.release(c);
        s->in.release(c);
    }
    delete s;
    return st;
}

}  // extern "C"
