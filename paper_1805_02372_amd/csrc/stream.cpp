// Block-serial hashing (paper section 3, Fig. 1-3): the key is processed in
// blocks whose partial hashes are XOR-merged (Eq. 4-7), with the accumulator
// resident in device memory.  Each block is an ordinary job (planned as
// pa_hash plans it, on the block and its seed slice); its output lands in a
// scratch word array that a small kernel XORs into the accumulator.
//
// Blocks from host memory are pipelined over two staging slots: a feed copies
// its block into pinned memory and starts the DMA on a copy stream while the
// previous block's kernels still run, then checks the previous block's
// certificate (FP64 fallback as in pa_hash), merges it and enqueues its own
// block behind its DMA.  The last block is checked by the next call on the
// stream (feed, state, resume or close).  The stream has its own lane (GPU
// stream and workspace), so it runs beside the context's other calls.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "direct.hpp"
#include "engine.hpp"
#include "planner.hpp"

using namespace pa;

struct pa_stream {
    Ctx* c = nullptr;
    uint64_t n = 0, m = 0;
    uint32_t flags = 0;
    uint64_t fed = 0;
    DevBuf acc;                     // the accumulator
    StreamRes* r = nullptr;         // lane, copy stream, staging slots
    int slot = 0;                   // slot of the next host block
    // the block in flight: its kernels enqueued, its certificate not yet read
    bool pending = false, pending_fft = false;
    uint64_t pending_len = 0;
};

static uint64_t nwords(uint64_t bits) { return (bits + 63) >> 6; }

// Settle the block in flight: wait for it, check its certificate (FP64
// fallback of failed tiles) and merge it into the accumulator.  On an error
// the block is dropped (accumulator and fed count unchanged).
static pa_status drain(pa_stream* s) {
    if (!s->pending) return PA_OK;
    s->pending = false;
    if (s->pending_fft) {
        pa_stats st{};
        const pa_status r = s->r->ln.finish(s->c, s->flags & PA_NO_FALLBACK, &st, nullptr);
        if (r != PA_OK) return r;
        if (launch_xor_words((uint64_t*)s->acc.ptr, (const uint64_t*)s->r->part.ptr, nwords(s->m), s->r->ln.stream))
            return PA_EDEVICE;
    }
    s->fed += s->pending_len;
    return PA_OK;
}

// Enqueue the partial hash of one block (device pointers) into `part` on the
// stream's lane; a direct-product block is merged at once (it has no
// certificate), an FFT block when drained.
static pa_status launch_block(pa_stream* s, const uint64_t* dseed, const uint64_t* dkey, uint64_t len) {
    Ctx* c = s->c;
    const uint64_t m = s->m;
    const int policy = policy_of(s->flags);
    TilePlan plan;
    if (!c->plan_cached(len, m, policy, &plan)) return PA_EINVAL;
    CostModel cm;
    {
        std::lock_guard<std::mutex> pk(c->plan_mu);
        cm = c->cost;
    }
    pa_stats st{};
    uint64_t* out = (uint64_t*)s->r->part.ptr;
    if (choose_direct(s->flags, len, m, cm, plan)) {
        pa_status r = s->r->ln.direct(c, dseed, dkey, len, m, out, false, &st);
        if (r != PA_OK) return r;
        if (launch_xor_words((uint64_t*)s->acc.ptr, out, nwords(m), s->r->ln.stream)) return PA_EDEVICE;
        s->pending_fft = false;
    } else {
        std::vector<JobDesc> jobs(1);
        fill_job(&jobs[0], dseed, dkey, out, len, m, plan);
        pa_status r = s->r->ln.launch(c, plan.prec, plan.cls, jobs, false, true, &st);
        if (r != PA_OK) return r;
        s->pending_fft = true;
    }
    s->pending = true;
    s->pending_len = len;
    return PA_OK;
}

namespace pa {
void StreamRes::release(Ctx* c) {
    if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    if (copy) (void)hipStreamSynchronize(copy);
    part.release(c);
    for (int b = 0; b < 2; ++b) {
        in[b].release(c);
        pin[b].release();
    }
    ln.release(c);   // synchronises its stream (the frees above were queued on it)
    if (copy) {
        (void)hipStreamSynchronize(copy);
        (void)hipStreamDestroy(copy);
    }
    copy = nullptr;
    for (int b = 0; b < 2; ++b) {
        if (staged[b]) (void)hipEventDestroy(staged[b]);
        if (used[b]) (void)hipEventDestroy(used[b]);
        staged[b] = used[b] = nullptr;
    }
}
}  // namespace pa

// Resources for a new stream: a closed stream's, else new ones.
static pa_status take_res(Ctx* c, uint64_t m, StreamRes** out) {
    StreamRes* r = nullptr;
    {
        std::lock_guard<std::mutex> lk(c->stream_mu);
        if (!c->idle_streams.empty()) {
            r = c->idle_streams.back();
            c->idle_streams.pop_back();
        }
    }
    pa_status st = PA_OK;
    if (!r) {
        r = new StreamRes();
        if (hipStreamCreateWithFlags(&r->ln.stream, hipStreamNonBlocking) != hipSuccess) st = PA_EDEVICE;
        r->ln.own_stream = r->ln.stream != nullptr;
        if (st == PA_OK && hipStreamCreateWithFlags(&r->copy, hipStreamNonBlocking) != hipSuccess) st = PA_EDEVICE;
        for (int b = 0; b < 2 && st == PA_OK; ++b)
            if (hipEventCreateWithFlags(&r->staged[b], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&r->used[b], hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(r->staged[b], r->copy) != hipSuccess ||   // waits on them find them recorded
                hipEventRecord(r->used[b], r->ln.stream) != hipSuccess)
                st = PA_EDEVICE;
    }
    if (st == PA_OK) st = r->part.ensure(c, nwords(m) * 8, r->ln.stream);
    if (st != PA_OK) {
        r->release(c);
        delete r;
        return st;
    }
    *out = r;
    return PA_OK;
}

// Close: keep one set of resources for the next stream, free the rest.
static void free_stream(pa_stream* s) {
    Ctx* c = s->c;
    (void)hipSetDevice(c->device);
    if (s->r) {
        (void)hipStreamSynchronize(s->r->ln.stream);
        (void)hipStreamSynchronize(s->r->copy);
    }
    s->acc.release(c);
    if (s->r) {
        bool kept = false;
        {
            std::lock_guard<std::mutex> lk(c->stream_mu);
            if (c->idle_streams.empty()) {
                c->idle_streams.push_back(s->r);
                kept = true;
            }
        }
        if (!kept) {
            s->r->release(c);
            delete s->r;
        }
    }
    delete s;
}

extern "C" {

pa_status pa_stream_open(pa_ctx* ctx, uint64_t n, uint64_t m, uint32_t flags, pa_stream** out) {
    if (!ctx || !out || n == 0 || m == 0 || n > (1ull << 40) || m > (1ull << 40)) return PA_EINVAL;
    if (policy_of(flags) < 0) return PA_EINVAL;
    *out = nullptr;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    pa_stream* s = new pa_stream();
    s->c = c;
    s->n = n;
    s->m = m;
    s->flags = flags;
    pa_status st = take_res(c, m, &s->r);
    if (st == PA_OK) st = s->acc.ensure(c, nwords(m) * 8, s->r->ln.stream);
    // x ^ x = 0: clear the accumulator with the XOR kernel itself
    if (st == PA_OK &&
        launch_xor_words((uint64_t*)s->acc.ptr, (const uint64_t*)s->acc.ptr, nwords(m), s->r->ln.stream))
        st = PA_EDEVICE;
    if (st == PA_OK && hipStreamSynchronize(s->r->ln.stream) != hipSuccess) st = PA_EDEVICE;
    if (st != PA_OK) {
        free_stream(s);
        return st;
    }
    *out = s;
    return PA_OK;
}

pa_status pa_stream_feed(pa_stream* s, const uint64_t* key_block, uint64_t lo, uint64_t len,
                         const uint64_t* seed_block) {
    if (!s || !key_block || !seed_block || len == 0 || lo >= s->n || len > s->n - lo) return PA_EINVAL;
    Ctx* c = s->c;
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    const uint64_t kw = nwords(len), sw = nwords(len + s->m - 1);
    if (s->flags & PA_DEVICE_PTRS) {   // the caller's buffers, read before the call returns
        pa_status st = launch_block(s, seed_block, key_block, len);
        if (st == PA_OK) st = drain(s);
        if (hipStreamSynchronize(s->r->ln.stream) != hipSuccess && st == PA_OK) st = PA_EDEVICE;
        return st;
    }
    // Stage the block in slot b while the previous block runs: the slot's
    // pinned image is free once its last DMA is done, its device buffer once
    // the block that read it is done (the copy stream waits for that).
    const int b = s->slot;
    const size_t sbytes = sw * 8, off = (sbytes + 255) & ~(size_t)255, kbytes = kw * 8;
    if (hipEventSynchronize(s->r->staged[b]) != hipSuccess) return PA_EDEVICE;
    pa_status st = s->r->pin[b].ensure(off + kbytes);
    if (st == PA_OK && s->r->in[b].bytes < off + kbytes) {
        // a larger block: the old buffer may be freed only after its reader
        if (hipStreamWaitEvent(s->r->copy, s->r->used[b], 0) != hipSuccess) return PA_EDEVICE;
        st = s->r->in[b].ensure(c, off + kbytes, s->r->copy);
    }
    if (st != PA_OK) return st;
    unsigned char* h = (unsigned char*)s->r->pin[b].ptr;
    c->copier.copy(h, seed_block, sbytes);
    c->copier.copy(h + off, key_block, kbytes);
    if (hipStreamWaitEvent(s->r->copy, s->r->used[b], 0) != hipSuccess ||
        hipMemcpyAsync(s->r->in[b].ptr, h, off + kbytes, hipMemcpyHostToDevice, s->r->copy) != hipSuccess ||
        hipEventRecord(s->r->staged[b], s->r->copy) != hipSuccess)
        return PA_EDEVICE;
    // the previous block: certificate, fallback, merge; its error is this call's
    st = drain(s);
    if (st != PA_OK) return st;
    if (hipStreamWaitEvent(s->r->ln.stream, s->r->staged[b], 0) != hipSuccess) return PA_EDEVICE;
    const uint64_t* dseed = (const uint64_t*)s->r->in[b].ptr;
    const uint64_t* dkey = (const uint64_t*)((const unsigned char*)s->r->in[b].ptr + off);
    st = launch_block(s, dseed, dkey, len);
    if (hipEventRecord(s->r->used[b], s->r->ln.stream) != hipSuccess && st == PA_OK) st = PA_EDEVICE;
    s->slot ^= 1;
    return st;
}

pa_status pa_stream_state(pa_stream* s, uint64_t* acc, uint64_t* fed_bits) {
    if (!s) return PA_EINVAL;
    Ctx* c = s->c;
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    pa_status st = drain(s);
    if (st != PA_OK) return st;
    if (fed_bits) *fed_bits = s->fed;
    if (!acc) return PA_OK;
    const hipMemcpyKind kind = (s->flags & PA_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (hipMemcpyAsync(acc, s->acc.ptr, nwords(s->m) * 8, kind, s->r->ln.stream) != hipSuccess ||
        hipStreamSynchronize(s->r->ln.stream) != hipSuccess)
        return PA_EDEVICE;
    return PA_OK;
}

pa_status pa_stream_resume(pa_stream* s, const uint64_t* acc, uint64_t fed_bits) {
    if (!s || !acc || fed_bits > s->n) return PA_EINVAL;
    Ctx* c = s->c;
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    (void)drain(s);   // a block in flight is replaced with the rest of the state
    const hipMemcpyKind kind = (s->flags & PA_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (hipMemcpyAsync(s->acc.ptr, acc, nwords(s->m) * 8, kind, s->r->ln.stream) != hipSuccess ||
        hipStreamSynchronize(s->r->ln.stream) != hipSuccess)
        return PA_EDEVICE;
    s->fed = fed_bits;
    return PA_OK;
}

pa_status pa_stream_close(pa_stream* s, uint64_t* out) {
    if (!s) return PA_EINVAL;
    (void)hipSetDevice(s->c->device);
    pa_status st = drain(s);
    if (st == PA_OK && out) st = s->fed == s->n ? pa_stream_state(s, out, nullptr) : PA_EINVAL;
    free_stream(s);
    return st;
}

}  // extern "C"
