// pa_hash_noalloc: pa_hash for callers that cannot allocate device memory.
//
// Everything the kernels need beyond the caller's inputs and output lives in
// one file-scope device array, `scratch`, of fixed size (each GPU that the
// library runs on holds its own copy until the process ends):
//
//   [0, 132 MiB)            tile workspace (pass 1 -> 2 -> 3: two FP32 tiles
//                           of 2^23 points with their 2 MiB bit planes), or
//                           the reversed key of the direct product
//   + 512 KiB               per-tile partial key weights (pass 1 -> 2)
//   + 256 KiB               per-tile certificates (at most 16384 tiles)
//   + 8 x 512 KiB           twiddle tables of up to 8 length classes
//
// Host code never passes the array's name to a kernel: set-up takes its device
// address with hipGetSymbolAddress once per device (pa_create, with the device
// current) and every use goes through that address.  The kernels are those of
// pa_hash; the plan is capped at 2^23-point tiles so that the FP64 re-run of a
// failed FP32 tile (16 bytes per point) fits the workspace.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "direct.hpp"
#include "engine.hpp"

namespace {
constexpr size_t kWsBytes = 132ull << 20;
constexpr size_t kPartBytes = 512ull << 10;
constexpr size_t kMetaBytes = 256ull << 10;
constexpr size_t kTabSlotBytes = 512ull << 10;
constexpr int kTabSlots = 8;
constexpr size_t kScratchBytes = kWsBytes + kPartBytes + kMetaBytes + kTabSlots * kTabSlotBytes;
constexpr int kCapLogL = 23;
constexpr int kMaxDevices = 16;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace pa {

namespace {

struct TabSlot {
    int prec = 0, cls = 0;    // class held (prec 0: empty)
    uint64_t used = 0;        // last use (eviction order)
    Tables t{};
};

struct NoAllocDev {
    std::mutex mu;            // one call at a time per device (host side)
    bool ready = false;
    unsigned char* ptr = nullptr;   // device address of `scratch` on this device
    Lane lane;                      // fixed views of the array
    TabSlot slots[kTabSlots];
    uint64_t clock = 0;
    alignas(64) unsigned char meta_host[kMetaBytes];   // certificates read back
};

NoAllocDev g_dev[kMaxDevices];

void fixed_view(DevBuf* b, void* p, size_t bytes) {
    b->ptr = p;
    b->bytes = bytes;
    b->owner = nullptr;
    b->fixed = true;
}

}  // namespace

pa_status noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return PA_EDEVICE;
    NoAllocDev& d = g_dev[device];
    std::lock_guard<std::mutex> lk(d.mu);
    if (d.ready) return PA_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return PA_EDEVICE;
    }
    if (hipEventCreateWithFlags(&d.lane.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return PA_EDEVICE;
    }
    d.ptr = (unsigned char*)p;
    Lane& ln = d.lane;
    fixed_view(&ln.ws, d.ptr, kWsBytes);
    fixed_view(&ln.aux, d.ptr, kWsBytes);   // the direct path uses no tile workspace
    fixed_view(&ln.part, d.ptr + kWsBytes, kPartBytes);
    fixed_view(&ln.meta, d.ptr + kWsBytes + kPartBytes, kMetaBytes);
    fixed_view(&ln.jobs_dev, nullptr, 0);   // one job per call: descriptors go by value
    fixed_view(&ln.io, nullptr, 0);         // device pointers only: nothing to stage
    ln.meta_host.ptr = d.meta_host;
    ln.meta_host.bytes = kMetaBytes;
    ln.meta_host.fixed = true;
    ln.jobs_host.fixed = true;
    ln.static_tables = true;
    d.ready = true;
    return PA_OK;
}

// Tables of class (prec, cls) in one of the array's table slots.  The caller
// holds the device's mutex.  A class not held yet is built on the host and
// copied into the least recently used slot in the order of the lane's stream
// (after the kernels already queued there).
pa_status noalloc_tables(int device, int prec, int cls, Tables* out) {
    if (device < 0 || device >= kMaxDevices || !g_dev[device].ready) return PA_EDEVICE;
    NoAllocDev& d = g_dev[device];
    TabSlot* victim = &d.slots[0];
    for (TabSlot& s : d.slots) {
        if (s.prec == prec && s.cls == cls) {
            s.used = ++d.clock;
            *out = s.t;
            return PA_OK;
        }
        if (s.used < victim->used) victim = &s;
    }
    std::vector<unsigned char> host;
    size_t off[kTableSections];
    int fshift = 0;
    pa_status st = table_image(prec, cls, &host, off, &fshift);
    if (st != PA_OK) return st;
    if (host.size() > kTabSlotBytes) return PA_ESCRATCH;
    unsigned char* base = d.ptr + kWsBytes + kPartBytes + kMetaBytes + (size_t)(victim - d.slots) * kTabSlotBytes;
    if (hipMemcpyAsync(base, host.data(), host.size(), hipMemcpyHostToDevice, d.lane.stream) != hipSuccess ||
        hipStreamSynchronize(d.lane.stream) != hipSuccess)
        return PA_EDEVICE;
    victim->prec = prec;
    victim->cls = cls;
    victim->used = ++d.clock;
    victim->t = table_view(prec, base, off, fshift);
    *out = victim->t;
    return PA_OK;
}

}  // namespace pa

using namespace pa;

extern "C" pa_status pa_hash_noalloc(pa_ctx* ctx, const uint64_t* seed, uint64_t n, uint64_t m,
                                     const uint64_t* key, uint64_t* out, uint32_t flags) {
    if (!ctx || !seed || !key || !out || n == 0 || m == 0 || n > (1ull << 40) || m > (1ull << 40))
        return PA_EINVAL;
    if (!(flags & PA_DEVICE_PTRS)) return PA_EINVAL;   // host buffers would need staging memory
    const int policy = policy_of(flags);
    if (policy < 0) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->device < 0 || c->device >= kMaxDevices) return PA_EDEVICE;
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    NoAllocDev& d = g_dev[c->device];
    std::lock_guard<std::mutex> dl(d.mu);
    if (!d.ready) return PA_EDEVICE;
    Lane& ln = d.lane;
    ln.stream = c->main.stream;

    CostModel cm;
    {
        std::lock_guard<std::mutex> pk(c->plan_mu);
        cm = c->cost;
    }
    TilePlan plan;
    if (!plan_job(n, m, policy, cm, &plan, kCapLogL)) return PA_EINVAL;
    pa_stats st{};
    fill_plan_stats(&st, plan);
    pa_status s = PA_OK;
    if (choose_direct(flags, n, m, cm, plan)) {
        if (direct_key_words(n) * 4 > kWsBytes) return PA_ESCRATCH;
        st = pa_stats{};
        st.prec = PA_PREC_DIRECT;
        st.chunk_bits = n;
        st.window_bits = m;
        s = ln.direct(c, seed, key, n, m, out, false, &st);
        if (s == PA_OK && !(flags & PA_ASYNC) && hipStreamSynchronize(ln.stream) != hipSuccess) s = PA_EDEVICE;
    } else {
        if (plan.tiles() * sizeof(TileMeta) > kMetaBytes) return PA_ESCRATCH;
        std::vector<JobDesc> jobs(1);
        fill_job(&jobs[0], seed, key, out, n, m, plan);
        const bool async = (flags & PA_ASYNC) && plan.rigorous < kRigorousLimit;
        s = ln.launch(c, plan.prec, plan.cls, jobs, false, !async, &st);
        if (s == PA_OK && !async) s = ln.finish(c, flags & ~PA_TIMING, &st, nullptr);
    }
    set_certified(&st, s);
    c->last = st;
    return s;
}
