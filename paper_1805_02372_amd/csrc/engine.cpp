// libpa host engine: contexts, workspace, twiddle tables, plan execution with
// per-tile certificates and FP64 fallback, and the C ABI of include/pa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "pa.h"
#include "pa_internal.hpp"
#include "planner.hpp"
#include "tables.hpp"
#include "engine.hpp"
#include "direct.hpp"

using namespace pa;

namespace pa {

const char* status_name(pa_status s) {
    switch (s) {
        case PA_OK: return "PA_OK";
        case PA_EINVAL: return "PA_EINVAL: invalid argument";
        case PA_ENOMEM: return "PA_ENOMEM: does not fit the HBM budget";
        case PA_EDEVICE: return "PA_EDEVICE: HIP runtime error";
        case PA_EPRECISION: return "PA_EPRECISION: floating-point certificate failed";
        case PA_EBUSY: return "PA_EBUSY: queue full";
        case PA_ENOTREADY: return "PA_ENOTREADY: not finished";
        case PA_ESCRATCH: return "PA_ESCRATCH: beyond the fixed scratch array of pa_hash_noalloc";
    }
    return "unknown pa_status";
}

static uint64_t words_of(uint64_t bits) { return (bits + 63) >> 6; }

// ------------------------------------------------------------ device memory

pa_status DevBuf::ensure(Ctx* c, size_t need, hipStream_t stream) {
    if (need <= bytes) return PA_OK;
    if (fixed) return PA_ESCRATCH;
    release(c);
    size_t want = std::max(need, (size_t)256);
    uint64_t cur = c->used.load();
    do {  // reserve against the budget
        if (cur + want > c->budget) return PA_ENOMEM;
    } while (!c->used.compare_exchange_weak(cur, cur + want));
    owner = c->pools ? stream : nullptr;
    const hipError_t e = owner ? hipMallocAsync(&ptr, want, owner) : hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        owner = nullptr;
        c->used -= want;
        (void)hipGetLastError();
        return PA_ENOMEM;
    }
    bytes = want;
    return PA_OK;
}

void DevBuf::release(Ctx* c) {
    if (fixed) return;
    if (ptr) {
        if (owner) {
            (void)hipFreeAsync(ptr, owner);   // after the owner's queued work
        } else {
            (void)hipDeviceSynchronize();     // no launch may still use it
            (void)hipFree(ptr);
        }
        c->used -= bytes;
    }
    ptr = nullptr;
    bytes = 0;
    owner = nullptr;
}

pa_status HostBuf::ensure(size_t need) {
    if (need <= bytes) return PA_OK;
    if (fixed) return PA_ESCRATCH;
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
    if (hipHostMalloc(&ptr, std::max(need, (size_t)256), hipHostMallocDefault) != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return PA_ENOMEM;
    }
    bytes = std::max(need, (size_t)256);
    return PA_OK;
}

void HostBuf::release() {
    if (fixed) return;
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// ------------------------------------------------------------ host staging

bool CopyPool::take_part(int* p) {
    if (taken >= nparts) return false;
    *p = taken++;
    return true;
}

void CopyPool::work() {
    std::unique_lock<std::mutex> lk(mu);
    uint64_t seen = gen;
    for (;;) {
        cv.wait(lk, [&] { return stop || gen != seen; });
        if (stop) return;
        seen = gen;
        int p;
        while (take_part(&p)) {
            const size_t lo = (size_t)p * part, len = std::min(part, bytes - lo);
            unsigned char* d = dst;
            const unsigned char* sp = src;
            lk.unlock();
            memcpy(d + lo, sp + lo, len);
            lk.lock();
            if (++finished == nparts) done_cv.notify_all();
        }
    }
}

void CopyPool::copy(void* d, const void* sv, size_t n) {
    constexpr size_t kMin = 1u << 20;
    if (n < kMin) {
        memcpy(d, sv, n);
        return;
    }
    std::lock_guard<std::mutex> jl(job_mu);
    std::unique_lock<std::mutex> lk(mu);
    if (workers.empty() && !stop) {
        const unsigned hc = std::thread::hardware_concurrency();
        const int nw = (int)std::max(1u, std::min(3u, hc > 1 ? hc / 2 : 1u));
        for (int i = 0; i < nw; ++i) workers.emplace_back([this] { work(); });
    }
    const int parts = (int)workers.size() + 1;
    dst = (unsigned char*)d;
    src = (const unsigned char*)sv;
    bytes = n;
    part = ((n + parts - 1) / parts + 4095) & ~(size_t)4095;
    nparts = (int)((n + part - 1) / part);
    taken = 0;
    finished = 0;
    ++gen;
    cv.notify_all();
    int p;
    while (take_part(&p)) {   // the caller copies parts too
        const size_t lo = (size_t)p * part, len = std::min(part, n - lo);
        lk.unlock();
        memcpy(dst + lo, src + lo, len);
        lk.lock();
        ++finished;
    }
    done_cv.wait(lk, [&] { return finished == nparts; });
}

void CopyPool::shutdown() {
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv.notify_all();
    for (std::thread& t : workers)
        if (t.joinable()) t.join();
    workers.clear();
}

// Host inputs to device memory through the lane's pinned staging buffer:
// (dst, src, bytes) triples copied into consecutive 256-byte aligned slots of
// the pinned buffer by the copy pool, then one DMA each on the lane's stream.
// The staging buffer is reused only after the call that filled it has
// synchronised its stream.
static pa_status stage_to_device(Ctx* c, Lane& ln, void* const* dst, const void* const* src, const size_t* bytes,
                                 int count) {
    size_t total = 0;
    for (int k = 0; k < count; ++k) total += (bytes[k] + 255) & ~(size_t)255;
    pa_status st = ln.io_host.ensure(total);
    if (st != PA_OK) return st;
    size_t off = 0;
    for (int k = 0; k < count; ++k) {
        unsigned char* h = (unsigned char*)ln.io_host.ptr + off;
        c->copier.copy(h, src[k], bytes[k]);
        if (hipMemcpyAsync(dst[k], h, bytes[k], hipMemcpyHostToDevice, ln.stream) != hipSuccess) return PA_EDEVICE;
        off += (bytes[k] + 255) & ~(size_t)255;
    }
    return PA_OK;
}

// Device outputs back to host memory through the pinned staging buffer
// (synchronises the lane's stream).
static pa_status stage_to_host(Ctx* c, Lane& ln, void* const* dst, const void* const* src, const size_t* bytes,
                               int count) {
    size_t total = 0;
    for (int k = 0; k < count; ++k) total += (bytes[k] + 255) & ~(size_t)255;
    pa_status st = ln.io_host.ensure(total);
    if (st != PA_OK) return st;
    size_t off = 0;
    for (int k = 0; k < count; ++k) {
        if (hipMemcpyAsync((unsigned char*)ln.io_host.ptr + off, src[k], bytes[k], hipMemcpyDeviceToHost,
                           ln.stream) != hipSuccess)
            return PA_EDEVICE;
        off += (bytes[k] + 255) & ~(size_t)255;
    }
    if (hipStreamSynchronize(ln.stream) != hipSuccess) return PA_EDEVICE;
    off = 0;
    for (int k = 0; k < count; ++k) {
        c->copier.copy(dst[k], (unsigned char*)ln.io_host.ptr + off, bytes[k]);
        off += (bytes[k] + 255) & ~(size_t)255;
    }
    return PA_OK;
}

pa_status stage_in(Ctx* c, Lane& ln, void* const* dst, const void* const* src, const size_t* bytes, int count) {
    return stage_to_device(c, ln, dst, src, bytes, count);
}

// ------------------------------------------------------------ twiddle tables

bool Ctx::plan_cached(uint64_t n, uint64_t m, int policy, TilePlan* out) {
    const auto key = std::make_tuple(n, m, policy, class_filter_key());
    {
        std::lock_guard<std::mutex> lk(plan_mu);
        auto it = plans.find(key);
        if (it != plans.end()) {
            *out = it->second;
            return true;
        }
    }
    CostModel cm;
    {
        std::lock_guard<std::mutex> lk(plan_mu);
        cm = cost;
    }
    if (!plan_job(n, m, policy, cm, out)) return false;
    std::lock_guard<std::mutex> lk(plan_mu);
    if (plans.size() >= 256) plans.clear();
    plans[key] = *out;
    return true;
}

pa_status table_image(int prec, int cls, std::vector<unsigned char>* host, size_t off[kTableSections],
                      int* fshift) {
    ClassGeom g;
    if (!class_geometry(prec, cls, &g)) return PA_EINVAL;
    auto pack = [&](auto& th) {
        using E = typename std::remove_reference<decltype(th.tw)>::type::value_type;
        const void* src[kTableSections] = {th.tw.data(),  th.tw2.data(),  th.fa.data(), th.fb.data(),
                                           th.stw.data(), th.fa64.data(), th.fb64.data()};
        const size_t bytes[kTableSections] = {th.tw.size() * sizeof(E),   th.tw2.size() * sizeof(E),
                                              th.fa.size() * sizeof(E),   th.fb.size() * sizeof(E),
                                              th.stw.size() * sizeof(E),  th.fa64.size() * sizeof(double),
                                              th.fb64.size() * sizeof(double)};
        size_t total = 0;
        for (int k = 0; k < kTableSections; ++k) {
            off[k] = bytes[k] ? total : ~(size_t)0;   // ~0: section absent
            total += (bytes[k] + 255) & ~(size_t)255;
        }
        host->assign(total, 0);
        for (int k = 0; k < kTableSections; ++k)
            if (bytes[k]) memcpy(host->data() + off[k], src[k], bytes[k]);
        *fshift = th.fshift;
    };
    const bool smooth = cls >= 32;
    if (prec == PREC_NTT) {
        TableHost<uint32_t> th;
        build_ntt_tables(g.L, g.n1, g.n2, &th);
        pack(th);
    } else if (prec == PREC_FP32) {
        TableHost<float> th;
        build_tables<float>(g.L, g.n1, g.n2, smooth, &th);
        pack(th);
    } else {
        TableHost<double> th;
        build_tables<double>(g.L, g.n1, g.n2, smooth, &th);
        pack(th);
    }
    return PA_OK;
}

Tables table_view(int prec, unsigned char* base, const size_t off[kTableSections], int fshift) {
    auto at = [&](int k) -> const void* { return off[k] == ~(size_t)0 ? nullptr : base + off[k]; };
    Tables t;
    t.fshift = fshift;
    t.tw = at(0);
    t.tw2 = at(1) ? at(1) : t.tw;   // power-of-two classes: one table for rows and columns
    t.fa = at(2);
    t.fb = at(3);
    t.stw = at(4);
    // an FP32 class carries its own FP64 two-level tables; an FP64 class uses fa, fb
    const bool own64 = prec == PREC_FP32;
    t.fa64 = (const double*)(own64 ? at(5) : at(2));
    t.fb64 = (const double*)(own64 ? at(6) : at(3));
    return t;
}

pa_status Ctx::tables(int prec, int cls, Tables* out) {
    std::lock_guard<std::mutex> lk(tab_mu);
    const int key = prec * 100 + cls;
    auto it = tabs.find(key);
    if (it == tabs.end()) {
        std::vector<unsigned char> host;
        size_t off[kTableSections];
        int fshift = 0;
        pa_status st = table_image(prec, cls, &host, off, &fshift);
        if (st != PA_OK) return st;
        DevTables dt;
        st = dt.buf.ensure(this, host.size());
        if (st != PA_OK) return st;
        if (hipMemcpy(dt.buf.ptr, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
            return PA_EDEVICE;
        dt.t = table_view(prec, (unsigned char*)dt.buf.ptr, off, fshift);
        it = tabs.emplace(key, dt).first;
    }
    *out = it->second.t;
    return PA_OK;
}

pa_status lane_tables(Ctx* c, const Lane& ln, int prec, int cls, Tables* out) {
    return ln.static_tables ? noalloc_tables(c->device, prec, cls, out) : c->tables(prec, cls, out);
}

// ------------------------------------------------------------ pass timing

hipEvent_t PassTimer::mark(hipStream_t s) {
    if (used == pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        pool.push_back(e);
    }
    hipEvent_t e = pool[used++];
    (void)hipEventRecord(e, s);
    return e;
}

void PassTimer::collect(double ms[4]) {
    for (auto& sp : spans) {
        float v = 0;
        if (sp.second.first && sp.second.second &&
            hipEventElapsedTime(&v, sp.second.first, sp.second.second) == hipSuccess)
            ms[sp.first] += v;
    }
    reset();
}

void PassTimer::destroy() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
    reset();
}

// ------------------------------------------------------------ plan execution

void fill_job(JobDesc* jd, const uint64_t* seed, const uint64_t* key, uint64_t* out, uint64_t n, uint64_t m,
              const TilePlan& p) {
    memset(jd, 0, sizeof(*jd));
    jd->key = key;
    jd->seed = seed;
    jd->out = out;
    jd->n = n;
    jd->m = m;
    jd->Bi = p.Bi;
    jd->Bo = p.Bo;
    jd->nchunks = (uint32_t)p.nchunks;
    jd->nouts = (uint32_t)p.nouts;
    jd->out_words = (uint32_t)words_of(m);
}

void Lane::release(Ctx* c) {
    ws.release(c);
    part.release(c);
    meta.release(c);
    jobs_dev.release(c);
    io.release(c);
    aux.release(c);
    if (stream) (void)hipStreamSynchronize(stream);   // the frees above are in its order
    meta_host.release();
    jobs_host.release();
    io_host.release();
    timer.destroy();
    if (done) (void)hipEventDestroy(done);
    done = nullptr;
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    stream = nullptr;
}

// Tiles [first, end) through the three passes, G tiles per launch.
static pa_status run_passes(const ClassKernels* K, JobTable jt, uint32_t first, uint32_t end, size_t G, Lane* ln,
                            const Tables& tb, bool timing, uint64_t* launches) {
    for (uint32_t t0 = first; t0 < end; t0 += (uint32_t)G) {
        jt.tile0 = t0;
        jt.ntiles = (uint32_t)std::min<size_t>(G, end - t0);
        const launch_fn fns[3] = {K->pass1, K->pass2, K->pass3};
        for (int p = 0; p < 3; ++p) {
            hipEvent_t a = timing ? ln->timer.mark(ln->stream) : nullptr;
            // 0: launched; 1: nothing to launch (one-kernel tiles); < 0: error
            const int r = fns[p](jt, ln->ws.ptr, (uint32_t*)ln->part.ptr, (TileMeta*)ln->meta.ptr, tb, ln->stream);
            if (r < 0) return PA_EDEVICE;
            if (r == 0) *launches += 1;
            if (timing) ln->timer.spans.push_back({p, {a, ln->timer.mark(ln->stream)}});
        }
    }
    return PA_OK;
}

pa_status Lane::launch(Ctx* c, int prec_, int cls_, std::vector<JobDesc>& js, bool timing, bool fetch_meta,
                       pa_stats* stats) {
    const ClassKernels* K = class_kernels(prec_, cls_);
    if (!K || js.empty()) return PA_EINVAL;
    prec = prec_;
    cls = cls_;
    const ClassCfg& cfg = K->cfg;
    // Tiles in job order; within a job chunk 0 comes first, so a window is
    // cleared (pass 1 of its chunk-0 tile) before any chunk XORs into it, also
    // when the tiles are split over several launches.
    uint32_t total = 0;
    for (JobDesc& jd : js) {
        jd.tile_begin = total;
        total += jd.nchunks * jd.nouts;
    }
    Tables tb;
    pa_status st = lane_tables(c, *this, prec, cls, &tb);
    if (st != PA_OK) return st;
    st = meta.ensure(c, (size_t)total * sizeof(TileMeta), stream);
    if (st != PA_OK) return st;

    if (js.size() > 1) {  // descriptors first: they are small but must fit
        st = jobs_dev.ensure(c, js.size() * sizeof(JobDesc), stream);
        if (st != PA_OK) return st;
        st = jobs_host.ensure(js.size() * sizeof(JobDesc));
        if (st != PA_OK) return st;
    }
    // tiles per launch: as many as the budget (and the lane cap) allows; on a
    // failed allocation halve until one tile
    const size_t elt = cfg.prec == 64 ? 16 : 8;
    const size_t tile_bytes = (size_t)class_len(cfg.cls) * elt + cfg.ws_extra;
    const size_t part_bytes = (size_t)(cfg.n1 / cfg.b1) * sizeof(uint32_t);
    size_t G = total;
    if (ws.fixed) {   // a fixed workspace: as many tiles as it holds
        G = std::min<size_t>(G, std::min<size_t>(ws.bytes / tile_bytes, part.bytes / part_bytes));
        if (G == 0) return PA_ESCRATCH;
    } else if (ws.bytes < G * tile_bytes || part.bytes < G * part_bytes) {
        const uint64_t u = c->used.load();
        const uint64_t mine = ws.bytes + part.bytes;
        uint64_t avail = c->budget > u ? c->budget - u + mine : mine;
        if (cap) avail = std::min<uint64_t>(avail, cap);
        G = std::max<size_t>(1, std::min<size_t>(G, avail / (tile_bytes + part_bytes)));
    }
    for (;;) {
        st = ws.ensure(c, G * tile_bytes, stream);
        if (st == PA_OK) st = part.ensure(c, G * part_bytes, stream);
        if (st == PA_OK || G == 1) break;
        G = (G + 1) / 2;
    }
    if (st != PA_OK) return st;

    JobTable jt{};
    if (js.size() == 1) {
        jt.one = js[0];
        jt.njobs = 0;
    } else {
        memcpy(jobs_host.ptr, js.data(), js.size() * sizeof(JobDesc));
        if (hipMemcpyAsync(jobs_dev.ptr, jobs_host.ptr, js.size() * sizeof(JobDesc), hipMemcpyHostToDevice,
                           stream) != hipSuccess)
            return PA_EDEVICE;
        jt.many = (const JobDesc*)jobs_dev.ptr;
        jt.njobs = (uint32_t)js.size();
        for (const JobDesc& jd : js) jt.clears |= (jd.nchunks > 1 && !jd.no_clear) ? 1u : 0u;
    }
    if (timing) timer.reset();
    st = run_passes(K, jt, 0, total, G, this, tb, timing, &stats->launches);
    if (st != PA_OK) return st;
    if (fetch_meta) {
        st = meta_host.ensure((size_t)total * sizeof(TileMeta));
        if (st != PA_OK) return st;
        if (hipMemcpyAsync(meta_host.ptr, meta.ptr, (size_t)total * sizeof(TileMeta), hipMemcpyDeviceToHost,
                           stream) != hipSuccess)
            return PA_EDEVICE;
    }
    if (!done && hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) return PA_EDEVICE;
    if (hipEventRecord(done, stream) != hipSuccess) return PA_EDEVICE;
    jobs = js;
    total_tiles = total;
    stats->tiles += total;
    return PA_OK;
}

static bool tile_ok(int prec, const TileMeta& mt, double* res, double* mabs) {
    float r, a;
    memcpy(&r, &mt.maxres, 4);
    memcpy(&a, &mt.maxabs, 4);
    *res = r;
    *mabs = a;
    const double abs_limit = prec == PREC_FP32 ? 1048576.0 : 1099511627776.0;   // 2^20, 2^40
    return std::isfinite(r) && std::isfinite(a) && r <= 0.125f && a < abs_limit && mt.badpar == 0;
}

// Wait for an event: poll for up to about 2 ms (a tile pipeline usually ends
// well within that and polling avoids the wake-up latency of a blocking
// wait), then block.
static hipError_t wait_event(hipEvent_t e) {
    const double t0 = now_seconds();
    for (;;) {
        const hipError_t q = hipEventQuery(e);
        if (q != hipErrorNotReady) return q;
        if (now_seconds() - t0 > 2e-3) return hipEventSynchronize(e);
    }
}

pa_status Lane::finish(Ctx* c, uint32_t flags, pa_stats* stats, std::vector<pa_status>* per_job) {
    if (wait_event(done) != hipSuccess) return PA_EDEVICE;
    if (flags & PA_TIMING) timer.collect(stats->ms_pass);
    const uint32_t total = total_tiles;
    const TileMeta* mt = (const TileMeta*)meta_host.ptr;
    std::vector<uint32_t> failed;
    for (uint32_t t = 0; t < total; ++t) {
        double r, a;
        const bool ok = tile_ok(prec, mt[t], &r, &a);
        stats->max_residual = std::max(stats->max_residual, r);
        stats->max_abs = std::max(stats->max_abs, a);
        if (!ok) failed.push_back(t);
    }
    if (failed.empty()) return PA_OK;
    auto job_of = [&](uint32_t t) {
        size_t lo = 0, hi = jobs.size() - 1;
        while (lo < hi) {
            size_t mid = (lo + hi + 1) / 2;
            if (jobs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
        }
        return lo;
    };
    const ClassKernels* K64 = class_kernels(PREC_FP64, cls);
    if (prec != PREC_FP32 || (flags & PA_NO_FALLBACK) || !K64) {
        if (per_job)
            for (uint32_t t : failed) (*per_job)[job_of(t)] = PA_EPRECISION;
        return PA_EPRECISION;
    }
    // Re-run in FP64 with the same geometry and length class.
    //  * One-chunk job: the failed tile alone (its window is overwritten).
    //  * Job that accumulates chunks (Eq. 7): per failed tile, the FP32 tile
    //    again and then the FP64 tile, both XOR-ing into the window without
    //    clearing it; the FP32 run is deterministic, so its bits cancel the
    //    first run's.  If the repeat's certificate is not bit-identical to the
    //    first run's, the whole job is rebuilt in FP64 instead (its windows
    //    cleared and rebuilt).
    const ClassKernels* K32 = class_kernels(PREC_FP32, cls);
    Tables tb, tb32;
    pa_status st = lane_tables(c, *this, PREC_FP64, cls, &tb);
    if (st == PA_OK) st = lane_tables(c, *this, PREC_FP32, cls, &tb32);
    if (st != PA_OK) return st;
    // the FP64 tile, or the FP32 tile with its bit planes
    st = ws.ensure(c, std::max<size_t>((size_t)class_len(cls) * 16,
                                       (size_t)class_len(cls) * 8 + (K32 ? K32->cfg.ws_extra : 0)),
                   stream);
    if (st != PA_OK) return st;
    const size_t part_words = std::max<size_t>(K64->cfg.n1 / K64->cfg.b1, K32 ? K32->cfg.n1 / K32->cfg.b1 : 0);
    st = part.ensure(c, part_words * sizeof(uint32_t), stream);
    if (st != PA_OK) return st;
    // (job, local tile, mode): 0 one-chunk tile, 1 accumulated tile, 2 whole job
    struct Run { size_t job; uint32_t tile; int mode; };
    std::vector<Run> runs;
    for (uint32_t t : failed) {
        const size_t jx = job_of(t);
        runs.push_back({jx, t - jobs[jx].tile_begin, jobs[jx].nchunks > 1 ? 1 : 0});
    }
    std::vector<uint8_t> rebuilt(jobs.size(), 0);
    auto fetch_meta = [&](uint32_t first, uint32_t end, std::vector<TileMeta>* out) -> pa_status {
        out->resize(end - first);
        if (hipMemcpyAsync(out->data(), (TileMeta*)meta.ptr + first, (end - first) * sizeof(TileMeta),
                           hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return PA_EDEVICE;
        return PA_OK;
    };
    pa_status result = PA_OK;
    for (size_t q = 0; q < runs.size(); ++q) {
        Run r = runs[q];
        const size_t jx = r.job;
        if (rebuilt[jx]) continue;
        const uint32_t ntiles = jobs[jx].nchunks * jobs[jx].nouts;
        JobTable jt{};
        jt.one = jobs[jx];
        jt.one.tile_begin = 0;
        jt.njobs = 0;
        st = meta.ensure(c, (size_t)ntiles * sizeof(TileMeta), stream);
        if (st != PA_OK) return st;
        if (r.mode == 1) {
            jt.one.no_clear = 1;
            bool same = K32 != nullptr;
            if (same) {
                st = run_passes(K32, jt, r.tile, r.tile + 1, 1, this, tb32, false, &stats->launches);
                if (st != PA_OK) return st;
                std::vector<TileMeta> again;
                st = fetch_meta(r.tile, r.tile + 1, &again);
                if (st != PA_OK) return st;
                const TileMeta& o = mt[jobs[jx].tile_begin + r.tile];
                same = memcmp(&again[0], &o, sizeof(TileMeta)) == 0;
                stats->tiles += 1;
            }
            if (!same) {   // rebuild the whole job
                r.mode = 2;
                jt.one.no_clear = 0;
                rebuilt[jx] = 1;
            }
        }
        const uint32_t first = r.mode == 2 ? 0u : r.tile, end = r.mode == 2 ? ntiles : r.tile + 1;
        st = run_passes(K64, jt, first, end, 1, this, tb, false, &stats->launches);
        if (st != PA_OK) return st;
        stats->fallback_tiles += end - first;
        stats->tiles += end - first;
        std::vector<TileMeta> m64;
        st = fetch_meta(first, end, &m64);
        if (st != PA_OK) return st;
        for (const TileMeta& m : m64) {
            double rr, aa;
            if (!tile_ok(PREC_FP64, m, &rr, &aa)) {
                result = PA_EPRECISION;
                if (per_job) (*per_job)[jx] = PA_EPRECISION;
            }
        }
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return PA_EDEVICE;
    return result;
}

pa_status Lane::direct(Ctx* c, const uint64_t* seed, const uint64_t* key, uint64_t n, uint64_t m, uint64_t* out,
                       bool timing, pa_stats* stats) {
    pa_status st = aux.ensure(c, direct_key_words(n) * 4, stream);
    if (st != PA_OK) return st;
    // PA_TIMING: ms_pass[0] the prep kernel, ms_pass[1] the product kernels
    hipEvent_t a = timing ? timer.mark(stream) : nullptr;
    if (launch_direct_prep(key, n, m, out, (uint32_t*)aux.ptr, stream, &stats->launches)) return PA_EDEVICE;
    hipEvent_t b = timing ? timer.mark(stream) : nullptr;
    if (launch_direct_main(seed, n, m, out, (const uint32_t*)aux.ptr, stream, &stats->launches)) return PA_EDEVICE;
    if (timing) {
        timer.spans.push_back({0, {a, b}});
        timer.spans.push_back({1, {b, timer.mark(stream)}});
    }
    stats->direct_jobs += 1;
    stats->model_bytes += (words_of(n + m - 1) + words_of(n) + words_of(m)) * 8;
    return PA_OK;
}

int policy_of(uint32_t flags) {
    switch (flags & PA_PREC_MASK) {
        case PA_PREC_AUTO: return PREC_FP32;
        case PA_PREC_DIRECT: return PREC_FP32;   // the FFT plan describes the job
        case PA_PREC_FP32_SEG: return PREC_FP32;
        case PA_PREC_FP64: return PREC_FP64;
        case PA_PREC_NTT: return PREC_NTT;
    }
    return -1;
}

uint32_t prec_flag(int prec) {
    return prec == PREC_FP32 ? PA_PREC_FP32_SEG : prec == PREC_FP64 ? PA_PREC_FP64 : PA_PREC_NTT;
}

void fill_plan_stats(pa_stats* s, const TilePlan& p) {
    ClassGeom g;
    class_geometry(p.prec, p.cls, &g);
    s->prec = prec_flag(p.prec);
    s->log2_len = (uint32_t)ceil_log2(p.L);
    s->fft_len = (uint32_t)p.L;
    s->n1 = (uint32_t)g.n1;
    s->n2 = (uint32_t)g.n2;
    s->chunk_bits = p.Bi;
    s->window_bits = p.Bo;
    s->bound = std::max(s->bound, p.bound);
    s->rigorous_bound = std::max(s->rigorous_bound, p.rigorous);
    if (p.prec == PREC_FP32 || p.prec == PREC_FP64) s->certified = PA_CERT_A_PRIORI;   // settled by set_certified
    s->model_bytes += p.tiles() * (p.prec == PREC_FP64 ? 48ull : 24ull) * p.L;
}

void set_certified(pa_stats* s, pa_status st) {
    if (st != PA_OK) s->certified = PA_CERT_NONE;
    else if (s->certified == PA_CERT_A_PRIORI && !(s->rigorous_bound < kRigorousLimit))
        s->certified = PA_CERT_A_POSTERIORI;
    else if (s->certified != PA_CERT_A_PRIORI) s->certified = PA_CERT_EXACT;
}

}  // namespace pa

// ================================================================ C ABI

extern "C" {

const char* pa_strerror(pa_status s) { return status_name(s); }

pa_status pa_create(pa_ctx** out, int device, uint64_t budget, void* hip_stream) {
    if (!out) return PA_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return PA_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return PA_EDEVICE;
    Ctx* c = new Ctx();
    c->device = device;
    int pools = 0;
    c->pools = hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, device) == hipSuccess &&
               pools != 0;
    (void)hipGetLastError();
    c->budget = budget ? budget : (8ull << 30);
    c->cost = default_cost_model();
    if (hip_stream) {
        c->main.stream = (hipStream_t)hip_stream;
        c->main.own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&c->main.stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return PA_EDEVICE;
        }
        c->main.own_stream = true;
    }
    c->serving_init();
    // the no-allocation entry's array: its device address, once per device
    // (a failure here only disables pa_hash_noalloc, which then reports it)
    (void)noalloc_setup(device);
    if (const char* tc = getenv("PA_TUNE_CACHE")) (void)tune_load(c, tc);  // optional
    *out = reinterpret_cast<pa_ctx*>(c);
    return PA_OK;
}

void pa_destroy(pa_ctx* ctx) {
    if (!ctx) return;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    (void)hipSetDevice(c->device);
    c->serving_shutdown();
    c->main.release(c);
    for (Lane& ln : c->side) ln.release(c);
    c->serving_release();
    for (StreamRes* r : c->idle_streams) {
        r->release(c);
        delete r;
    }
    c->idle_streams.clear();
    for (auto& kv : c->tabs) kv.second.buf.release(c);
    c->copier.shutdown();
    delete c;
}

static bool job_args_ok(const void* seed, const void* key, const void* out, uint64_t n, uint64_t m) {
    return seed && key && out && n > 0 && m > 0 && n <= (1ull << 40) && m <= (1ull << 40);
}

pa_status pa_hash(pa_ctx* ctx, const uint64_t* seed, uint64_t n, uint64_t m, const uint64_t* key, uint64_t* out,
                  uint32_t flags) {
    if (!ctx || !job_args_ok(seed, key, out, n, m)) return PA_EINVAL;
    const int policy = policy_of(flags);
    if (policy < 0) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    Lane& ln = c->main;
    pa_stats st{};
    TilePlan plan;
    if (!c->plan_cached(n, m, policy, &plan)) return PA_EINVAL;
    fill_plan_stats(&st, plan);

    const uint64_t sw = words_of(n + m - 1), kw = words_of(n), ow = words_of(m);
    const uint64_t *dseed = seed, *dkey = key;
    uint64_t* dout = out;
    const bool dev = flags & PA_DEVICE_PTRS;
    if (!dev) {  // stage host buffers through library memory
        pa_status s = ln.io.ensure(c, (sw + kw + ow) * 8, ln.stream);
        if (s != PA_OK) return s;
        uint64_t* base = (uint64_t*)ln.io.ptr;
        void* dsts[2] = {base, base + sw};
        const void* srcs[2] = {seed, key};
        const size_t lens[2] = {sw * 8, kw * 8};
        s = stage_to_device(c, ln, dsts, srcs, lens, 2);
        if (s != PA_OK) return s;
        dseed = base;
        dkey = base + sw;
        dout = base + sw + kw;
    }
    const bool timing = flags & PA_TIMING;
    pa_status s = PA_OK;
    CostModel cm;
    {
        std::lock_guard<std::mutex> pk(c->plan_mu);
        cm = c->cost;
    }
    if (choose_direct(flags, n, m, cm, plan)) {
        // exact: no certificate, so PA_ASYNC may return once enqueued
        st = pa_stats{};
        st.prec = PA_PREC_DIRECT;
        st.chunk_bits = n;
        st.window_bits = m;
        if (timing) ln.timer.reset();
        s = ln.direct(c, dseed, dkey, n, m, dout, timing, &st);
        const bool async = dev && (flags & PA_ASYNC) && !timing;
        if (s == PA_OK && !async && hipStreamSynchronize(ln.stream) != hipSuccess) s = PA_EDEVICE;
        if (s == PA_OK && timing) ln.timer.collect(st.ms_pass);
    } else {
        std::vector<JobDesc> jobs(1);
        fill_job(&jobs[0], dseed, dkey, dout, n, m, plan);
        // Only an a-priori certified plan (worst-case bound below 0.5, or
        // NTT) may skip the certificate read-back; kernel timing needs the
        // launch to finish.
        const bool async = dev && (flags & PA_ASYNC) && plan.rigorous < kRigorousLimit && !timing;
        s = ln.launch(c, plan.prec, plan.cls, jobs, timing, !async, &st);
        if (s == PA_OK && !async) s = ln.finish(c, flags, &st, nullptr);
    }
    if (s == PA_OK && !dev) {
        void* dsts[1] = {out};
        const void* srcs[1] = {dout};
        const size_t lens[1] = {ow * 8};
        s = stage_to_host(c, ln, dsts, srcs, lens, 1);
    }
    set_certified(&st, s);
    c->last = st;
    return s;
}

}  // extern "C"

namespace pa {
// Side streams for batches: PA_BATCH_LANES (default 2, 1..8) streams in all,
// the context's stream included.  Called with the context mutex held.
pa_status ensure_side_lanes(Ctx* c) {
    const char* e = getenv("PA_BATCH_LANES");
    const int want = std::max(1, std::min(e ? atoi(e) : 2, 8)) - 1;
    if ((int)c->side.size() >= want) return PA_OK;
    while ((int)c->side.size() < want) {
        c->side.emplace_back();
        Lane& ln = c->side.back();
        if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess) {
            c->side.pop_back();
            return PA_EDEVICE;
        }
        ln.own_stream = true;
    }
    return PA_OK;
}
}  // namespace pa

extern "C" {

pa_status pa_hash_batch(pa_ctx* ctx, const pa_job* jobs_in, uint64_t count, uint32_t flags, pa_status* per_job) {
    if (!ctx || (!jobs_in && count)) return PA_EINVAL;
    if (count == 0) return PA_OK;
    if (count > 65535) return PA_EINVAL;
    const int policy = policy_of(flags);
    if (policy < 0) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::vector<uint64_t> ns, ms;
    for (uint64_t i = 0; i < count; ++i) {
        const pa_job& j = jobs_in[i];
        if (!job_args_ok(j.seed, j.key, j.out, j.n, j.m)) {
            if (per_job)
                for (uint64_t k = 0; k < count; ++k) per_job[k] = k == i ? PA_EINVAL : PA_OK;
            return PA_EINVAL;
        }
        ns.push_back(j.n);
        ms.push_back(j.m);
    }
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    Lane& ln = c->main;
    CostModel cm;
    {
        std::lock_guard<std::mutex> pk(c->plan_mu);
        cm = c->cost;
    }
    // jobs on the direct path, and the FFT jobs (planned in length-class
    // groups); a batch of the same shapes as a recent one reuses its plan
    std::vector<uint64_t> shapes(2 * count);
    for (uint64_t i = 0; i < count; ++i) {
        shapes[2 * i] = ns[i];
        shapes[2 * i + 1] = ms[i];
    }
    auto bkey = std::make_tuple(policy, flags & PA_PREC_MASK, class_filter_key(), std::move(shapes));
    std::vector<char> is_direct;
    std::vector<BatchGroup> groups;
    bool cached = false;
    {
        std::lock_guard<std::mutex> pk(c->plan_mu);
        auto it = c->batch_plans.find(bkey);
        if (it != c->batch_plans.end()) {
            is_direct = it->second.is_direct;
            groups = it->second.groups;
            cached = true;
        }
    }
    if (!cached) {
        is_direct.assign(count, 0);
        std::vector<uint64_t> fns, fms;
        std::vector<size_t> fidx;
        std::vector<TilePlan> fplans;
        for (uint64_t i = 0; i < count; ++i) {
            TilePlan p;
            if (!c->plan_cached(ns[i], ms[i], policy, &p)) return PA_EINVAL;
            is_direct[i] = choose_direct(flags, ns[i], ms[i], cm, p);
            if (!is_direct[i]) {
                fidx.push_back(i);
                fns.push_back(ns[i]);
                fms.push_back(ms[i]);
                fplans.push_back(p);
            }
        }
        if (!fidx.empty()) {
            if (!plan_batch_groups(fns, fms, policy, cm, &groups, &fplans)) return PA_EINVAL;
            for (BatchGroup& g : groups)
                for (size_t& q : g.jobs) q = fidx[q];
        }
        std::lock_guard<std::mutex> pk(c->plan_mu);
        if (c->batch_plans.size() >= 16) c->batch_plans.clear();
        c->batch_plans[std::move(bkey)] = Ctx::BatchPlan{is_direct, groups};
    }
    std::vector<const TilePlan*> plan_of(count, nullptr);
    pa_stats st{};
    for (const BatchGroup& g : groups)   // ascending classes: the stats name the largest
        for (size_t q = 0; q < g.jobs.size(); ++q) {
            plan_of[g.jobs[q]] = &g.plans[q];
            fill_plan_stats(&st, g.plans[q]);
        }
    st.chunk_bits = 0;   // differ per job
    st.window_bits = 0;

    const bool dev = flags & PA_DEVICE_PTRS;
    std::vector<JobDesc> all(count);
    std::vector<uint64_t> out_off(count, 0);
    if (!dev) {
        uint64_t total_words = 0;
        for (uint64_t i = 0; i < count; ++i)
            total_words += words_of(ns[i] + ms[i] - 1) + words_of(ns[i]) + words_of(ms[i]);
        pa_status s = ln.io.ensure(c, total_words * 8, ln.stream);
        if (s != PA_OK) return s;
    }
    uint64_t off = 0;
    std::vector<void*> sdst;
    std::vector<const void*> ssrc;
    std::vector<size_t> slen;
    for (uint64_t i = 0; i < count; ++i) {
        const pa_job& j = jobs_in[i];
        const uint64_t *dseed = j.seed, *dkey = j.key;
        uint64_t* dout = j.out;
        if (!dev) {
            uint64_t* base = (uint64_t*)ln.io.ptr + off;
            const uint64_t sw = words_of(j.n + j.m - 1), kw = words_of(j.n), ow = words_of(j.m);
            sdst.insert(sdst.end(), {(void*)base, (void*)(base + sw)});
            ssrc.insert(ssrc.end(), {(const void*)j.seed, (const void*)j.key});
            slen.insert(slen.end(), {(size_t)(sw * 8), (size_t)(kw * 8)});
            dseed = base;
            dkey = base + sw;
            dout = base + sw + kw;
            out_off[i] = off + sw + kw;
            off += sw + kw + ow;
        }
        if (is_direct[i]) {   // pointers only
            all[i].seed = dseed;
            all[i].key = dkey;
            all[i].out = dout;
            all[i].n = j.n;
            all[i].m = j.m;
        } else {
            fill_job(&all[i], dseed, dkey, dout, j.n, j.m, *plan_of[i]);
        }
    }
    if (!dev) {
        const pa_status ss = stage_to_device(c, ln, sdst.data(), ssrc.data(), slen.data(), (int)sdst.size());
        if (ss != PA_OK) return ss;
    }
    // One pipeline launch per length class.  The groups run concurrently on
    // the context's stream and on side streams (forked from it), largest
    // first; a stream takes the next group as soon as its launch is finished.
    std::vector<pa_status> status(count, PA_OK);
    pa_status s = ensure_side_lanes(c);
    if (s != PA_OK) return s;
    std::vector<Lane*> lanes{&ln};
    for (Lane& sl : c->side) lanes.push_back(&sl);
    if (lanes.size() > 1) {
        hipEvent_t fork = nullptr;
        if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return PA_EDEVICE;
        bool ok = hipEventRecord(fork, ln.stream) == hipSuccess;
        for (size_t k = 1; k < lanes.size() && ok; ++k) ok = hipStreamWaitEvent(lanes[k]->stream, fork, 0) == hipSuccess;
        (void)hipEventDestroy(fork);
        if (!ok) return PA_EDEVICE;
    }
    // direct jobs on the context's stream, beside the side streams' groups
    pa_stats dst{};
    const size_t ndirect = (size_t)std::count(is_direct.begin(), is_direct.end(), (char)1);
    for (uint64_t i = 0; i < count && s == PA_OK; ++i) {
        if (!is_direct[i]) continue;
        const pa_status ds = ln.direct(c, all[i].seed, all[i].key, all[i].n, all[i].m, all[i].out, false, &dst);
        if (ds != PA_OK) {
            status[i] = ds;
            s = ds;
        }
    }
    bool stop = s != PA_OK;
    std::vector<size_t> order(groups.size());
    for (size_t g = 0; g < order.size(); ++g) order[g] = g;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return groups[a].cost > groups[b].cost; });
    std::vector<int> on_lane(lanes.size(), -1);          // group running on each lane
    std::vector<pa_stats> lst(lanes.size(), pa_stats{});
    std::deque<size_t> queue(order.begin(), order.end());
    std::deque<size_t> fifo;                              // lanes in launch order
    while (true) {
        for (size_t k = 0; k < lanes.size() && !stop && !queue.empty(); ++k) {
            if (on_lane[k] >= 0) continue;
            const BatchGroup& g = groups[queue.front()];
            std::vector<JobDesc> jobs(g.jobs.size());
            for (size_t q = 0; q < g.jobs.size(); ++q) jobs[q] = all[g.jobs[q]];
            const pa_status ls = lanes[k]->launch(c, g.plans[0].prec, g.cls, jobs, flags & PA_TIMING, true, &lst[k]);
            if (ls != PA_OK) {
                for (size_t q = 0; q < g.jobs.size(); ++q) status[g.jobs[q]] = ls;
                s = ls;
                stop = true;   // device or allocation error: no further groups are started
                break;
            }
            on_lane[k] = (int)queue.front();
            queue.pop_front();
            fifo.push_back(k);
        }
        if (fifo.empty()) break;
        const size_t k = fifo.front();
        fifo.pop_front();
        const BatchGroup& g = groups[(size_t)on_lane[k]];
        on_lane[k] = -1;
        std::vector<pa_status> gst(g.jobs.size(), PA_OK);
        const pa_status gs = lanes[k]->finish(c, flags, &lst[k], &gst);
        const bool per_tile = gs == PA_OK || gs == PA_EPRECISION;
        for (size_t q = 0; q < g.jobs.size(); ++q) status[g.jobs[q]] = per_tile ? gst[q] : gs;
        if (gs != PA_OK && (s == PA_OK || !per_tile)) s = gs;
        if (!per_tile) stop = true;
        if (stop) queue.clear();
    }
    if (ndirect && hipStreamSynchronize(ln.stream) != hipSuccess && s == PA_OK) s = PA_EDEVICE;
    lst.push_back(dst);
    st.direct_jobs = dst.direct_jobs;
    if (ndirect == count) st.prec = PA_PREC_DIRECT;
    for (const pa_stats& x : lst) {
        st.model_bytes += x.model_bytes;
        st.tiles += x.tiles;
        st.fallback_tiles += x.fallback_tiles;
        st.launches += x.launches;
        st.max_residual = std::max(st.max_residual, x.max_residual);
        st.max_abs = std::max(st.max_abs, x.max_abs);
        for (int q = 0; q < 4; ++q) st.ms_pass[q] += x.ms_pass[q];
    }
    if (s != PA_OK && s != PA_EPRECISION) {
        for (uint64_t i = 0; i < count; ++i)
            if (status[i] == PA_OK) status[i] = s;
    }
    if (!dev && (s == PA_OK || s == PA_EPRECISION)) {
        std::vector<void*> odst(count);
        std::vector<const void*> osrc(count);
        std::vector<size_t> olen(count);
        for (uint64_t i = 0; i < count; ++i) {
            odst[i] = jobs_in[i].out;
            osrc[i] = (uint64_t*)ln.io.ptr + out_off[i];
            olen[i] = words_of(ms[i]) * 8;
        }
        const pa_status os = stage_to_host(c, ln, odst.data(), osrc.data(), olen.data(), (int)count);
        if (os != PA_OK) s = os;
    }
    if (per_job)
        for (uint64_t i = 0; i < count; ++i) per_job[i] = (s == PA_OK || s == PA_EPRECISION) ? status[i] : s;
    set_certified(&st, s);
    c->last = st;
    return s;
}

pa_status pa_last_stats(pa_ctx* ctx, pa_stats* out) {
    if (!ctx || !out) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->mu);
    *out = c->last;
    return PA_OK;
}

pa_status pa_plan_query(uint64_t n, uint64_t m, uint32_t flags, pa_plan* out) {
    if (!out || n == 0 || m == 0) return PA_EINVAL;
    const int policy = policy_of(flags);
    if (policy < 0) return PA_EINVAL;
    const CostModel& cm = default_cost_model();
    TilePlan p;
    if (!plan_job(n, m, policy, cm, &p)) return PA_EINVAL;
    ClassGeom g;
    class_geometry(p.prec, p.cls, &g);
    out->prec = prec_flag(p.prec);
    out->log2_len = (uint32_t)ceil_log2(p.L);
    out->fft_len = (uint32_t)p.L;
    out->n1 = (uint32_t)g.n1;
    out->n2 = (uint32_t)g.n2;
    out->chunk_bits = p.Bi;
    out->window_bits = p.Bo;
    out->chunks = p.nchunks;
    out->windows = p.nouts;
    out->bound = p.bound;
    out->cost = p.cost;
    out->direct_cost = direct_cost(n, m, cm);
    out->direct = choose_direct(flags, n, m, cm, p) ? 1u : 0u;
    out->rigorous_bound = p.rigorous;
    return PA_OK;
}

pa_status pa_hash_select(pa_ctx* ctx, const uint64_t* seed, uint64_t n, uint64_t m, const uint64_t* key,
                         const uint64_t* idx, uint64_t count, uint8_t* bits, uint32_t flags) {
    if (!ctx || !seed || !key || n == 0 || m == 0 || n > (1ull << 40) || m > (1ull << 40)) return PA_EINVAL;
    if (count == 0) return PA_OK;
    if (!idx || !bits || count > (1ull << 20)) return PA_EINVAL;
    for (uint64_t k = 0; k < count; ++k)
        if (idx[k] >= m) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    Lane& ln = c->main;
    const uint64_t *dseed = seed, *dkey = key;
    if (!(flags & PA_DEVICE_PTRS)) {
        const uint64_t sw = words_of(n + m - 1), kw = words_of(n);
        pa_status s = ln.io.ensure(c, (sw + kw) * 8, ln.stream);
        if (s != PA_OK) return s;
        uint64_t* base = (uint64_t*)ln.io.ptr;
        void* dsts[2] = {base, base + sw};
        const void* srcs[2] = {seed, key};
        const size_t lens[2] = {sw * 8, kw * 8};
        s = stage_to_device(c, ln, dsts, srcs, lens, 2);
        if (s != PA_OK) return s;
        dseed = base;
        dkey = base + sw;
    }
    // scratch: reversed key | indices | result bits (256-byte aligned sections)
    auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    const uint64_t kr_bytes = up(direct_key_words(n) * 4), idx_bytes = up(count * 8), res_words = words_of(count);
    pa_status s = ln.aux.ensure(c, kr_bytes + idx_bytes + res_words * 8, ln.stream);
    if (s == PA_OK) s = ln.jobs_host.ensure(idx_bytes + res_words * 8);
    if (s != PA_OK) return s;
    uint8_t* dbase = (uint8_t*)ln.aux.ptr;
    uint64_t* didx = (uint64_t*)(dbase + kr_bytes);
    uint64_t* dres = (uint64_t*)(dbase + kr_bytes + idx_bytes);
    uint64_t* hidx = (uint64_t*)ln.jobs_host.ptr;
    uint64_t* hres = (uint64_t*)((uint8_t*)ln.jobs_host.ptr + idx_bytes);
    memcpy(hidx, idx, count * 8);
    if (hipMemcpyAsync(didx, hidx, count * 8, hipMemcpyHostToDevice, ln.stream) != hipSuccess) return PA_EDEVICE;
    if (launch_direct_select(dseed, dkey, n, m, didx, (uint32_t)count, dres, (uint32_t*)dbase, ln.stream))
        return PA_EDEVICE;
    if (hipMemcpyAsync(hres, dres, res_words * 8, hipMemcpyDeviceToHost, ln.stream) != hipSuccess ||
        hipStreamSynchronize(ln.stream) != hipSuccess)
        return PA_EDEVICE;
    for (uint64_t k = 0; k < count; ++k) bits[k] = (uint8_t)((hres[k >> 6] >> (k & 63)) & 1u);
    return PA_OK;
}

double pa_error_model(uint32_t prec, uint32_t log2_len, uint64_t chunk_bits) {
    if ((prec & PA_PREC_MASK) == PA_PREC_DIRECT) return 0.0;   // exact
    const int p = policy_of(prec);
    if (p < 0) return -1.0;
    if (log2_len < 1 || log2_len > 40) return -1.0;
    return error_bound(p, 1ull << log2_len, chunk_bits);
}

}  // extern "C"
