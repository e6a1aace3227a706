// Host engine internals of libpa (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "pa.h"
#include "pa_internal.hpp"
#include "planner.hpp"

namespace pa {

struct Ctx;

// Device allocation charged to the context's HBM budget.  A buffer that one
// stream's work uses (a lane's workspace) is allocated and freed in that
// stream's order (hipMallocAsync / hipFreeAsync), so growing it waits for
// nothing else on the device; other buffers are freed after a device-wide
// synchronisation.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipStream_t owner = nullptr;
    bool fixed = false;   // a view of memory owned elsewhere: never grown or freed
                          // (ensure fails with PA_ESCRATCH beyond `bytes`)
    pa_status ensure(Ctx* c, size_t need, hipStream_t stream = nullptr);
    void release(Ctx* c);
};

// Pinned host allocation (staging of descriptors and certificates).
struct HostBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    bool fixed = false;   // as DevBuf::fixed
    pa_status ensure(size_t need);
    void release();
};

// Copies from pageable host memory into pinned staging buffers (and back),
// split over a few host threads: one thread reads pageable memory at a few
// GB/s, well below what the DMA engines take from pinned memory.  Jobs below
// 1 MiB are copied by the caller alone.  Threads start at the first large
// copy and stop when the context is destroyed.
struct CopyPool {
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::vector<std::thread> workers;
    unsigned char* dst = nullptr;
    const unsigned char* src = nullptr;
    size_t bytes = 0, part = 0;
    int nparts = 0, taken = 0, finished = 0;
    uint64_t gen = 0;
    bool stop = false;
    std::mutex job_mu;   // one copy job at a time
    void copy(void* d, const void* s, size_t n);
    void shutdown();
    ~CopyPool() { shutdown(); }

  private:
    void work();
    bool take_part(int* p);
};

struct DevTables {
    DevBuf buf;
    Tables t;
};

// Events bracketing the passes of one launch (PA_TIMING).
struct PassTimer {
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> spans;  // pass index, (start, stop)
    size_t used = 0;
    hipEvent_t mark(hipStream_t s);
    void reset() { used = 0; spans.clear(); }
    void collect(double ms[4]);
    void destroy();
};

// A stream with its own workspace: runs one plan at a time.
struct Lane {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t cap = 0;     // workspace cap in bytes (0: the context budget)
    DevBuf ws, part, meta, jobs_dev, io;
    DevBuf aux;           // direct path: reversed key, selected indices and bits
    HostBuf meta_host, jobs_host;
    HostBuf io_host;      // pinned staging of host inputs and outputs
    PassTimer timer;
    bool static_tables = false;   // twiddle tables from the no-allocation entry's array

    // In-flight state of an asynchronous launch (serving).
    int prec = 0, cls = 0;
    uint32_t total_tiles = 0;
    std::vector<JobDesc> jobs;
    hipEvent_t done = nullptr;

    void release(Ctx* c);

    // Enqueue every tile of `jobs` (planned at precision prec, class cls); sets
    // tile_begin.  With `fetch_meta` the tile
    // certificates are copied to meta_host behind the kernels.
    pa_status launch(Ctx* c, int prec, int cls, std::vector<JobDesc>& jobs, bool timing, bool fetch_meta,
                     pa_stats* stats);
    // After the launch completed: check certificates, re-run failed FP32
    // tiles (whole jobs when they accumulate chunks) in FP64.  Synchronous on
    // this lane's stream.
    pa_status finish(Ctx* c, uint32_t flags, pa_stats* stats, std::vector<pa_status>* per_job);
    // Enqueue the direct GF(2) product of one job (device pointers); out is
    // written completely.  Asynchronous on this lane's stream.
    pa_status direct(Ctx* c, const uint64_t* seed, const uint64_t* key, uint64_t n, uint64_t m, uint64_t* out,
                     bool timing, pa_stats* stats);
};

// GPU resources of a block stream (pa_stream_*): its lane, a copy stream and
// two staging slots (device buffer, pinned host image, events).  A closed
// stream's resources stay with the context for the next stream.
struct StreamRes {
    Lane ln;
    hipStream_t copy = nullptr;
    DevBuf part, in[2];
    HostBuf pin[2];
    hipEvent_t staged[2] = {}, used[2] = {};
    void release(Ctx* c);
};

// One serving request.
struct Request {
    uint64_t ticket = 0;
    uint32_t seed_id = 0;
    uint64_t n = 0, m = 0;
    const uint64_t* seed = nullptr;   // device copy of the registered seed
    const uint64_t* key = nullptr;
    uint64_t* out = nullptr;
    double t_submit = 0, t_done = 0;
    pa_status status = PA_OK;
    int state = 0;  // 0 queued, 1 running, 2 done
};

struct Ctx {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    std::mutex mu;        // serialises the public calls that use `main`
    std::mutex tab_mu;    // twiddle table cache
    Lane main;
    std::vector<Lane> side;   // extra streams for the length-class groups of a batch
    std::map<int, DevTables> tabs;
    CostModel cost;
    // Plans of recent single-job shapes (key: n, m, policy and the class
    // filter in force); cleared when the cost model changes.
    std::mutex plan_mu;
    std::map<std::tuple<uint64_t, uint64_t, int, uint64_t>, TilePlan> plans;
    bool plan_cached(uint64_t n, uint64_t m, int policy, TilePlan* out);
    // Plans of recent batches: which jobs take the direct path and the
    // length-class groups of the others.  Key: policy, precision flags, class
    // filter, then n and m of every job in order.  Cleared with `plans`.
    struct BatchPlan {
        std::vector<char> is_direct;
        std::vector<BatchGroup> groups;
    };
    std::map<std::tuple<int, uint32_t, uint64_t, std::vector<uint64_t>>, BatchPlan> batch_plans;
    void cost_changed() {   // with plan_mu held
        plans.clear();
        batch_plans.clear();
    }
    std::mutex stream_mu;
    std::vector<StreamRes*> idle_streams;   // resources of closed block streams
    bool pools = false;   // stream-ordered allocation supported on the device
    pa_stats last{};
    CopyPool copier;

    pa_status tables(int prec, int cls, Tables* out);

    // ---- serving
    std::mutex smu;
    std::condition_variable scv, done_cv;
    std::deque<Request*> pending;
    std::map<uint64_t, Request*> requests;
    std::deque<DevBuf> seeds;      // a deque: registering a seed moves no other
    std::vector<uint64_t> seed_bits;
    std::vector<Lane> lanes;
    std::vector<std::vector<Request*>> lane_reqs;
    pa_stats serve_total{};   // summed over the finished serving launches
    std::thread worker;
    bool stop = false, worker_started = false;
    uint64_t next_ticket = 1;
    size_t queue_cap = 1 << 16;
    void serving_init();
    void serving_shutdown();
    void serving_release();
    void serve_loop();
};

const char* status_name(pa_status s);
int policy_of(uint32_t flags);
uint32_t prec_flag(int prec);
void fill_plan_stats(pa_stats* s, const TilePlan& p);
// Settle pa_stats.certified once a call has ended with status st.
void set_certified(pa_stats* s, pa_status st);
void fill_job(JobDesc* jd, const uint64_t* seed, const uint64_t* key, uint64_t* out, uint64_t n, uint64_t m,
              const TilePlan& p);
double now_seconds();
// Host buffers to device memory on a lane's stream through its pinned staging
// buffer (copied in by the context's copy pool, then one DMA each); the lane's
// stream must be synchronised before the staging buffer is used again.
pa_status stage_in(Ctx* c, Lane& ln, void* const* dst, const void* const* src, const size_t* bytes, int count);
pa_status tune_context(Ctx* c, uint32_t flags, int reps, const char* path);
pa_status tune_load(Ctx* c, const char* path);

// Twiddle tables of a length class as one host image: sections tw, tw2, fa,
// fb, stw (element type of the class), fa64, fb64 (FP64), each on a 256-byte
// boundary; `off` receives the section offsets (~0 for an empty section).
constexpr int kTableSections = 7;
pa_status table_image(int prec, int cls, std::vector<unsigned char>* host, size_t off[kTableSections], int* fshift);
// Device pointers of the sections of an image copied to `base`.
Tables table_view(int prec, unsigned char* base, const size_t off[kTableSections], int fshift);
// Tables of a class for a lane: the context's cache, or the no-allocation
// entry's array (Lane::static_tables).
pa_status lane_tables(Ctx* c, const Lane& ln, int prec, int cls, Tables* out);
// No-allocation entry: per-device set-up (called by pa_create with the device
// current) and its tables.
pa_status noalloc_setup(int device);
pa_status noalloc_tables(int device, int prec, int cls, Tables* out);

}  // namespace pa
