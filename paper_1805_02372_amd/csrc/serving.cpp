// Serving: resident seeds, a request queue, and a worker that keeps several
// lanes (streams with their own workspace) busy.  Whenever a lane is free and
// requests are waiting, the worker admits the oldest requests that fit the
// lane's share of the HBM budget into one batched launch (one pipeline launch
// for all their tiles); requests that arrive while batches run join the next
// launch on whichever lane frees first, so their work overlaps on the device
// with the batches already running.  The paper motivates this by real-time
// CV-QKD with keys already resident on the GPU (section 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>

#include "engine.hpp"

namespace pa {

double now_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

static uint64_t words_of(uint64_t bits) { return (bits + 63) >> 6; }

void Ctx::serving_init() {}

static int serve_lanes() {
    const char* e = getenv("PA_SERVE_LANES");
    int v = e ? atoi(e) : 2;
    return std::max(1, std::min(v, 8));
}

void Ctx::serving_shutdown() {
    {
        std::lock_guard<std::mutex> lk(smu);
        stop = true;
    }
    scv.notify_all();
    if (worker_started && worker.joinable()) worker.join();
    worker_started = false;
}

void Ctx::serving_release() {
    for (Lane& ln : lanes) ln.release(this);
    lanes.clear();
    for (DevBuf& b : seeds) b.release(this);
    seeds.clear();
    for (auto& kv : requests) delete kv.second;
    requests.clear();
    pending.clear();
}

// Tile-workspace bytes of a request at its own best FP32 plan (all tiles
// resident at once; a launch runs fewer at a time if the budget is short).
// Workspace bytes of a request's cheapest FP32 plan (all tiles resident) and
// of one of its tiles; the plan's length class goes to *cls.
static uint64_t request_bytes(Ctx* c, uint64_t n, uint64_t m, uint64_t* min_bytes, int* cls) {
    TilePlan p;
    if (!c->plan_cached(n, m, PREC_FP32, &p)) {
        *min_bytes = ~0ull;
        *cls = 0;
        return ~0ull;
    }
    *min_bytes = 8 * p.L;
    *cls = p.cls;
    return p.tiles() * *min_bytes;
}

// Whether AUTO puts request (n, m) on the direct GF(2) path (short outputs).
static bool request_direct(Ctx* c, uint64_t n, uint64_t m) {
    TilePlan p;
    if (!c->plan_cached(n, m, PREC_FP32, &p)) return false;
    CostModel cm;
    {
        std::lock_guard<std::mutex> pl(c->plan_mu);
        cm = c->cost;
    }
    return choose_direct(PA_PREC_AUTO, n, m, cm, p);
}

void Ctx::serve_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(smu);
    std::vector<pa_stats> lane_stats(lanes.size());
    std::vector<uint8_t> busy(lanes.size(), 0);
    const uint64_t lane_budget = budget / (lanes.size() + 1);
    while (true) {
        bool any_busy = false;
        // completions
        for (size_t i = 0; i < lanes.size(); ++i) {
            if (!busy[i]) continue;
            if (hipEventQuery(lanes[i].done) == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            (void)hipGetLastError();
            std::vector<Request*> reqs = lane_reqs[i];
            std::vector<pa_status> per(reqs.size(), PA_OK);
            lk.unlock();
            pa_status s = lanes[i].finish(this, 0, &lane_stats[i], &per);
            const double t = now_seconds();
            lk.lock();
            {
                const pa_stats& x = lane_stats[i];
                serve_total.tiles += x.tiles;
                serve_total.direct_jobs += x.direct_jobs;
                serve_total.fallback_tiles += x.fallback_tiles;
                serve_total.launches += x.launches;
                serve_total.model_bytes += x.model_bytes;
                serve_total.max_residual = std::max(serve_total.max_residual, x.max_residual);
                serve_total.max_abs = std::max(serve_total.max_abs, x.max_abs);
                serve_total.rigorous_bound = std::max(serve_total.rigorous_bound, x.rigorous_bound);
            }
            for (size_t k = 0; k < reqs.size(); ++k) {
                reqs[k]->status = (s == PA_OK || s == PA_EPRECISION) ? per[k] : s;
                reqs[k]->t_done = t;
                reqs[k]->state = 2;
            }
            lane_reqs[i].clear();
            busy[i] = 0;
            done_cv.notify_all();
        }
        // admissions
        for (size_t i = 0; i < lanes.size() && !pending.empty() && !stop; ++i) {
            if (busy[i]) continue;
            // continuous batching: the oldest request and the waiting requests
            // of its kind (within a scan window), up to the lane's budget.  A
            // kind is a length class, or the direct path (cls = 0) for the
            // short outputs that AUTO gives it
            std::vector<Request*> batch;
            uint64_t bytes = 0;
            int cls0 = 0;
            std::deque<Request*> rest;
            size_t scanned = 0;
            while (!pending.empty()) {
                Request* r = pending.front();
                pending.pop_front();
                if (batch.size() >= 4096 || scanned >= 1024) {
                    rest.push_back(r);
                    continue;
                }
                ++scanned;
                uint64_t bmin = 0;
                int cls = 0;
                uint64_t b;
                if (request_direct(this, r->n, r->m)) {
                    b = bmin = ((r->n + 127) / 128) * 16;   // the reversed key
                } else {
                    b = request_bytes(this, r->n, r->m, &bmin, &cls);
                }
                if (bmin > budget) {
                    r->status = PA_ENOMEM;
                    r->t_done = now_seconds();
                    r->state = 2;
                    done_cv.notify_all();
                    continue;
                }
                if (batch.empty()) cls0 = cls;
                if (cls != cls0 || (!batch.empty() && bytes + b > lane_budget)) {
                    rest.push_back(r);
                    continue;
                }
                r->state = 1;
                bytes += b;
                batch.push_back(r);
            }
            pending.swap(rest);
            if (batch.empty()) continue;
            std::vector<uint64_t> ns, ms;
            for (Request* r : batch) {
                ns.push_back(r->n);
                ms.push_back(r->m);
            }
            lk.unlock();
            if (cls0 == 0) {
                // direct products, one after another on the lane's stream
                Lane& ln = lanes[i];
                lane_stats[i] = pa_stats{};
                pa_status s = PA_OK;
                for (size_t k = 0; k < batch.size() && s == PA_OK; ++k)
                    s = ln.direct(this, batch[k]->seed, batch[k]->key, ns[k], ms[k], batch[k]->out, false,
                                  &lane_stats[i]);
                ln.jobs.clear();
                ln.total_tiles = 0;
                if (s == PA_OK && !ln.done && hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess)
                    s = PA_EDEVICE;
                if (s == PA_OK && hipEventRecord(ln.done, ln.stream) != hipSuccess) s = PA_EDEVICE;
                lk.lock();
                if (s != PA_OK) {
                    const double t = now_seconds();
                    for (Request* r : batch) {
                        r->status = s;
                        r->t_done = t;
                        r->state = 2;
                    }
                    done_cv.notify_all();
                } else {
                    lane_reqs[i] = batch;
                    busy[i] = 1;
                    any_busy = true;
                }
                continue;
            }
            const int cls = cls0;
            CostModel cm;
            {
                std::lock_guard<std::mutex> pl(plan_mu);
                cm = cost;
            }
            std::vector<TilePlan> plans(batch.size());
            pa_status s = PA_OK;
            for (size_t k = 0; k < batch.size() && s == PA_OK; ++k)
                if (!plan_at_class(ns[k], ms[k], PREC_FP32, cls, cm, &plans[k])) s = PA_EINVAL;
            std::vector<JobDesc> jobs(batch.size());
            if (s == PA_OK) {
                for (size_t k = 0; k < batch.size(); ++k)
                    fill_job(&jobs[k], batch[k]->seed, batch[k]->key, batch[k]->out,
                             batch[k]->n, batch[k]->m, plans[k]);
                lane_stats[i] = pa_stats{};
                for (const TilePlan& tp : plans) fill_plan_stats(&lane_stats[i], tp);
                s = lanes[i].launch(this, PREC_FP32, cls, jobs, false, true, &lane_stats[i]);
            }
            lk.lock();
            if (s != PA_OK) {
                const double t = now_seconds();
                for (Request* r : batch) {
                    r->status = s;
                    r->t_done = t;
                    r->state = 2;
                }
                done_cv.notify_all();
            } else {
                lane_reqs[i] = batch;
                busy[i] = 1;
                any_busy = true;
            }
        }
        if (stop && !any_busy) break;
        if (any_busy)
            scv.wait_for(lk, std::chrono::microseconds(20));
        else if (pending.empty())
            scv.wait(lk, [&] { return stop || !pending.empty(); });
    }
}

}  // namespace pa

using namespace pa;

extern "C" {

pa_status pa_seed_register(pa_ctx* ctx, const uint64_t* seed, uint64_t nbits, uint32_t flags, uint32_t* seed_id) {
    if (!ctx || !seed || !seed_id || nbits == 0) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    DevBuf b;
    const size_t bytes = words_of(nbits) * 8;
    pa_status st = b.ensure(c, bytes);
    if (st != PA_OK) return st;
    const hipMemcpyKind kind = (flags & PA_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (hipMemcpy(b.ptr, seed, bytes, kind) != hipSuccess) {
        b.release(c);
        return PA_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(c->smu);
    c->seeds.push_back(b);
    c->seed_bits.push_back(nbits);
    *seed_id = (uint32_t)(c->seeds.size() - 1);
    return PA_OK;
}

pa_status pa_submit(pa_ctx* ctx, uint32_t seed_id, uint64_t n, uint64_t m, const uint64_t* key, uint64_t* out,
                    uint64_t* ticket) {
    if (!ctx || !key || !out || !ticket || n == 0 || m == 0) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::unique_lock<std::mutex> lk(c->smu);
    if (seed_id >= c->seeds.size() || n + m - 1 > c->seed_bits[seed_id]) return PA_EINVAL;
    if (c->pending.size() >= c->queue_cap) return PA_EBUSY;
    if (!c->worker_started) {
        lk.unlock();
        if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
        {
            // direct calls keep their workspace between calls; hand it back to
            // the budget so that the serving lanes get their shares (it grows
            // again on the next direct call)
            std::lock_guard<std::mutex> g(c->mu);
            std::vector<Lane*> direct{&c->main};
            for (Lane& ln : c->side) direct.push_back(&ln);
            for (Lane* ln : direct) {
                ln->ws.release(c);
                ln->part.release(c);
            }
        }
        std::vector<Lane> lanes(serve_lanes());
        for (Lane& ln : lanes) {
            if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess) return PA_EDEVICE;
            ln.own_stream = true;
            ln.cap = c->budget / (lanes.size() + 1);  // each lane's share; the rest for seeds and direct calls
        }
        lk.lock();
        if (!c->worker_started) {
            c->lanes = std::move(lanes);
            c->lane_reqs.assign(c->lanes.size(), {});
            c->stop = false;
            c->worker = std::thread([c] { c->serve_loop(); });
            c->worker_started = true;
        } else {
            for (Lane& ln : lanes) ln.release(c);
        }
    }
    Request* r = new Request();
    r->ticket = c->next_ticket++;
    r->seed_id = seed_id;
    r->seed = (const uint64_t*)c->seeds[seed_id].ptr;   // read under smu: registration may run concurrently
    r->n = n;
    r->m = m;
    r->key = key;
    r->out = out;
    r->t_submit = now_seconds();
    c->requests[r->ticket] = r;
    c->pending.push_back(r);
    *ticket = r->ticket;
    lk.unlock();
    c->scv.notify_all();
    return PA_OK;
}

pa_status pa_poll(pa_ctx* ctx, uint64_t ticket, int* done) {
    if (!ctx || !done) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->smu);
    auto it = c->requests.find(ticket);
    if (it == c->requests.end()) return PA_EINVAL;
    *done = it->second->state == 2;
    return PA_OK;
}

pa_status pa_wait(pa_ctx* ctx, uint64_t ticket) {
    if (!ctx) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::unique_lock<std::mutex> lk(c->smu);
    auto it = c->requests.find(ticket);
    if (it == c->requests.end()) return PA_EINVAL;
    Request* r = it->second;
    c->done_cv.wait(lk, [&] { return r->state == 2; });
    return r->status;
}

pa_status pa_serve_stats(pa_ctx* ctx, pa_stats* stats) {
    if (!ctx || !stats) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->smu);
    *stats = c->serve_total;
    stats->live_requests = c->requests.size();
    return PA_OK;
}

pa_status pa_ticket_release(pa_ctx* ctx, uint64_t ticket) {
    if (!ctx) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->smu);
    auto it = c->requests.find(ticket);
    if (it == c->requests.end()) return PA_EINVAL;
    if (it->second->state != 2) return PA_ENOTREADY;
    delete it->second;
    c->requests.erase(it);
    return PA_OK;
}

pa_status pa_ticket_latency(pa_ctx* ctx, uint64_t ticket, double* seconds) {
    if (!ctx || !seconds) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->smu);
    auto it = c->requests.find(ticket);
    if (it == c->requests.end()) return PA_EINVAL;
    if (it->second->state != 2) return PA_ENOTREADY;
    *seconds = it->second->t_done - it->second->t_submit;
    return PA_OK;
}

}  // extern "C"
