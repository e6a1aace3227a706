// Tuner: measured per-tile cost of every FFT length class (paper section 3,
// step 2 sizes blocks and batches from the resources and the precision the
// transform needs; here the planner minimises the summed measured cost of a
// plan's tiles plus one launch cost per launch).  Runs each class on synthetic
// tiles (key and seed bits from a fixed xorshift generator) and times the
// kernel passes with HIP events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "engine.hpp"

namespace pa {

static uint64_t xorshift(uint64_t& s) {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
}

static const char* prec_key(int prec) { return prec == PREC_FP32 ? "fp32" : prec == PREC_FP64 ? "fp64" : "ntt"; }

// {"launch": s, "direct": s, "direct_launch": s, "fp32": {"<L>": [tile_s, first_s], ...}, ...}
static pa_status save_json(const CostModel& cm, const std::vector<int>& precs, const char* path) {
    FILE* f = fopen(path, "w");
    if (!f) return PA_EINVAL;
    fprintf(f, "{\"launch\": %.9g, \"direct\": %.9g, \"direct_launch\": %.9g", cm.launch_s, cm.direct_s,
            cm.direct_launch_s);
    for (size_t i = 0; i < precs.size(); ++i) {
        fprintf(f, ", \"%s\": {", prec_key(precs[i]));
        bool first = true;
        for (int k = kMinClassId; k <= kMaxClassId; ++k) {
            ClassGeom g;
            if (!class_geometry(precs[i], k, &g)) continue;
            fprintf(f, "%s\"%llu\": [%.9g, %.9g]", first ? "" : ", ", (unsigned long long)g.L, cm.tile(precs[i], k),
                    cm.first(precs[i], k));
            first = false;
        }
        fprintf(f, "}");
    }
    fprintf(f, "}\n");
    return fclose(f) == 0 ? PA_OK : PA_EINVAL;
}

// Kernel time (s) of one launch of `count` identical one-tile jobs of class id k.
static pa_status time_launch(Ctx* c, int prec, int k, const TilePlan& p, int count, uint64_t* dseed,
                             uint64_t* dkey, uint64_t* douts, uint64_t out_words, int reps, double* best) {
    const uint64_t L = class_len(k);
    *best = 1e30;
    for (int r = 0; r <= reps; ++r) {  // the first run warms tables and workspace
        std::vector<JobDesc> jobs(count);
        for (int q = 0; q < count; ++q)
            fill_job(&jobs[q], dseed, dkey, douts + q * out_words, L / 2, L / 2 + 1, p);
        pa_stats ps{};
        pa_status st = c->main.launch(c, prec, k, jobs, true, true, &ps);
        if (st == PA_OK) st = c->main.finish(c, PA_TIMING | PA_NO_FALLBACK, &ps, nullptr);
        if (st != PA_OK && st != PA_EPRECISION) return st;
        const double ms = ps.ms_pass[0] + ps.ms_pass[1] + ps.ms_pass[2] + ps.ms_pass[3];
        if (r > 0 && ms > 0) *best = std::min(*best, ms * 1e-3);
    }
    return PA_OK;
}

// Per class: kernel time of one launch with 1 tile (T1) and with 4 tiles (T4);
// the marginal tile cost (T4 - T1) / 3 goes to the class's tile_s, the rest of
// T1 (ramp-up and tail of the launch, and what one tile leaves of the device
// idle) to its first_s; the median of the latter is the launch cost of the
// direct path.
pa_status tune_context(Ctx* c, uint32_t flags, int reps, const char* path) {
    std::vector<int> precs;
    switch (flags & PA_PREC_MASK) {
        case PA_PREC_AUTO: precs = {PREC_FP32, PREC_FP64}; break;
        case PA_PREC_FP32_SEG: precs = {PREC_FP32}; break;
        case PA_PREC_FP64: precs = {PREC_FP64}; break;
        case PA_PREC_NTT: precs = {PREC_NTT}; break;
        case PA_PREC_DIRECT: break;   // the direct path only
        default: return PA_EINVAL;
    }
    if (reps < 1) reps = 1;
    constexpr int kMany = 4;
    const uint64_t maxL = 1ull << 24;
    // synthetic job: n = L/2, m = L/2 + 1 fills one tile of class L exactly
    const uint64_t words = (maxL + 64) / 64 + 2, out_words = maxL / 2 / 64 + 2;
    std::vector<uint64_t> host(2 * words);
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (uint64_t& w : host) w = xorshift(s);
    DevBuf buf;
    pa_status st = buf.ensure(c, (2 * words + kMany * out_words) * 8);
    if (st != PA_OK) return st;
    uint64_t* dseed = (uint64_t*)buf.ptr;
    uint64_t* dkey = dseed + words;
    uint64_t* douts = dkey + words;
    if (hipMemcpy(dseed, host.data(), 2 * words * 8, hipMemcpyHostToDevice) != hipSuccess) {
        buf.release(c);
        return PA_EDEVICE;
    }
    CostModel cm;
    {
        std::lock_guard<std::mutex> lk(c->plan_mu);
        cm = c->cost;
    }
    std::vector<double> fixed;
    for (int prec : precs) {
        int ids[kMaxClassId + 1];
        const int nid = class_ids(prec, ids);
        for (int q = 0; q < nid; ++q) {
            const int k = ids[q];
            const uint64_t L = class_len(k);
            TilePlan p;
            if (!plan_at_class(L / 2, L / 2 + 1, prec, k, cm, &p) || p.tiles() != 1) continue;
            double t1 = 0, t4 = 0;
            st = time_launch(c, prec, k, p, 1, dseed, dkey, douts, out_words, reps, &t1);
            if (st == PA_OK) st = time_launch(c, prec, k, p, kMany, dseed, dkey, douts, out_words, reps, &t4);
            if (st != PA_OK) {
                buf.release(c);
                return st;
            }
            if (t1 >= 1e30 || t4 >= 1e30) continue;
            const double marginal = std::max((t4 - t1) / (kMany - 1), 0.1 * t1);
            cm.set(prec, k, marginal);
            cm.set_first(prec, k, std::max(t1 - marginal, 0.0));
            fixed.push_back(std::max(t1 - marginal, 0.0));
        }
    }
    // direct path: the slope between two output lengths at n = 2^22 is the
    // cost per output and 32-bit key word
    const uint32_t pbits = flags & PA_PREC_MASK;
    if (pbits == PA_PREC_AUTO || pbits == PA_PREC_DIRECT) {
        const uint64_t n = 1ull << 22, ms[2] = {1024, 4096};
        double t[2] = {1e30, 1e30};
        for (int q = 0; q < 2 && st == PA_OK; ++q)
            for (int r = 0; r <= reps && st == PA_OK; ++r) {
                pa_stats ps{};
                c->main.timer.reset();
                st = c->main.direct(c, dseed, dkey, n, ms[q], douts, true, &ps);
                if (st == PA_OK && hipStreamSynchronize(c->main.stream) != hipSuccess) st = PA_EDEVICE;
                c->main.timer.collect(ps.ms_pass);
                const double ms = ps.ms_pass[0] + ps.ms_pass[1];   // prep and product kernels
                if (r > 0 && ms > 0) t[q] = std::min(t[q], ms * 1e-3);
            }
        if (st != PA_OK) {
            buf.release(c);
            return st;
        }
        const double words = (double)((n / 32 + 3) / 4 * 4);
        const double slope = (t[1] - t[0]) / ((double)(ms[1] - ms[0]) * words);
        if (t[1] < 1e30 && slope > 0) {
            cm.direct_s = slope;
            cm.direct_launch_s = std::max(t[0] - slope * (double)ms[0] * words, 0.0);   // the intercept
        }
    }
    buf.release(c);
    if (!fixed.empty()) {
        std::sort(fixed.begin(), fixed.end());
        cm.launch_s = fixed[fixed.size() / 2];
    }
    {
        std::lock_guard<std::mutex> lk(c->plan_mu);
        c->cost = cm;
        c->cost_changed();
    }
    if (path) return save_json(cm, precs, path);
    return PA_OK;
}

pa_status tune_load(Ctx* c, const char* path) {
    std::lock_guard<std::mutex> lk(c->plan_mu);
    CostModel cm = c->cost;
    if (load_tune_table(cm, path) <= 0) return PA_EINVAL;
    c->cost = cm;
    c->cost_changed();
    return PA_OK;
}

}  // namespace pa

using namespace pa;

extern "C" {

pa_status pa_tune(pa_ctx* ctx, uint32_t flags, int reps, const char* path) {
    if (!ctx) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return PA_EDEVICE;
    return tune_context(c, flags, reps, path);
}

pa_status pa_tune_load(pa_ctx* ctx, const char* path) {
    if (!ctx || !path) return PA_EINVAL;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->mu);
    return tune_load(c, path);
}

}  // extern "C"
