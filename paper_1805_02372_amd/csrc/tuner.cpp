// Tuner: measured per-tile cost of every FFT length class (paper section 3,
// step 2 sizes blocks and batches from the resources and the precision the
// transform needs; here the planner minimises the summed measured cost of a
// plan's tiles).  Runs each class on one synthetic tile (key and seed bits from
// a fixed xorshift generator) and times the kernel passes with HIP events.
#include <hip/hip_runtime.h>

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

static pa_status save_json(const CostModel& cm, const std::vector<int>& precs, const char* path) {
    FILE* f = fopen(path, "w");
    if (!f) return PA_EINVAL;
    fprintf(f, "{");
    for (size_t i = 0; i < precs.size(); ++i) {
        fprintf(f, "%s\"%s\": {", i ? ", " : "", prec_key(precs[i]));
        for (int k = 12; k <= 24; ++k) fprintf(f, "%s\"%d\": %.9g", k > 12 ? ", " : "", k, cm.tile(precs[i], k));
        fprintf(f, "}");
    }
    fprintf(f, "}\n");
    return fclose(f) == 0 ? PA_OK : PA_EINVAL;
}

// Minimal reader for the format save_json writes.
static pa_status load_json(CostModel& cm, const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return PA_EINVAL;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    int loaded = 0;
    for (int prec : {PREC_FP32, PREC_FP64, PREC_NTT}) {
        const std::string tag = std::string("\"") + prec_key(prec) + "\"";
        size_t at = text.find(tag);
        if (at == std::string::npos) continue;
        const size_t open = text.find('{', at), close = text.find('}', at);
        if (open == std::string::npos || close == std::string::npos || close < open) return PA_EINVAL;
        const std::string body = text.substr(open + 1, close - open - 1);
        for (int k = 12; k <= 24; ++k) {
            const std::string key = "\"" + std::to_string(k) + "\":";
            size_t p = body.find(key);
            if (p == std::string::npos) continue;
            const double v = strtod(body.c_str() + p + key.size(), nullptr);
            if (v > 0 && v < 10.0) {
                cm.set(prec, k, v);
                ++loaded;
            }
        }
    }
    return loaded ? PA_OK : PA_EINVAL;
}

pa_status tune_context(Ctx* c, uint32_t flags, int reps, const char* path) {
    std::vector<int> precs;
    switch (flags & PA_PREC_MASK) {
        case PA_PREC_AUTO: precs = {PREC_FP32, PREC_FP64}; break;
        case PA_PREC_FP32_SEG: precs = {PREC_FP32}; break;
        case PA_PREC_FP64: precs = {PREC_FP64}; break;
        case PA_PREC_NTT: precs = {PREC_NTT}; break;
        default: return PA_EINVAL;
    }
    if (reps < 1) reps = 1;
    Lane& ln = c->main;
    const uint64_t maxL = 1ull << 24;
    // synthetic job: n = L/2, m = L/2 + 1 fills one tile of class L exactly
    const uint64_t words = (maxL + 64) / 64 + 2;
    std::vector<uint64_t> host(2 * words);
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (uint64_t& w : host) w = xorshift(s);
    DevBuf buf;
    pa_status st = buf.ensure(c, (2 * words + words) * 8);
    if (st != PA_OK) return st;
    uint64_t* dseed = (uint64_t*)buf.ptr;
    uint64_t* dkey = dseed + words;
    uint64_t* dout = dkey + words;
    if (hipMemcpy(dseed, host.data(), 2 * words * 8, hipMemcpyHostToDevice) != hipSuccess) {
        buf.release(c);
        return PA_EDEVICE;
    }
    for (int prec : precs)
        for (int k = 12; k <= 24; ++k) {
            const uint64_t L = 1ull << k;
            TilePlan p;
            if (!plan_at_class(L / 2, L / 2 + 1, prec, k, c->cost, &p) || p.tiles() != 1) continue;
            double best = 1e30;
            for (int r = 0; r <= reps; ++r) {  // first run warms tables and workspace
                std::vector<JobDesc> jobs(1);
                fill_job(&jobs[0], dseed, dkey, dout, L / 2, L / 2 + 1, p);
                pa_stats ps{};
                st = ln.launch(c, prec, k, jobs, true, true, &ps);
                if (st == PA_OK) st = ln.finish(c, PA_TIMING | PA_NO_FALLBACK, &ps, nullptr);
                if (st != PA_OK && st != PA_EPRECISION) {
                    buf.release(c);
                    return st;
                }
                const double ms = ps.ms_pass[0] + ps.ms_pass[1] + ps.ms_pass[2] + ps.ms_pass[3];
                if (r > 0 && ms > 0) best = std::min(best, ms * 1e-3);
            }
            if (best < 1e30) c->cost.set(prec, k, best);
        }
    buf.release(c);
    if (path) return save_json(c->cost, precs, path);
    return PA_OK;
}

pa_status tune_load(Ctx* c, const char* path) { return load_json(c->cost, path); }

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
