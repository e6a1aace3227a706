// Tile planning (paper section 3, step 2: choose the number of blocks and
// batches from the input length, the device memory and the precision the FFT
// needs).  Here a job is cut into key chunks (the paper's blocks/batches, Eq.
// 4-5) and, when the output is long, output windows; every tile of a plan uses
// one FFT length class.
#include "planner.hpp"

#include "pa.h"

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>

namespace pa {

namespace {
double g_kappa = 1.0;

int prec_index(int prec) { return prec == PREC_FP32 ? 0 : prec == PREC_FP64 ? 1 : 2; }

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
uint64_t round_up64(uint64_t a) { return (a + 63) & ~uint64_t(63); }
}  // namespace

// Smallest class; PA_MIN_LOG2_LEN (12..24) raises it (with PA_MAX_LOG2_LEN it
// pins the class, e.g. to exercise one kernel family).
int min_logL(int) {
    int lo = 12;
    if (const char* e = getenv("PA_MIN_LOG2_LEN")) {
        int v = atoi(e);
        if (v > lo && v <= 24) lo = v;
    }
    return lo;
}

// Largest class; PA_MAX_LOG2_LEN (12..24) lowers it, e.g. to force key
// chunking and output windows on small inputs.
int max_logL(int prec) {
    (void)prec;
    int cap = 24;
    if (const char* e = getenv("PA_MAX_LOG2_LEN")) {
        int v = atoi(e);
        if (v >= 12 && v < cap) cap = v;
    }
    return cap;
}

int ceil_log2(uint64_t L) {
    int k = 0;
    while ((1ull << k) < L) ++k;
    return k;
}

bool class_geometry(int prec, int cls, ClassGeom* g) {
    if (!class_id_valid(cls)) return false;
    const uint64_t L = class_len(cls);
    g->prec = prec;
    g->cls = cls;
    g->L = L;
    g->r = 16;
    if (cls >= 32) {   // mixed-radix class L = P 2^k (FP32 and FP64 only)
        if (prec != PREC_FP32 && prec != PREC_FP64) return false;
        // power-of-two rows: those of the class 2^k below 2^20, else 8192;
        // the columns carry the factor P (radix-P stage, 4P points per thread)
        const int P = smooth_P(cls), k = smooth_k(cls);
        // rows of the three-pass geometry of 2^k (its short lengths run as
        // one-kernel tiles, whose row is the whole length)
        const int n2log = std::max(k - 13, std::min(prec == PREC_FP64 ? 11 : 10, k / 2));
        g->n1 = L >= (1ull << 20) ? 8192 : 1 << (k - n2log);
        g->n2 = (int)(L / (uint64_t)g->n1);
        g->b1 = prec == PREC_FP64 ? 4 : 8;
        g->b3 = prec == PREC_FP64 ? 8 : 16;
        g->r = 4 * P;
        return true;
    }
    const int logL = cls;
    if (prec == PREC_NTT) {
        const int n2log = std::min(11, logL / 2);
        g->n2 = 1 << n2log;
        g->n1 = 1 << (logL - n2log);
        g->b1 = 4;
        g->b3 = 8;
        return true;
    }
    if (logL >= 20) {  // wave-level classes: rows of 8192
        const int n2 = 1 << (logL - 13);
        const bool f32 = prec != PREC_FP64;
        const int w = n2 > 1024 ? n2 / 1024 : 1, m = n2 > 1024 ? 1024 : n2;
        const int waves1 = (f32 && w > 1) ? 16 : 8;
        const int g3 = 1024 / (n2 / 2);
        const int waves3 = (f32 && g3 == 1) ? 16 : 8;
        g->n1 = 8192;
        g->n2 = n2;
        g->b1 = waves1 * (1024 / m) / w;
        g->b3 = waves3 * g3;
        return true;
    }
    if (logL <= 13) {   // one-kernel tiles: the whole length in one workgroup
        g->n1 = 1 << logL;
        g->n2 = 1;
        g->b1 = g->n1;
        g->b3 = g->n1;
        return true;
    }
    int n2cap = prec == PREC_FP64 ? 11 : 10;
    int n2log = std::max(logL - 13, std::min(n2cap, logL / 2));
    g->n2 = 1 << n2log;
    g->n1 = 1 << (logL - n2log);
    g->b1 = prec == PREC_FP64 ? 4 : 8;
    g->b3 = prec == PREC_FP64 ? 8 : 16;
    return true;
}

static uint64_t env_u64(const char* name) {
    const char* e = getenv(name);
    return e ? strtoull(e, nullptr, 10) : 0;
}

int class_ids(int prec, int* ids, int cap_logL) {
    const uint64_t lo = 1ull << min_logL(prec), hi = 1ull << std::min(max_logL(prec), cap_logL);
    const uint64_t only = env_u64("PA_ONLY_LEN");
    const bool pow2 = env_u64("PA_POW2_ONLY") != 0;
    int count = 0;
    for (int id = kMinClassId; id <= kMaxClassId; ++id) {
        ClassGeom g;
        if (!class_geometry(prec, id, &g)) continue;
        if (g.L < lo || g.L > hi || (only && g.L != only) || (pow2 && id >= 32)) continue;
        ids[count++] = id;
    }
    std::sort(ids, ids + count, [](int a, int b) { return class_len(a) < class_len(b); });
    return count;
}

uint64_t class_filter_key() {
    return (uint64_t)min_logL(0) | ((uint64_t)max_logL(0) << 8) | ((env_u64("PA_POW2_ONLY") != 0 ? 1ull : 0ull) << 16) |
           (env_u64("PA_ONLY_LEN") << 20);
}

void set_error_kappa(double kappa) { g_kappa = kappa; }
double error_kappa() { return g_kappa; }

static double unit_roundoff(int prec) {
    return prec == PREC_FP32 ? std::ldexp(1.0, -24) : prec == PREC_FP64 ? std::ldexp(1.0, -53) : 0.0;
}

// Low-frequency term.  The key chunk is a 0/1 sequence on [0, Bi) padded with
// zeros, so its mean (1/2 per bit) gives it the spectrum of a box,
// |X_k| ~ D_k / 2 with the Dirichlet kernel D_k = |sin(pi Bi k / L) / sin(pi k / L)|,
// which reaches L / (2 pi k) at the lowest frequencies.  With the two sequences
// packed in one complex transform, an absolute error of about u |X_k| leaks
// into the separated W_k, and the product picks up about u |X_k|^2 there.  The
// inverse transform spreads these few bins over every output as a smooth
// wave of rms u sqrt(sum_k 2 (D_k / 2)^4) / L; the sum converges like k^-4 and
// 16 terms hold it (the rest is below 10^-4 of it).  The maximum over a tile
// is about 2-4 times the rms.
static double box_leak_rms(int prec, uint64_t Lc, uint64_t Bi) {
    const double L = (double)Lc;
    const uint64_t twoL = 2 * Lc;
    // sin(pi Bi k / L) and sin(pi k / L) for k = 1, 2, ... by rotation
    const double a = M_PI * (double)(Bi % twoL) / L, b = M_PI / L;
    const double sa = std::sin(a), ca = std::cos(a), sb = std::sin(b), cb = std::cos(b);
    double sak = sa, cak = ca, sbk = sb, cbk = cb, s4 = 0;
    for (uint64_t k = 1; k <= 16 && (double)k < L / 2; ++k) {
        const double d = std::fabs(sak / sbk) / 2;
        s4 += 2 * d * d * d * d;
        const double s1 = sak * ca + cak * sa, c1 = cak * ca - sak * sa;
        const double s2 = sbk * cb + cbk * sb, c2 = cbk * cb - sbk * sb;
        sak = s1, cak = c1, sbk = s2, cbk = c2;
    }
    return unit_roundoff(prec) * std::sqrt(s4) / L;
}

double error_bound(int prec, uint64_t Lc, uint64_t Bi) {
    if (prec == PREC_NTT) return 0.0;
    // the noise term: the packed transform carries the seed's norm sqrt(L)
    // beside the chunk's sqrt(Bi), so even a one-bit chunk sees u sqrt(L log L)
    const double L = (double)Lc;
    return 6.0 * g_kappa * unit_roundoff(prec) * std::sqrt(std::log2(L) * ((double)Bi + L)) +
           5.0 * box_leak_rms(prec, Lc, Bi);
}

// Worst-case bound of Percival's form (Math. Comp. 72, 2003): an FFT
// convolution of a and b whose 3k radix-2 levels each add a relative error of
// at most (1+u) for the additions, (1+u sqrt5) for a complex product and
// (1+beta) for the twiddle (beta = 2u: table roots rounded once, four-step
// roots an FP64 product rounded once) has max error at most
// ||a|| ||b|| ((1+u)^3k (1+u sqrt5)^(3k+1) (1+beta)^3k - 1).  Read for this
// pipeline: radix-4/8/16 stages count as their radix-2 levels, a radix-3/5/7
// stage as ceil(log2 P) + 1 levels (k = ceil(log2 L) + 1 for a mixed-radix
// length), the spectrum separation and the half-length Hermitian inverse add
// two levels (3k+2), and the two sequences share one transform, so
// ||a|| ||b|| is replaced by (||x|| + ||w||)^2 with ||x|| <= sqrt(Bi) (0/1
// chunk) and ||w|| = sqrt(Bi+Bo-1) (+-1 seed slice).  It holds for every
// input bit pattern.
double rigorous_bound(int prec, uint64_t L, uint64_t Bi, uint64_t Bo) {
    if (prec == PREC_NTT || prec == PREC_DIRECT) return 0.0;
    const int levels = ceil_log2(L) + ((L & (L - 1)) ? 1 : 0);
    const double u = unit_roundoff(prec), lv = 3.0 * levels + 2.0, beta = 2.0 * u;
    const double g = lv * std::log1p(u) + (lv + 1) * std::log1p(u * std::sqrt(5.0)) + lv * std::log1p(beta);
    const double norms = std::sqrt((double)Bi) + std::sqrt((double)(Bi + Bo - 1));
    return norms * norms * std::expm1(g);
}

CostModel::CostModel() {
    launch_s = 12e-6;
    // two VALU operations per output and key word at half the vector rate
    // (256 CUs x 64 lanes x 2.4 GHz)
    direct_s = 1.0e-13;
    direct_launch_s = 12e-6;
    for (int p = 0; p < 3; ++p)
        for (int id = 0; id < 64; ++id) {
            const uint64_t Lc = class_len(id);
            if (Lc == 0) {
                tile_s[p][id] = 1.0;
                continue;
            }
            const double L = (double)Lc, lg = std::log2(L);
            // bytes moved by the three passes and a VALU estimate
            const double bytes = (p == 1 ? 48.0 : 24.0) * L;
            const double instr = L * (5.0 * lg + 40.0) * (p == 2 ? 3.0 : 1.0);
            const double t_mem = bytes / 5.0e12, t_alu = instr / 20.0e12;
            // the long mixed-radix classes run workgroup-wide Stockham column
            // passes, slower per point than the wave-level ones (measured on
            // MI355X: about 1.8x in FP32 and 1.4x in FP64)
            const double generic = (id >= 32 && Lc >= (1ull << 20)) ? (p == 1 ? 1.4 : 1.8) : 1.0;
            tile_s[p][id] = generic * std::max(t_mem, t_alu) + 1e-6;
            first_s[p][id] = launch_s;
        }
}

double CostModel::tile(int prec, int cls) const { return tile_s[prec_index(prec)][cls]; }
double CostModel::first(int prec, int cls) const { return first_s[prec_index(prec)][cls]; }
void CostModel::set(int prec, int cls, double s) { tile_s[prec_index(prec)][cls] = s; }
void CostModel::set_first(int prec, int cls, double s) { first_s[prec_index(prec)][cls] = s; }

static const char* prec_key(int prec) { return prec == PREC_FP32 ? "fp32" : prec == PREC_FP64 ? "fp64" : "ntt"; }

// Minimal reader of the table pa_tune writes:
//   {"launch": s, "direct": s, "direct_launch": s,
//    "fp32": {"<L>": [tile_s, first_s], ...}, "fp64": {...}}
// (a plain number instead of the pair sets tile_s only).
int load_tune_table(CostModel& cm, const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return -1;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    int loaded = 0;
    const size_t la = text.find("\"launch\":");
    if (la != std::string::npos) {
        const double v = strtod(text.c_str() + la + 9, nullptr);
        if (v >= 0 && v < 1.0) cm.launch_s = v;
    }
    const size_t di = text.find("\"direct\":");
    if (di != std::string::npos) {
        const double v = strtod(text.c_str() + di + 9, nullptr);
        if (v > 0 && v < 1e-6) {
            cm.direct_s = v;
            ++loaded;
        }
    }
    const size_t dl = text.find("\"direct_launch\":");
    if (dl != std::string::npos) {
        const double v = strtod(text.c_str() + dl + 16, nullptr);
        if (v >= 0 && v < 1e-2) cm.direct_launch_s = v;
    }
    for (int prec : {PREC_FP32, PREC_FP64, PREC_NTT}) {
        const std::string tag = std::string("\"") + prec_key(prec) + "\"";
        const size_t at = text.find(tag);
        if (at == std::string::npos) continue;
        const size_t open = text.find('{', at), close = text.find('}', at);
        if (open == std::string::npos || close == std::string::npos || close < open) return -1;
        const std::string body = text.substr(open + 1, close - open - 1);
        for (int k = kMinClassId; k <= kMaxClassId; ++k) {
            ClassGeom g;
            if (!class_geometry(prec, k, &g)) continue;
            const std::string key = "\"" + std::to_string(g.L) + "\":";
            const size_t p = body.find(key);
            if (p == std::string::npos) continue;
            const char* q = body.c_str() + p + key.size();
            while (*q == ' ') ++q;
            const bool pair = *q == '[';
            char* end = nullptr;
            const double v = strtod(pair ? q + 1 : q, &end);
            if (!(v > 0 && v < 10.0)) continue;
            cm.set(prec, k, v);
            ++loaded;
            if (pair && end) {
                while (*end == ' ' || *end == ',') ++end;
                const double w = strtod(end, nullptr);
                if (w >= 0 && w < 1.0) cm.set_first(prec, k, w);
            }
        }
    }
    return loaded;
}

const CostModel& default_cost_model() {
    static const CostModel cm = [] {
        CostModel m;
        const char* e = getenv("PA_TUNE_DEFAULT");
        if (e && e[0] == '0') return m;
        Dl_info info;
        if (dladdr((const void*)&load_tune_table, &info) && info.dli_fname) {
            std::string dir(info.dli_fname);
            const size_t slash = dir.rfind('/');
            dir = slash == std::string::npos ? std::string(".") : dir.substr(0, slash);
            (void)load_tune_table(m, (dir + "/tune_mi355x.json").c_str());
        }
        return m;
    }();
    return cm;
}

double direct_cost(uint64_t n, uint64_t m, const CostModel& cm) {
    const double outs = (double)(ceil_div(m, 256) * 256), words = (double)(ceil_div(ceil_div(n, 32), 4) * 4);
    return cm.direct_launch_s + cm.direct_s * outs * words;
}

bool choose_direct(uint32_t flags, uint64_t n, uint64_t m, const CostModel& cm, const TilePlan& fft) {
    const uint32_t p = flags & PA_PREC_MASK;
    if (p == PA_PREC_DIRECT) return true;
    return p == PA_PREC_AUTO && direct_cost(n, m, cm) < fft.cost;
}

bool plan_at_class(uint64_t n, uint64_t m, int prec, int cls, const CostModel& cm, TilePlan* out) {
    ClassGeom g;
    if (n == 0 || m == 0 || !class_geometry(prec, cls, &g)) return false;
    const uint64_t L = g.L;
    // largest chunk the error model admits at this length
    uint64_t bi_cap = n;
    if (prec != PREC_NTT) {
        const double per = 6.0 * g_kappa * unit_roundoff(prec) * std::sqrt(std::log2((double)L));
        const double cap = std::floor((kPlanErrorLimit / per) * (kPlanErrorLimit / per) - (double)L);
        if (cap < (double)bi_cap) bi_cap = (uint64_t)std::max(0.0, cap);
    }
    TilePlan best;
    bool found = false;
    const uint64_t max_outs = std::min<uint64_t>(ceil_div(m, 64), 1u << 14);
    uint64_t last_bo = 0;
    const uint64_t min_chunks = ceil_div(n, std::min<uint64_t>(L, bi_cap == 0 ? 1 : bi_cap));
    // fewer than ceil(m / L) windows cannot fit a window in L
    for (uint64_t w = std::max<uint64_t>(1, ceil_div(m, L)); w <= std::max<uint64_t>(1, max_outs); ++w) {
        // every later candidate has >= w windows and >= min_chunks chunks
        if (found && w * min_chunks >= best.tiles()) break;
        uint64_t Bo = (w == 1) ? m : round_up64(ceil_div(m, w));
        if (Bo == last_bo) continue;
        last_bo = Bo;
        if (Bo > L) continue;
        const uint64_t nouts = ceil_div(m, Bo);
        uint64_t bi_max = std::min<uint64_t>(L - Bo + 1, bi_cap);
        if (bi_max == 0) continue;
        const uint64_t nchunks = ceil_div(n, bi_max);
        const uint64_t Bi = ceil_div(n, nchunks);
        const uint64_t tiles = nchunks * nouts;
        if (!found || tiles < best.tiles()) {
            found = true;
            best.prec = prec;
            best.cls = cls;
            best.L = L;
            best.Bi = Bi;
            best.Bo = Bo;
            best.nchunks = nchunks;
            best.nouts = nouts;
        }
        if (nouts == 1 && nchunks == 1) break;
    }
    if (!found) return false;
    best.bound = error_bound(prec, L, best.Bi);
    best.rigorous = rigorous_bound(prec, L, best.Bi, best.Bo);
    if (best.bound > kPlanErrorLimit) return false;   // not reached by FP32 up to 2^24
    best.cost = (double)best.tiles() * cm.tile(prec, cls) + cm.first(prec, cls);
    *out = best;
    return true;
}

bool plan_job(uint64_t n, uint64_t m, int policy, const CostModel& cm, TilePlan* out, int cap_logL) {
    if (n == 0 || m == 0) return false;
    const int prec = policy;
    int ids[kMaxClassId + 1];
    const int nid = class_ids(prec, ids, cap_logL);
    // Classes come in increasing length.  A plan that moves more points (tiles
    // x L) replaces the best so far only when its modeled cost is lower by
    // more than the noise of the measured costs (10%), so near-ties keep the
    // plan with fewer bytes.
    auto better = [](const TilePlan& p, const TilePlan& best) {
        const double pts = (double)p.tiles() * (double)p.L, bpts = (double)best.tiles() * (double)best.L;
        return pts <= bpts ? p.cost < best.cost : p.cost < 0.9 * best.cost;
    };
    if (prec == PREC_FP64 || prec == PREC_NTT) {
        // one tile: the shortest class that holds the whole product, unless a
        // longer class is clearly cheaper
        bool one = false;
        TilePlan best1;
        for (int q = 0; q < nid; ++q) {
            TilePlan p;
            if (n + m - 1 > class_len(ids[q]) || !plan_at_class(n, m, prec, ids[q], cm, &p)) continue;
            if (!one || better(p, best1)) {
                best1 = p;
                one = true;
            }
        }
        if (one) {
            *out = best1;
            return true;
        }
    }
    bool found = false;
    TilePlan best;
    for (int q = 0; q < nid; ++q) {
        TilePlan p;
        if (!plan_at_class(n, m, prec, ids[q], cm, &p)) continue;
        if (!found || better(p, best)) {
            best = p;
            found = true;
        }
    }
    if (found) *out = best;
    return found;
}

bool plan_batch_groups(const std::vector<uint64_t>& ns, const std::vector<uint64_t>& ms, int policy,
                       const CostModel& cm, std::vector<BatchGroup>* groups, const std::vector<TilePlan>* own) {
    if (ns.empty() || ns.size() != ms.size() || (own && own->size() != ns.size())) return false;
    // plans of job i at class id k, computed once: memo[i * NK + k], state 0
    // unknown, 1 found, -1 none
    constexpr int NK = kMaxClassId + 1;
    std::vector<TilePlan> memo(ns.size() * NK);
    std::vector<signed char> known(ns.size() * NK, 0);
    auto at_class = [&](size_t i, int k, TilePlan* p) {
        if (k < 0 || k >= NK) return false;
        const size_t x = i * NK + (size_t)k;
        if (!known[x]) known[x] = plan_at_class(ns[i], ms[i], policy, k, cm, &memo[x]) ? 1 : -1;
        if (known[x] < 0) return false;
        *p = memo[x];
        return true;
    };
    std::map<int, BatchGroup> by_class;
    for (size_t i = 0; i < ns.size(); ++i) {
        TilePlan p;
        if (own) p = (*own)[i];
        else if (!plan_job(ns[i], ms[i], policy, cm, &p)) return false;
        BatchGroup& g = by_class[p.cls];
        g.cls = p.cls;
        g.jobs.push_back(i);
        g.plans.push_back(p);
        g.cost += p.cost - cm.first(policy, p.cls);
    }
    std::vector<BatchGroup> gs;
    for (auto& kv : by_class) {
        kv.second.cost += cm.first(policy, kv.second.cls);
        gs.push_back(std::move(kv.second));
    }
    // fold groups while that saves more than it costs
    for (;;) {
        double best_gain = 0;
        size_t bg = 0, bh = 0;
        std::vector<TilePlan> best_plans;
        for (size_t g = 0; g < gs.size(); ++g)
            for (size_t h = 0; h < gs.size(); ++h) {
                if (g == h) continue;
                std::vector<TilePlan> moved(gs[g].jobs.size());
                double c = 0;
                bool ok = true;
                for (size_t q = 0; q < gs[g].jobs.size() && ok; ++q) {
                    const size_t i = gs[g].jobs[q];
                    ok = at_class(i, gs[h].cls, &moved[q]);
                    c += moved[q].cost - cm.first(policy, gs[h].cls);
                }
                if (!ok) continue;
                const double gain = gs[g].cost - c;   // the launch of g disappears
                if (gain > best_gain) {
                    best_gain = gain;
                    bg = g;
                    bh = h;
                    best_plans = std::move(moved);
                }
            }
        if (best_gain <= 0) break;
        BatchGroup& h = gs[bh];
        for (size_t q = 0; q < gs[bg].jobs.size(); ++q) {
            h.jobs.push_back(gs[bg].jobs[q]);
            h.plans.push_back(best_plans[q]);
            h.cost += best_plans[q].cost - cm.first(policy, h.cls);
        }
        gs.erase(gs.begin() + (long)bg);
    }
    std::sort(gs.begin(), gs.end(),
              [](const BatchGroup& a, const BatchGroup& b) { return class_len(a.cls) < class_len(b.cls); });
    *groups = std::move(gs);
    return true;
}

bool plan_batch(const std::vector<uint64_t>& ns, const std::vector<uint64_t>& ms, int policy,
                const CostModel& cm, int* cls_out, std::vector<TilePlan>* plans) {
    if (ns.empty() || ns.size() != ms.size()) return false;
    bool found = false;
    double best_cost = 0;
    std::vector<TilePlan> tmp(ns.size());
    int ids[kMaxClassId + 1];
    const int nid = class_ids(policy, ids);
    for (int q = 0; q < nid; ++q) {
        const int k = ids[q];
        double cost = cm.first(policy, k);
        bool ok = true;
        for (size_t i = 0; i < ns.size() && ok; ++i) {
            ok = plan_at_class(ns[i], ms[i], policy, k, cm, &tmp[i]);
            if (ok) cost += tmp[i].cost - cm.first(policy, k);
        }
        if (!ok) continue;
        if (!found || cost < best_cost) {
            found = true;
            best_cost = cost;
            *cls_out = k;
            *plans = tmp;
        }
    }
    return found;
}

}  // namespace pa
