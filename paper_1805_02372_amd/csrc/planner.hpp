// Tile planning: FFT length class, key-chunk and output-window sizes, and the
// rounding-error model that bounds them.  Pure host code.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

#include "pa_internal.hpp"

namespace pa {

enum Prec { PREC_FP32 = 32, PREC_FP64 = 64, PREC_NTT = 1, PREC_DIRECT = 2 };

struct ClassGeom {
    int prec, cls;        // precision, class id (pa_internal.hpp)
    uint64_t L;           // FFT length n1 * n2
    int n1, n2, b1, b3, r;
};

// Geometry of class `cls` in the given precision; false if none.
bool class_geometry(int prec, int cls, ClassGeom* g);
// ceil(log2 L)
int ceil_log2(uint64_t L);
int min_logL(int prec);
int max_logL(int prec);
// The class ids a plan of precision `prec` may use, in increasing FFT length:
// 2^min_logL <= L <= 2^min(max_logL, cap_logL).  Environment (tests and
// measurements): PA_MIN_LOG2_LEN / PA_MAX_LOG2_LEN bound L; PA_ONLY_LEN=<L>
// keeps the class of that length only; PA_POW2_ONLY=1 drops the mixed-radix
// classes.  Writes at most kMaxClassId + 1 ids; returns the count.
int class_ids(int prec, int* ids, int cap_logL = 24);
// A key of the environment settings above (plan caches depend on them).
uint64_t class_filter_key();

// Cost of a class's launches (seconds), by prec and class id: a launch of T
// tiles costs first_s + T tile_s.  tile_s is the marginal cost of a tile on a
// full device; first_s the rest of a one-tile launch (launch latency, ramp-up,
// and the part of the device one tile leaves idle).  Filled from tuning data
// when present, else from the built-in model.
struct CostModel {
    double tile_s[3][64];   // [0] FP32, [1] FP64, [2] NTT; index class id
    double first_s[3][64];  // extra cost of a launch (its first tile)
    double launch_s;        // launch cost of a class without its own first_s
    double direct_s;        // direct GF(2) path: seconds per output per 32-bit key word
    double direct_launch_s; // direct GF(2) path: fixed cost of a job (its two launches)
    CostModel();
    double tile(int prec, int cls) const;
    double first(int prec, int cls) const;
    void set(int prec, int cls, double s);
    void set_first(int prec, int cls, double s);
};
// The model a context starts from: the built-in one, replaced class by class
// by the tuning table measured on MI355X that ships beside the library
// (tune_mi355x.json next to libpa.so; PA_TUNE_DEFAULT=0 skips it).
const CostModel& default_cost_model();
// Read a tuning table (pa_tune's JSON) into cm; returns the number of values
// taken, or -1 if the file cannot be read.
int load_tune_table(CostModel& cm, const char* path);

struct TilePlan {
    int prec = 0, cls = 0;
    uint64_t L = 0;        // FFT length of the class
    uint64_t Bi = 0, Bo = 0, nchunks = 0, nouts = 0;
    double bound = 0, cost = 0;
    double rigorous = 0;   // worst-case rounding bound of a tile (any input bits)
    uint64_t tiles() const { return nchunks * nouts; }
};

// Error model of one floating-point tile, a predicted maximum of the output
// error for an FFT convolution of a +-1 sequence with a 0/1 chunk of Bi bits at
// length L: 6 sigma of the random rounding noise, sigma = kappa u
// sqrt(log2 L (Bi + L)), plus 5 times the rms of the low-frequency error that
// the chunk's zero padding causes (about 0.036 u L once Bi > L/3; the larger
// term from 2^22 on in FP32).
double error_bound(int prec, uint64_t L, uint64_t Bi);
// Worst-case (a-priori) bound of a tile's max error for any input bits:
// (||x|| + ||w||)^2 times the relative error growth of the forward FFT,
// product and inverse FFT, with ||x|| <= sqrt(Bi), ||w|| = sqrt(Bi+Bo-1).  A
// tile whose bound is below 0.5 rounds to the exact integers.
double rigorous_bound(int prec, uint64_t L, uint64_t Bi, uint64_t Bo);
constexpr double kRigorousLimit = 0.5;
void set_error_kappa(double kappa);
double error_kappa();

// The admissible error for a floating-point plan before the a-posteriori
// certificate (half the rounding margin of 0.5).
constexpr double kPlanErrorLimit = 0.25;

// Modeled time of the direct GF(2) path for one job: outputs are processed in
// blocks of 256, each against ceil(n/32) key words (rounded up to 4).
double direct_cost(uint64_t n, uint64_t m, const CostModel& cm);
// Whether the precision bits of `flags` put job (n, m) on the direct path:
// always for PA_PREC_DIRECT; for PA_PREC_AUTO when the direct path is modeled
// cheaper than the FFT plan `fft`.
bool choose_direct(uint32_t flags, uint64_t n, uint64_t m, const CostModel& cm, const TilePlan& fft);

// Best (Bi, Bo) for job (n, m) at a fixed class; false if impossible.
bool plan_at_class(uint64_t n, uint64_t m, int prec, int cls, const CostModel& cm, TilePlan* out);

// Best plan over classes for one job.  policy: PREC_FP32 (segmented, bound
// limited), PREC_FP64 and PREC_NTT (a single tile if one fits, else the
// cheapest plan over the classes).  Among plans whose modeled costs differ by
// less than 10% the one that moves fewer points wins.  Classes longer than
// 2^cap_logL are not used.
bool plan_job(uint64_t n, uint64_t m, int policy, const CostModel& cm, TilePlan* out, int cap_logL = 24);

// Jobs of a batch that share one FFT length class (one pipeline launch).
struct BatchGroup {
    int cls = 0;
    std::vector<size_t> jobs;      // indices into the batch
    std::vector<TilePlan> plans;   // plan of each job in `jobs`, at class cls
    double cost = 0;               // launch (first_s) plus tiles
};

// Batch plan with one launch per length class: every job starts in its own
// cheapest class, then a group is folded into another group's class while that
// lowers the summed cost (tiles plus one launch per group).  Groups come out
// in increasing FFT length.  `own` (optional): each job's own best plan, already
// known to the caller.
bool plan_batch_groups(const std::vector<uint64_t>& ns, const std::vector<uint64_t>& ms, int policy,
                       const CostModel& cm, std::vector<BatchGroup>* groups,
                       const std::vector<TilePlan>* own = nullptr);

// One class for a whole batch: minimises the summed cost of every job's tiles.
bool plan_batch(const std::vector<uint64_t>& ns, const std::vector<uint64_t>& ms, int policy,
                const CostModel& cm, int* cls, std::vector<TilePlan>* plans);

}  // namespace pa
