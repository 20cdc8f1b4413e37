// gf_internal.h -- the lattice object and the helpers shared by the C ABI
// (gf_capi.hip) and the pool (gf_pool.hip).  Not part of the public ABI.
#pragma once

#include <map>
#include <string>
#include <tuple>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "gf.h"
#include "gf_kernels.h"
#include "gf_su2.h"

// One lattice: geometry, device link fields and measurement scratch.
struct gf_lattice_ {
    int32_t dims[4] = {0, 0, 0, 0};
    gf_prec prec = GF_FP64;
    hipStream_t stream = nullptr;
    gf::Geom geom{};
    int64_t volume = 0;
    int64_t bytes = 0;
    gf::ChunkOf<double>::T* f64 = nullptr;  // float64 links (GF_FP64, GF_MIXED polish and rebuild)
    gf::ChunkOf<float>::T* f32 = nullptr;   // float32 links (GF_FP32, GF_MIXED bulk)
    gf::GField gacc{nullptr, 0};            // GF_MIXED: float32 g(x) accumulated by the bulk sweeps
    int phase = 0;                          // GF_MIXED: 0 = float32 bulk, 1 = float64 (after promotion)
    double* partial = nullptr;              // measurement partial sums (2 per block)
    double* dres = nullptr;                 // device results (theta, F, ...)
    double* hres = nullptr;                 // pinned host copy of dres
    double* dslices = nullptr;              // Coulomb gauge: device theta_C(t), F_C(t) pairs (2 Nt)
    double* hslices = nullptr;              // pinned host copy of dslices
    int gauge = gf::GAUGE_LANDAU;           // functional: GAUGE_LANDAU or GAUGE_COULOMB
    int group = 3;                          // gauge group SU(3) or SU(2); f64 / f32 hold quaternions for SU(2)
    bool min8 = false;                      // SU(3) links of the sweeping precision in 8 reals: f64 holds a
                                            // Link8Field (GF_FP64), f32 a Link8Field32 (GF_FP32, GF_MIXED)
    double* est = nullptr;                  // per-block sums of a sweep's theta estimate (allocated on use)
    size_t est_cap = 0;                     // doubles held by est
    bool adaptive = false;                  // gf_fix_until: exact measurement only near a decision
    double margin = 100.0;                  // ... when the estimate is below margin x the threshold
    int64_t n_measures = 0, n_estimates = 0;  // exact measurements / fused estimates taken
    bool has_links = false;
    uint32_t anneal_sweeps = 0;             // heat-bath sweep counter (Philox counter word)
    gf::SweepConfig cfg64;     // overrelaxation sweeps
    gf::SweepConfig cfg32;
    gf::SweepConfig cfg_hb64;  // heat-bath sweeps (gf_anneal)
    gf::SweepConfig cfg_hb32;
    // hipGraphs of n back-to-back sweeps, keyed by (n, omega, mode, precision
    // and g tracking plus 4 x gauge, tps, block, cache policy); only on a
    // non-default stream
    std::map<std::tuple<int32_t, double, int, int, int, int, int>, hipGraphExec_t> sweep_graphs;
};

namespace gf {
namespace detail {

extern thread_local std::string g_last_error;

gf_status fail(gf_status st, const char* fmt, ...);

#define GF_HIP(expr)                                                                                        \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return fail(e_ == hipErrorOutOfMemory ? GF_E_NOMEM : GF_E_HIP, "%s: %s (%s:%d)", #expr,         \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                         \
    } while (0)

#define GF_TRY(expr)                     \
    do {                                 \
        gf_status s_ = (expr);           \
        if (s_ != GF_OK) return s_;      \
    } while (0)

// Device buffers of one lattice (bytes; partial and nslices in doubles).
struct LatticeSizes {
    size_t f64 = 0, f32 = 0, gacc = 0, partial = 0, nslices = 0;
    int64_t total = 0;  // every device byte the lattice holds
};

LatticeSizes lattice_sizes(const Geom& g, gf_prec prec, int group = 3, bool min8 = false);
Su2Field<double> su2_64(const gf_lattice_* L);
Su2Field<float> su2_32(const gf_lattice_* L);
// Doubles per link of the canonical host / device arrays (18 for SU(3), 8 for SU(2)).
inline size_t canon_per_link(const gf_lattice_* L)
{
    return L->group == 2 ? 8 : 18;
}
bool make_fastdiv(uint32_t d, uint32_t limit, FastDiv* out);
bool make_geom(const int32_t dims[4], Geom* out);
gf_status check_dims(const int32_t dims[4], int64_t* V);
LinkField<double> field64(const gf_lattice_* L);
Link8Field field8(const gf_lattice_* L);
Link8Field32 field8f(const gf_lattice_* L);
LinkField<float> field32(const gf_lattice_* L);
bool is_fp32(const gf_lattice_* L);
// The float64 field is in 8 reals (GF_FP64 lattices only; a GF_MIXED lattice
// keeps its float64 links in 12).
inline bool min8_64(const gf_lattice_* L)
{
    return L->min8 && L->prec == GF_FP64;
}
GField g_tracking(const gf_lattice_* L);
gf_status check_ready(gf_lattice L);
gf_status check_omega(double omega, int mode);
gf_status do_half_sweep(gf_lattice L, int parity, double omega, int mode);
gf_status do_sweeps(gf_lattice L, int32_t n, double omega, int mode);
gf_status do_reunitarize(gf_lattice L);
gf_status do_promote(gf_lattice L);
gf_status do_measure(gf_lattice L, double* theta, double* F);
gf_status measure_enqueue(gf_lattice L, hipStream_t st);
gf_status measure_read(gf_lattice L, double* theta, double* F);
gf_status do_est_sweep(gf_lattice L, double omega, int mode, double* theta_est);
gf_status do_fp32_floor(gf_lattice L, double* floor);
gf_status resolve_switch(gf_lattice L, double theta_target, double theta_switch, double* out);
gf_status upload_canonical(gf_lattice L, const double* dev_canon);
gf_status download_canonical(gf_lattice L, double* dev_canon);
gf_status do_set_storage(gf_lattice L, bool min8);
gf_status create_lattice(const int32_t dims[4], gf_prec prec, int group, bool min8, void* hip_stream,
                         gf_lattice* out);
void release(gf_lattice L);

// Float32 phase of GF_MIXED: it is left once theta < theta_switch, or once
// theta has reached no new minimum for kStallChecks consecutive checks with
// its best value below kStallTheta (update_stall runs after every check that
// followed sweeps).  Float32 rounding puts a floor of about 1e-12 under theta
// (a few float32 units of |K| in each component of Delta); a stall well above
// it is the iteration's own slow convergence, which float32 sweeps pursue as
// well as float64 ones at half the traffic, so it does not end the phase.
constexpr int kStallChecks = 16;
constexpr double kStallTheta = 1e-10;

// Chosen switch point (theta_switch < 0 in gf_fix_params):
// max(theta_target, kFloorMargin * floor), floor = the lattice's float32
// rounding floor of theta (launch_fp32_floor).  Float32 sweeps converge at the
// float64 rate while theta is well above that floor (on MI355X: identical
// sweep counts to theta < 1e-12 for every switch point from 1e-8 down to the
// target), so the float32 phase is run as far as the floor allows.
constexpr double kFloorMargin = 100.0;

inline bool leave_fp32(double theta, double theta_switch, double best, int stall)
{
    return theta < theta_switch || (stall >= kStallChecks && best < kStallTheta);
}

// Multi-sweep calls on a non-default stream are captured once as a hipGraph
// and replayed while the lattice has fewer than this many sites per colour;
// larger lattices launch directly: their kernels hide the launch cost, and on
// MI355X replayed kernels of a 32^4 lattice took 2-6 % longer than the same
// kernels launched directly.
constexpr uint32_t kGraphMaxHalfSites = 1u << 16;

// A named range on the roctx marker stream for the lifetime of the object
// (rocprofv3 --marker-trace shows it around the kernels it encloses; without
// a profiler attached the calls do nothing).
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

inline void update_stall(double theta, double* best, int* stall)
{
    if (theta < *best) {
        *best = theta;
        *stall = 0;
    } else {
        ++*stall;
    }
}

// Temperature of annealing sweep s of n: linear from T_start (s = 0) to T_end
// (s = n - 1), both endpoints exact.
inline double anneal_temperature(int32_t s, int32_t n, double T_start, double T_end)
{
    if (n <= 1 || s == 0) return T_start;
    if (s == n - 1) return T_end;
    return T_start + (T_end - T_start) * (double)s / (double)(n - 1);
}

}  // namespace detail
}  // namespace gf
