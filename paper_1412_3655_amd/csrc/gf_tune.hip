// gf_tune.hip -- run-time autotuning of the sweep kernel (include/gf.h,
// gf_autotune).  The paper's cuLGT2 picks 4 or 8 threads per site, register
// limits and texture loads by trying them at run time (Sec. 4 and 5); here the
// axes are lanes per site (1, 2, 4, 8), threads per block (64..512), the
// cache policy of the link accesses (plain / non-temporal / non-temporal
// stores only) and the register limit (the compiler's allocation, or at most
// 256 registers for 2 waves per SIMD), timed with HIP events on a scratch copy
// of the links so the lattice is unchanged.  The kernel timed is that of the lattice's gauge.
// Every configuration gives bitwise the same links, so only time decides.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gf_internal.h"

using namespace gf;
using namespace gf::detail;

namespace {

// timing rounds over the configurations (each keeps its fastest)
constexpr int kTuneRounds = 2;

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// A GF_MIXED lattice's float32 sweeps also update g(x) (another 96 B per site
// update and more registers), so they are a kernel of their own: "fp32g".  The
// Coulomb kernels (K over three directions) are keyed apart with a "-coulomb"
// suffix, SU(2) lattices with "-su2" and 8-real links with "-min8".
std::string cache_key(gf_lattice L, gf_prec kernel, bool min8)
{
    char buf[128];
    const char* k = kernel == GF_FP64 ? "fp64" : (L->gacc.base ? "fp32g" : "fp32");
    snprintf(buf, sizeof buf, "%s %d %d %d %d %s%s%s%s", device_arch().c_str(), L->dims[0], L->dims[1], L->dims[2],
             L->dims[3], k, L->gauge == GAUGE_COULOMB ? "-coulomb" : "", L->group == 2 ? "-su2" : "",
             min8 ? "-min8" : "");
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, SweepConfig* out)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        if (strncmp(line, key.c_str(), key.size()) != 0 || line[key.size()] != ' ') continue;
        int t = 0, b = 0, nt = 0, w = 0;
        double us = 0.0;
        const int got = sscanf(line + key.size(), "%d %d %d %d %lf", &t, &b, &nt, &w, &us);
        if (got < 5) w = 0;  // lines of three values: written before the register-limit axis
        const SweepConfig c{t, b, nt, w};
        if (got >= 3 && (sweep_config_valid(c) || su2_config_valid(c))) {
            *out = c;
            found = true;  // the last matching line wins
        }
    }
    fclose(f);
    return found;
}

// Time every valid configuration of the overrelaxation sweep (heat_bath =
// false) or of the heat-bath sweep (true, at T = 1) of precision `kernel` on a
// scratch copy of the links, apply the fastest to the lattice and append it to
// the cache; shared by gf_autotune and gf_autotune_anneal.
// other_storage (SU(3) lattices, kernel = the lattice's sweeping precision:
// GF_FP64 for GF_FP64 lattices, GF_FP32 for GF_FP32 and GF_MIXED): time the
// sweep of the lattice's links converted to the other storage (12 <-> 8
// reals) on the scratch copy, and leave the lattice's configuration alone (the
// caller decides whether to switch).
gf_status tune(gf_lattice L, gf_prec kernel, bool heat_bath, int32_t n_sweeps, const char* cache_path,
               gf_tune_entry* table, int32_t cap, int32_t* n_out, gf_tune_entry* chosen, bool other_storage = false)
{
    GF_TRY(check_ready(L));
    if (kernel != GF_FP64 && kernel != GF_FP32) return fail(GF_E_ARG, "kernel precision must be GF_FP64 or GF_FP32");
    if ((kernel == GF_FP64 && !L->f64) || (kernel == GF_FP32 && !L->f32))
        return fail(GF_E_ARG, "the lattice has no links of that precision");
    if (n_sweeps < 1 || cap < 0 || (cap > 0 && !table)) return fail(GF_E_ARG, "bad arguments");
    if (n_out) *n_out = 0;
    if (other_storage && (L->group != 3 || (kernel == GF_FP64) != (L->prec == GF_FP64)))
        return fail(GF_E_STATE, "the storage of links can change for SU(3) links of the sweeping precision only");
    const bool cur8 = kernel == GF_FP64 ? min8_64(L) : L->min8;  // storage of the kernel's links
    const bool m8 = cur8 != other_storage;                       // storage of the links timed
    SweepConfig scratch_target{};
    SweepConfig& target = other_storage ? scratch_target
                                        : heat_bath ? (kernel == GF_FP32 ? L->cfg_hb32 : L->cfg_hb64)
                                                    : (kernel == GF_FP32 ? L->cfg32 : L->cfg64);
    const std::string key = cache_key(L, kernel, m8) + (heat_bath ? "-hb" : "");
    SweepConfig best{};
    if (cache_path && cache_lookup(cache_path, key, &best)) {
        target = best;
        if (chosen) *chosen = gf_tune_entry{best.tps, best.block, best.nt, best.minw, 0.0};
        return GF_OK;
    }

    const bool su2 = L->group == 2;
    const size_t chunks = (size_t)2 * 4 * L->geom.ld *
                          (kernel == GF_FP32 ? (su2 ? 1 : (m8 ? kMin8Chunks32 : 3)) : (su2 ? 2 : (m8 ? kMin8Chunks : 6)));
    const size_t bytes = chunks * 16;
    void* scratch = nullptr;
    void* gscratch = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    gf_status st = GF_OK;
    double best_us = 1e300;
    int n = 0;
    const bool track = kernel == GF_FP32 && L->gacc.base != nullptr;
    const size_t gbytes = (size_t)2 * 3 * L->geom.ld * 16;
    hipError_t e = hipMalloc(&scratch, bytes);
    if (e == hipSuccess && track) e = hipMalloc(&gscratch, gbytes);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess && other_storage && kernel == GF_FP32 && m8)
        e = launch_convert(field32(L), Link8Field32{(float4*)scratch, L->geom.ld}, L->geom, L->stream);
    else if (e == hipSuccess && other_storage && kernel == GF_FP32)
        e = launch_convert(field8f(L), LinkField<float>{(float4*)scratch, L->geom.ld}, L->geom, L->stream);
    else if (e == hipSuccess && other_storage && m8)
        e = launch_convert(field64(L), Link8Field{(double2*)scratch, L->geom.ld}, L->geom, L->stream);
    else if (e == hipSuccess && other_storage)
        e = launch_convert(field8(L), LinkField<double>{(double2*)scratch, L->geom.ld}, L->geom, L->stream);
    else if (e == hipSuccess)
        e = hipMemcpyAsync(scratch, kernel == GF_FP32 ? (void*)L->f32 : (void*)L->f64, bytes, hipMemcpyDeviceToDevice,
                           L->stream);
    if (e == hipSuccess && track) e = hipMemcpyAsync(gscratch, L->gacc.base, gbytes, hipMemcpyDeviceToDevice, L->stream);
    const GField g_none{nullptr, 0};
    const GField g_s{(float4*)gscratch, L->geom.ld};
    const LinkField<float> f32{(float4*)scratch, L->geom.ld};
    const LinkField<double> f64{(double2*)scratch, L->geom.ld};
    const Su2Field<float> q32{(float4*)scratch, L->geom.ld};
    const Su2Field<double> q64{(double2*)scratch, L->geom.ld};
    const Link8Field f8{(double2*)scratch, L->geom.ld};
    const Link8Field32 f8f{(float4*)scratch, L->geom.ld};
    uint32_t hb_sweep = 0;
    // the register cap changes only the one-lane float64 kernel (every other
    // shape already runs 2 or more waves per SIMD)
    const bool cap_axis = !su2 && !m8 && kernel == GF_FP64;
    std::vector<SweepConfig> configs;
    for (int minw : {0, 2})
        for (int nt : {0, 1, 2})
            for (int tps : {1, 2, 4, 8})
                for (int block : {64, 128, 256, 512}) {
                    const SweepConfig c{tps, block, nt, minw};
                    if (minw && !cap_axis) continue;
                    if (su2 ? su2_config_valid(c) : sweep_config_valid(c)) configs.push_back(c);
                }
    // Two timing rounds over all configurations, each configuration keeping its
    // faster time: a slow moment of the device (clocks, other traffic) then
    // costs a configuration only if it recurs at the same point of both rounds.
    std::vector<double> us_of(configs.size(), 1e300);
    for (int round = 0; round < kTuneRounds && e == hipSuccess; ++round) {
        for (size_t ci = 0; ci < configs.size() && e == hipSuccess; ++ci) {
            const SweepConfig& c = configs[ci];
            auto sweep = [&]() -> hipError_t {
                for (int p = 0; p < 2; ++p) {
                    hipError_t r;
                    if (su2 && heat_bath && kernel == GF_FP32)
                        r = launch_su2_hb(q32, L->geom, p, 1.0f, 1u, hb_sweep, c, L->stream, L->gauge);
                    else if (su2 && heat_bath)
                        r = launch_su2_hb(q64, L->geom, p, 1.0, 1u, hb_sweep, c, L->stream, L->gauge);
                    else if (su2 && kernel == GF_FP32)
                        r = launch_su2_or(q32, L->geom, p, 1.7f, GF_OR_EXACT, c, L->stream, L->gauge, nullptr);
                    else if (su2)
                        r = launch_su2_or(q64, L->geom, p, 1.7, GF_OR_EXACT, c, L->stream, L->gauge, nullptr);
                    else if (m8 && heat_bath && kernel == GF_FP32)
                        r = launch_hb_half_sweep(f8f, L->geom, p, 1.0f, 1u, hb_sweep, c, track ? g_s : g_none,
                                                 L->stream, L->gauge);
                    else if (m8 && kernel == GF_FP32)
                        r = launch_or_half_sweep(f8f, L->geom, p, 1.7f, GF_OR_EXACT, c, track ? g_s : g_none,
                                                 L->stream, L->gauge);
                    else if (m8 && heat_bath)
                        r = launch_hb_half_sweep(f8, L->geom, p, 1.0, 1u, hb_sweep, c, L->stream, L->gauge);
                    else if (m8)
                        r = launch_or_half_sweep(f8, L->geom, p, 1.7, GF_OR_EXACT, c, L->stream, L->gauge);
                    else if (heat_bath && kernel == GF_FP32)
                        r = launch_hb_half_sweep(f32, L->geom, p, 1.0f, 1u, hb_sweep, c, track ? g_s : g_none,
                                                 L->stream, L->gauge);
                    else if (heat_bath)
                        r = launch_hb_half_sweep(f64, L->geom, p, 1.0, 1u, hb_sweep, c, L->stream, L->gauge);
                    else if (kernel == GF_FP32)
                        r = launch_or_half_sweep(f32, L->geom, p, 1.7f, GF_OR_EXACT, c, track ? g_s : g_none,
                                                 L->stream, L->gauge);
                    else
                        r = launch_or_half_sweep(f64, L->geom, p, 1.7, GF_OR_EXACT, c, L->stream, L->gauge);
                    if (r != hipSuccess) return r;
                }
                ++hb_sweep;
                return hipSuccess;
            };
            e = sweep();
            if (e == hipSuccess) e = hipEventRecord(e0, L->stream);
            for (int k = 0; k < n_sweeps && e == hipSuccess; ++k) e = sweep();
            if (e == hipSuccess) e = hipEventRecord(e1, L->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) us_of[ci] = std::min(us_of[ci], 1e3 * (double)ms / n_sweeps);
        }
    }
    if (e == hipSuccess) {
        for (size_t ci = 0; ci < configs.size(); ++ci) {
            const SweepConfig& c = configs[ci];
            if (n < cap) table[n] = gf_tune_entry{c.tps, c.block, c.nt, c.minw, us_of[ci]};
            ++n;
            if (us_of[ci] < best_us) {
                best_us = us_of[ci];
                best = c;
            }
        }
    }
    if (e != hipSuccess) st = fail(GF_E_HIP, "autotune: %s", hipGetErrorString(e));
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(L->stream);
    if (scratch) (void)hipFree(scratch);
    if (gscratch) (void)hipFree(gscratch);
    if (st != GF_OK) return st;
    target = best;
    if (n_out) *n_out = std::min(n, cap);
    if (chosen) *chosen = gf_tune_entry{best.tps, best.block, best.nt, best.minw, best_us};
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s %d %d %d %d %.3f\n", key.c_str(), best.tps, best.block, best.nt, best.minw, best_us);
            fclose(f);
        }
    }
    return GF_OK;
}

}  // namespace

extern "C" gf_status gf_autotune(gf_lattice L, gf_prec kernel, int32_t n_sweeps, const char* cache_path,
                                 gf_tune_entry* table, int32_t cap, int32_t* n_out, gf_tune_entry* chosen)
{
    TraceRange range("gf_autotune");
    return tune(L, kernel, false, n_sweeps, cache_path, table, cap, n_out, chosen);
}

extern "C" gf_status gf_autotune_storage(gf_lattice L, int32_t n_sweeps, int32_t* reals_per_link, double* us_12,
                                         double* us_8)
{
    TraceRange range("gf_autotune_storage");
    GF_TRY(check_ready(L));
    if (L->group != 3) return fail(GF_E_STATE, "the storage of links can change on SU(3) lattices only");
    // the links of the sweeping precision: float64 of GF_FP64, float32 of GF_FP32 and GF_MIXED
    const gf_prec kernel = L->prec == GF_FP64 ? GF_FP64 : GF_FP32;
    gf_tune_entry cur{}, oth{};
    GF_TRY(tune(L, kernel, false, n_sweeps, nullptr, nullptr, 0, nullptr, &cur, false));
    GF_TRY(tune(L, kernel, false, n_sweeps, nullptr, nullptr, 0, nullptr, &oth, true));
    const double t_cur = cur.us_per_sweep, t_oth = oth.us_per_sweep;
    if (us_12) *us_12 = L->min8 ? t_oth : t_cur;
    if (us_8) *us_8 = L->min8 ? t_cur : t_oth;
    if (t_oth < t_cur) {
        GF_TRY(do_set_storage(L, !L->min8));
        (kernel == GF_FP64 ? L->cfg64 : L->cfg32) = SweepConfig{oth.tps, oth.block, oth.nontemporal, oth.min_waves};
    }
    if (reals_per_link) *reals_per_link = L->min8 ? 8 : 12;
    return GF_OK;
}

extern "C" gf_status gf_autotune_anneal(gf_lattice L, gf_prec kernel, int32_t n_sweeps, const char* cache_path,
                                        gf_tune_entry* table, int32_t cap, int32_t* n_out, gf_tune_entry* chosen)
{
    TraceRange range("gf_autotune_anneal");
    return tune(L, kernel, true, n_sweeps, cache_path, table, cap, n_out, chosen);
}
