// gf_capi.hip -- the C ABI of libgf (declared in include/gf.h): lattice
// objects, argument checking, the fix-until driver (Sec. 2 of
// arXiv:1412.3655: sweep black then white, iterate until the gauge condition
// holds to a given precision) and error reporting.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "gf_internal.h"

using gf::FastDiv;
using gf::Geom;
using gf::LinkField;
using gf::SweepConfig;

namespace gf {
namespace detail {

thread_local std::string g_last_error;

gf_status fail(gf_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

// d >= 1; exact for 0 <= n < limit (checked exhaustively).
bool make_fastdiv(uint32_t d, uint32_t limit, FastDiv* out)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    FastDiv f;
    f.m = (uint64_t)(((unsigned __int128)1 << (32 + l)) / d) + 1;
    f.shift = 32 + l;
    f.d = d;
    for (uint32_t n = 0; n < limit; ++n)
        if ((uint32_t)(((unsigned __int128)n * f.m) >> f.shift) != n / d) return false;
    *out = f;
    return true;
}

// Geometry of a lattice of extents dims (each even and >= 2, V <= 2^31;
// checked by the caller).  False if a magic-number division fails its check.
bool make_geom(const int32_t dims[4], Geom* out)
{
    Geom g{};
    int64_t V = 1;
    for (int m = 0; m < 4; ++m) {
        g.n[m] = dims[m];
        V *= dims[m];
    }
    g.hx = dims[0] / 2;
    g.vh = (uint32_t)(V / 2);
    g.ld = (g.vh + gf::kLinkTile - 1) / gf::kLinkTile * gf::kLinkTile;  // whole tiles of the link layout
    g.hs1 = (uint32_t)g.hx;
    g.hs2 = (uint32_t)g.hx * (uint32_t)dims[1];
    g.hs3 = g.hs2 * (uint32_t)dims[2];
    if (!make_fastdiv((uint32_t)g.hx, g.vh, &g.div_hx) ||
        !make_fastdiv((uint32_t)dims[1], g.vh / (uint32_t)g.hx, &g.div_ny) ||
        !make_fastdiv((uint32_t)dims[2], g.vh / g.hs2, &g.div_nz))
        return false;
    *out = g;
    return true;
}

// Extents each even and >= 2 with at most 2^31 sites; *V receives the volume.
gf_status check_dims(const int32_t dims[4], int64_t* V)
{
    if (!dims) return fail(GF_E_ARG, "null extents");
    int64_t v = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 2 || dims[m] % 2 != 0)
            return fail(GF_E_ARG, "extent %d of direction %d must be even and >= 2", dims[m], m);
        v *= dims[m];
    }
    if (v > (int64_t)1 << 31) return fail(GF_E_ARG, "volume %lld exceeds 2^31 sites", (long long)v);
    *V = v;
    return GF_OK;
}

// Device allocations of a lattice of geometry g and precision prec (sizes of
// the buffers gf_create_lattice allocates; the pool's admission budget counts
// exactly these).
LatticeSizes lattice_sizes(const Geom& g, gf_prec prec, int group, bool min8)
{
    LatticeSizes z;
    const size_t nchunks = (size_t)2 * 4 * g.ld;  // per chunk slot
    const bool su2 = group == 2;
    // min8: the links of the lattice's sweeping precision in 8 reals (the
    // float64 field of GF_FP64, the float32 field of GF_FP32 and GF_MIXED)
    const size_t c64 = su2 ? 2 : (min8 && prec == GF_FP64 ? (size_t)gf::kMin8Chunks : 6);
    const size_t c32 = su2 ? 1 : (min8 ? (size_t)gf::kMin8Chunks32 : 3);
    if (prec == GF_FP64 || prec == GF_MIXED) z.f64 = nchunks * c64 * sizeof(double2);
    if (prec == GF_FP32 || prec == GF_MIXED) z.f32 = nchunks * c32 * sizeof(float4);
    if (prec == GF_MIXED) z.gacc = (size_t)2 * 3 * g.ld * sizeof(float4);
    // partial sums of the whole-lattice reductions, or of the per-timeslice
    // Coulomb ones, whichever needs more
    z.partial = su2 ? 2 * (size_t)gf::su2_partials(g)
                    : 2 * std::max((size_t)gf::measure_blocks(g), (size_t)gf::slice_partials(g));
    z.nslices = 2 * (size_t)g.n[3];
    z.total = (int64_t)(z.f64 + z.f32 + z.gacc + (z.partial + 4 + z.nslices) * sizeof(double));
    return z;
}

LinkField<double> field64(const gf_lattice_* L)
{
    return LinkField<double>{L->f64, L->geom.ld};
}

Link8Field field8(const gf_lattice_* L)
{
    return Link8Field{L->f64, L->geom.ld};
}

LinkField<float> field32(const gf_lattice_* L)
{
    return LinkField<float>{L->f32, L->geom.ld};
}

Link8Field32 field8f(const gf_lattice_* L)
{
    return Link8Field32{L->f32, L->geom.ld};
}

Su2Field<double> su2_64(const gf_lattice_* L)
{
    return Su2Field<double>{L->f64, L->geom.ld};
}

Su2Field<float> su2_32(const gf_lattice_* L)
{
    return Su2Field<float>{L->f32, L->geom.ld};
}

// Whether the working links are the float32 field (GF_FP32, or GF_MIXED before promotion).
bool is_fp32(const gf_lattice_* L)
{
    return L->prec == GF_FP32 || (L->prec == GF_MIXED && L->phase == 0);
}

gf::GField g_tracking(const gf_lattice_* L)
{
    return L->prec == GF_MIXED && L->phase == 0 ? L->gacc : gf::GField{nullptr, 0};
}

gf_status check_ready(gf_lattice L)
{
    if (!L) return fail(GF_E_ARG, "null lattice");
    if (!L->has_links) return fail(GF_E_STATE, "links were never set on this lattice");
    return GF_OK;
}

gf_status check_omega(double omega, int mode)
{
    if (!(omega >= 1.0 && omega < 2.0)) return fail(GF_E_ARG, "omega = %g is outside [1, 2)", omega);
    if (mode != GF_OR_EXACT && mode != GF_OR_BINOMIAL1) return fail(GF_E_ARG, "unknown overrelaxation mode %d", mode);
    return GF_OK;
}

gf_status do_half_sweep(gf_lattice L, int parity, double omega, int mode)
{
    if (L->group == 2) {
        if (is_fp32(L))
            GF_HIP(gf::launch_su2_or(su2_32(L), L->geom, parity, (float)omega, mode, L->cfg32, L->stream, L->gauge,
                                     nullptr));
        else
            GF_HIP(gf::launch_su2_or(su2_64(L), L->geom, parity, omega, mode, L->cfg64, L->stream, L->gauge, nullptr));
        return GF_OK;
    }
    if (min8_64(L))
        GF_HIP(gf::launch_or_half_sweep(field8(L), L->geom, parity, omega, mode, L->cfg64, L->stream, L->gauge));
    else if (is_fp32(L) && L->min8)
        GF_HIP(gf::launch_or_half_sweep(field8f(L), L->geom, parity, (float)omega, mode, L->cfg32, g_tracking(L),
                                        L->stream, L->gauge));
    else if (is_fp32(L))
        GF_HIP(gf::launch_or_half_sweep(field32(L), L->geom, parity, (float)omega, mode, L->cfg32, g_tracking(L),
                                        L->stream, L->gauge));
    else
        GF_HIP(gf::launch_or_half_sweep(field64(L), L->geom, parity, omega, mode, L->cfg64, L->stream, L->gauge));
    return GF_OK;
}

gf_status launch_sweeps(gf_lattice L, int32_t n, double omega, int mode)
{
    for (int32_t k = 0; k < n; ++k) {
        GF_TRY(do_half_sweep(L, 0, omega, mode));
        GF_TRY(do_half_sweep(L, 1, omega, mode));
    }
    return GF_OK;
}

void clear_graphs(gf_lattice L)
{
    for (auto& kv : L->sweep_graphs) (void)hipGraphExecDestroy(kv.second);
    L->sweep_graphs.clear();
}

// n sweeps.  On a non-default stream runs of two or more sweeps on a lattice
// of fewer than kGraphMaxHalfSites sites per colour are captured once in a
// hipGraph (kernel nodes only) and replayed, which removes the launch gaps
// between the 2n short half-sweeps; larger lattices launch directly.
gf_status do_sweeps(gf_lattice L, int32_t n, double omega, int mode)
{
    if (n < 2 || L->stream == nullptr || L->geom.vh >= kGraphMaxHalfSites) return launch_sweeps(L, n, omega, mode);
    const bool fp32 = is_fp32(L);
    const SweepConfig& c = fp32 ? L->cfg32 : L->cfg64;
    const int kind = (fp32 ? (g_tracking(L).base ? 2 : 1) : 0) + 4 * L->gauge + 8 * (L->group == 2) + 16 * L->min8;
    const auto key = std::make_tuple(n, omega, mode, kind, c.tps, c.block, c.nt + 4 * c.minw);
    auto it = L->sweep_graphs.find(key);
    if (it == L->sweep_graphs.end()) {
        if (L->sweep_graphs.size() >= 16) clear_graphs(L);
        hipGraph_t graph = nullptr;
        GF_HIP(hipStreamBeginCapture(L->stream, hipStreamCaptureModeRelaxed));
        gf_status st = launch_sweeps(L, n, omega, mode);
        hipError_t e = hipStreamEndCapture(L->stream, &graph);
        if (st != GF_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(GF_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(GF_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        it = L->sweep_graphs.emplace(key, exec).first;
    }
    GF_HIP(hipGraphLaunch(it->second, L->stream));
    return GF_OK;
}

gf_status do_reunitarize(gf_lattice L)
{
    // 8-real links decode to SU(3) to rounding and are re-encoded from rows 0
    // and 1 at every store: they are reunitarised at every sweep already (g(x)
    // of a GF_MIXED lattice is not)
    if (L->group == 2) {
        if (is_fp32(L))
            GF_HIP(gf::launch_su2_reunitarize(su2_32(L), L->geom, L->stream));
        else
            GF_HIP(gf::launch_su2_reunitarize(su2_64(L), L->geom, L->stream));
        return GF_OK;
    }
    if (is_fp32(L) && !L->min8)
        GF_HIP(gf::launch_reunitarize(field32(L), L->geom, L->stream));
    else if (!is_fp32(L) && !min8_64(L))
        GF_HIP(gf::launch_reunitarize(field64(L), L->geom, L->stream));
    if (g_tracking(L).base) GF_HIP(gf::launch_g_reunitarize(L->gacc, L->geom, L->stream));
    return GF_OK;
}

// GF_MIXED: leave the float32 phase.  The float64 field still holds the
// original links U0; it becomes g(x) U0_mu(x) g(x+mu^)^dag, which is on the
// gauge orbit of U0 to float64 precision whatever the float32 rounding did.
gf_status do_promote(gf_lattice L)
{
    if (L->prec != GF_MIXED || L->phase != 0) return GF_OK;
    GF_HIP(gf::launch_rebuild_from_g(field64(L), L->gacc, L->geom, L->stream));
    L->phase = 1;
    return GF_OK;
}

// The measurement's kernels and the copy of its result to pinned host memory,
// enqueued on `st` (the lattice's stream, or another one that no work on the
// lattice runs on meanwhile); measure_read takes the result after `st` has
// been synchronised.
gf_status measure_enqueue(gf_lattice L, hipStream_t st)
{
    if (L->gauge == gf::GAUGE_COULOMB) {
        if (L->group == 2 && is_fp32(L))
            GF_HIP(gf::launch_su2_measure(su2_32(L), L->geom, gf::GAUGE_COULOMB, L->partial, L->dslices, st));
        else if (L->group == 2)
            GF_HIP(gf::launch_su2_measure(su2_64(L), L->geom, gf::GAUGE_COULOMB, L->partial, L->dslices, st));
        else if (min8_64(L))
            GF_HIP(gf::launch_measure_slices(field8(L), L->geom, L->partial, L->dslices, st));
        else if (is_fp32(L) && L->min8)
            GF_HIP(gf::launch_measure_slices(field8f(L), L->geom, L->partial, L->dslices, st));
        else if (is_fp32(L))
            GF_HIP(gf::launch_measure_slices(field32(L), L->geom, L->partial, L->dslices, st));
        else
            GF_HIP(gf::launch_measure_slices(field64(L), L->geom, L->partial, L->dslices, st));
        GF_HIP(hipMemcpyAsync(L->hslices, L->dslices, 2 * (size_t)L->dims[3] * sizeof(double), hipMemcpyDeviceToHost,
                              st));
        return GF_OK;
    }
    if (L->group == 2 && is_fp32(L))
        GF_HIP(gf::launch_su2_measure(su2_32(L), L->geom, gf::GAUGE_LANDAU, L->partial, L->dres, st));
    else if (L->group == 2)
        GF_HIP(gf::launch_su2_measure(su2_64(L), L->geom, gf::GAUGE_LANDAU, L->partial, L->dres, st));
    else if (min8_64(L))
        GF_HIP(gf::launch_measure(field8(L), L->geom, L->partial, L->dres, st));
    else if (is_fp32(L) && L->min8)
        GF_HIP(gf::launch_measure(field8f(L), L->geom, L->partial, L->dres, st));
    else if (is_fp32(L))
        GF_HIP(gf::launch_measure(field32(L), L->geom, L->partial, L->dres, st));
    else
        GF_HIP(gf::launch_measure(field64(L), L->geom, L->partial, L->dres, st));
    GF_HIP(hipMemcpyAsync(L->hres, L->dres, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    return GF_OK;
}

// Coulomb gauge: theta_C(t), F_C(t) of every timeslice are in L->hslices;
// *theta = the largest theta_C(t) (the condition holds once it holds in every
// timeslice), *F = the mean of F_C(t), added in timeslice order.
gf_status measure_read(gf_lattice L, double* theta, double* F)
{
    if (L->gauge == gf::GAUGE_COULOMB) {
        const int nt = L->dims[3];
        double th = 0.0, f = 0.0;
        bool finite = true;
        for (int t = 0; t < nt; ++t) {
            const double a = L->hslices[2 * t], b = L->hslices[2 * t + 1];
            finite = finite && std::isfinite(a) && std::isfinite(b);
            if (a > th) th = a;
            f += b;
        }
        *theta = th;
        *F = f / (double)nt;
        if (!finite) return fail(GF_E_NUMERIC, "a timeslice's theta_C or F_C is not finite");
        return GF_OK;
    }
    *theta = L->hres[0];
    *F = L->hres[1];
    if (!std::isfinite(*theta) || !std::isfinite(*F))
        return fail(GF_E_NUMERIC, "theta = %g, F = %g is not finite", *theta, *F);
    return GF_OK;
}

gf_status do_measure(gf_lattice L, double* theta, double* F)
{
    ++L->n_measures;
    GF_TRY(measure_enqueue(L, L->stream));
    GF_HIP(hipStreamSynchronize(L->stream));
    return measure_read(L, theta, F);
}

// One sweep whose half-sweeps also sum tr[Delta Delta^dag] of every site's K
// just before its update; *theta_est = that sum / (3V): the black sites'
// terms before the black half-sweep, the white sites' after it.  It tracks
// theta one sweep behind (for Coulomb gauge: the mean over timeslices of
// theta_C, never above their maximum).  The links are updated exactly as by a
// plain sweep.  Syncs.
gf_status do_est_sweep(gf_lattice L, double omega, int mode, double* theta_est)
{
    const SweepConfig& c = is_fp32(L) ? L->cfg32 : L->cfg64;
    const bool su2 = L->group == 2;
    const uint32_t nb = su2 ? gf::su2_sweep_blocks(L->geom, c) : gf::sweep_blocks(L->geom, c);
    const size_t need = 4 * (size_t)nb;
    if (need > L->est_cap) {
        if (L->est) GF_HIP(hipFree(L->est));
        L->bytes -= (int64_t)(L->est_cap * sizeof(double));
        L->est = nullptr;
        L->est_cap = 0;
        GF_HIP(hipMalloc((void**)&L->est, need * sizeof(double)));
        L->est_cap = need;
        L->bytes += (int64_t)(need * sizeof(double));
    }
    for (int parity = 0; parity < 2; ++parity) {
        if (su2 && is_fp32(L))
            GF_HIP(gf::launch_su2_or(su2_32(L), L->geom, parity, (float)omega, mode, L->cfg32, L->stream, L->gauge,
                                     L->est));
        else if (su2)
            GF_HIP(gf::launch_su2_or(su2_64(L), L->geom, parity, omega, mode, L->cfg64, L->stream, L->gauge, L->est));
        else if (min8_64(L))
            GF_HIP(gf::launch_or_half_sweep(field8(L), L->geom, parity, omega, mode, L->cfg64, L->stream, L->gauge,
                                            L->est));
        else if (is_fp32(L) && L->min8)
            GF_HIP(gf::launch_or_half_sweep(field8f(L), L->geom, parity, (float)omega, mode, L->cfg32, g_tracking(L),
                                            L->stream, L->gauge, L->est));
        else if (is_fp32(L))
            GF_HIP(gf::launch_or_half_sweep(field32(L), L->geom, parity, (float)omega, mode, L->cfg32, g_tracking(L),
                                            L->stream, L->gauge, L->est));
        else
            GF_HIP(gf::launch_or_half_sweep(field64(L), L->geom, parity, omega, mode, L->cfg64, L->stream, L->gauge,
                                            L->est));
    }
    const double V = 2.0 * (double)L->geom.vh;
    const double nc = su2 ? 2.0 : 3.0;
    GF_HIP(gf::launch_finalize(L->est, 2 * nb, 1.0 / (nc * V), 0.0, L->dres + 2, L->stream));
    GF_HIP(hipMemcpyAsync(L->hres + 2, L->dres + 2, sizeof(double), hipMemcpyDeviceToHost, L->stream));
    GF_HIP(hipStreamSynchronize(L->stream));
    ++L->n_estimates;
    *theta_est = L->hres[2];
    return GF_OK;
}

gf_status do_fp32_floor(gf_lattice L, double* floor)
{
    if (L->group == 2) return fail(GF_E_STATE, "the float32 floor is defined for SU(3) lattices");
    if (min8_64(L)) return fail(GF_E_STATE, "the float32 floor needs float64 links in 12 reals");
    if (!L->f64) return fail(GF_E_STATE, "the float32 floor needs float64 links (GF_FP64 or GF_MIXED lattice)");
    // a GF_MIXED lattice in 8 reals: the floor of its 8-real float32 links
    GF_HIP(gf::launch_fp32_floor(field64(L), L->geom, L->partial, L->dres, L->stream, L->min8));
    GF_HIP(hipMemcpyAsync(L->hres, L->dres, sizeof(double), hipMemcpyDeviceToHost, L->stream));
    GF_HIP(hipStreamSynchronize(L->stream));
    *floor = L->hres[0];
    if (!std::isfinite(*floor)) return fail(GF_E_NUMERIC, "float32 floor = %g is not finite", *floor);
    return GF_OK;
}

gf_status resolve_switch(gf_lattice L, double theta_target, double theta_switch, double* out)
{
    if (theta_switch >= 0.0 || L->prec != GF_MIXED || L->phase != 0) {
        *out = theta_switch;
        return GF_OK;
    }
    double floor = 0.0;
    GF_TRY(do_fp32_floor(L, &floor));
    *out = std::max(theta_target, kFloorMargin * floor);
    return GF_OK;
}

gf_status upload_canonical(gf_lattice L, const double* dev_canon)
{
    if (L->group == 2) {
        if (L->f32) GF_HIP(gf::launch_su2_pack(dev_canon, su2_32(L), L->geom, L->stream));
        if (L->f64) GF_HIP(gf::launch_su2_pack(dev_canon, su2_64(L), L->geom, L->stream));
        L->phase = 0;
        L->has_links = true;
        L->anneal_sweeps = 0;
        return GF_OK;
    }
    if (L->f32 && L->min8)
        GF_HIP(gf::launch_pack(dev_canon, field8f(L), L->geom, L->stream));
    else if (L->f32)
        GF_HIP(gf::launch_pack(dev_canon, field32(L), L->geom, L->stream));
    if (L->f64 && min8_64(L))
        GF_HIP(gf::launch_pack(dev_canon, field8(L), L->geom, L->stream));
    else if (L->f64)
        GF_HIP(gf::launch_pack(dev_canon, field64(L), L->geom, L->stream));
    if (L->gacc.base) GF_HIP(gf::launch_g_identity(L->gacc, L->geom, L->stream));
    L->phase = 0;
    L->has_links = true;
    L->anneal_sweeps = 0;
    return GF_OK;
}

gf_status download_canonical(gf_lattice L, double* dev_canon)
{
    if (L->group == 2) {
        if (is_fp32(L))
            GF_HIP(gf::launch_su2_unpack(su2_32(L), L->geom, dev_canon, L->stream));
        else
            GF_HIP(gf::launch_su2_unpack(su2_64(L), L->geom, dev_canon, L->stream));
        return GF_OK;
    }
    if (min8_64(L))
        GF_HIP(gf::launch_unpack(field8(L), L->geom, dev_canon, L->stream));
    else if (is_fp32(L) && L->min8)
        GF_HIP(gf::launch_unpack(field8f(L), L->geom, dev_canon, L->stream));
    else if (is_fp32(L))
        GF_HIP(gf::launch_unpack(field32(L), L->geom, dev_canon, L->stream));
    else
        GF_HIP(gf::launch_unpack(field64(L), L->geom, dev_canon, L->stream));
    return GF_OK;
}

// Convert the links of an SU(3) lattice's sweeping precision (the float64
// field of GF_FP64, the float32 field of GF_FP32 and GF_MIXED) to the other
// storage (min8 = true: 8 reals per link).  Allocates the new field, converts
// the links if there are any, frees the old field.  Syncs.
gf_status do_set_storage(gf_lattice L, bool min8)
{
    if (L->group != 3) return fail(GF_E_STATE, "the storage of links can change on SU(3) lattices only");
    if (L->min8 == min8) return GF_OK;
    const LatticeSizes from = lattice_sizes(L->geom, L->prec, L->group, L->min8);
    const LatticeSizes to = lattice_sizes(L->geom, L->prec, L->group, min8);
    const bool f64 = L->prec == GF_FP64;
    void* f = nullptr;
    GF_HIP(hipMalloc(&f, f64 ? to.f64 : to.f32));
    hipError_t e = hipSuccess;
    if (L->has_links && f64) {
        if (min8)
            e = gf::launch_convert(field64(L), Link8Field{(double2*)f, L->geom.ld}, L->geom, L->stream);
        else
            e = gf::launch_convert(field8(L), LinkField<double>{(double2*)f, L->geom.ld}, L->geom, L->stream);
    } else if (L->has_links) {
        if (min8)
            e = gf::launch_convert(field32(L), Link8Field32{(float4*)f, L->geom.ld}, L->geom, L->stream);
        else
            e = gf::launch_convert(field8f(L), LinkField<float>{(float4*)f, L->geom.ld}, L->geom, L->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) {
        (void)hipFree(f);
        return fail(GF_E_HIP, "storage conversion: %s", hipGetErrorString(e));
    }
    if (f64) {
        (void)hipFree(L->f64);
        L->f64 = (double2*)f;
        L->bytes += (int64_t)to.f64 - (int64_t)from.f64;
        L->cfg64.minw = 0;
        L->cfg_hb64.minw = 0;
    } else {
        (void)hipFree(L->f32);
        L->f32 = (float4*)f;
        L->bytes += (int64_t)to.f32 - (int64_t)from.f32;
    }
    L->min8 = min8;
    clear_graphs(L);  // captured launches hold the old field's address
    return GF_OK;
}

void release(gf_lattice L)
{
    clear_graphs(L);
    if (L->f64) (void)hipFree(L->f64);
    if (L->f32) (void)hipFree(L->f32);
    if (L->gacc.base) (void)hipFree(L->gacc.base);
    if (L->partial) (void)hipFree(L->partial);
    if (L->dres) (void)hipFree(L->dres);
    if (L->hres) (void)hipHostFree(L->hres);
    if (L->est) (void)hipFree(L->est);
    L->est = nullptr;
    L->est_cap = 0;
    if (L->dslices) (void)hipFree(L->dslices);
    if (L->hslices) (void)hipHostFree(L->hslices);
    L->dslices = nullptr;
    L->hslices = nullptr;
    L->f64 = nullptr;
    L->f32 = nullptr;
    L->gacc.base = nullptr;
    L->partial = nullptr;
    L->dres = nullptr;
    L->hres = nullptr;
}

}  // namespace detail
}  // namespace gf

using namespace gf::detail;

extern "C" {

const char* gf_last_error(void)
{
    return g_last_error.c_str();
}

const char* gf_version(void)
{
    return "libgf 0.1 (gfx950)";
}

}  // extern "C"

namespace gf {
namespace detail {

gf_status create_lattice(const int32_t dims[4], gf_prec prec, int group, bool min8, void* hip_stream,
                         gf_lattice* out)
{
    if (!dims || !out) return fail(GF_E_ARG, "null argument");
    *out = nullptr;
    int64_t V = 1;
    GF_TRY(check_dims(dims, &V));
    if (prec != GF_FP64 && prec != GF_FP32 && prec != GF_MIXED)
        return fail(GF_E_ARG, "unsupported precision %d", (int)prec);
    if (group == 2 && prec == GF_MIXED)
        return fail(GF_E_ARG, "SU(2) lattices are GF_FP64 or GF_FP32 (no mixed precision)");

    gf_lattice_* L = new (std::nothrow) gf_lattice_();
    if (!L) return fail(GF_E_NOMEM, "host allocation failed");
    for (int m = 0; m < 4; ++m) L->dims[m] = dims[m];
    L->prec = prec;
    L->group = group;
    L->min8 = min8;
    L->stream = (hipStream_t)hip_stream;
    L->volume = V;

    Geom& g = L->geom;
    if (!make_geom(dims, &g)) {
        delete L;
        return fail(GF_E_ARG, "internal: index division check failed");
    }

    const LatticeSizes z = lattice_sizes(g, prec, group, min8);
    hipError_t e = hipSuccess;
    if (z.f64) e = hipMalloc((void**)&L->f64, z.f64);
    if (e == hipSuccess && z.f32) e = hipMalloc((void**)&L->f32, z.f32);
    if (e == hipSuccess && z.gacc) {
        e = hipMalloc((void**)&L->gacc.base, z.gacc);
        L->gacc.ld = g.ld;
    }
    if (e == hipSuccess) e = hipMalloc((void**)&L->partial, z.partial * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&L->dres, 4 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&L->hres, 4 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&L->dslices, z.nslices * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&L->hslices, z.nslices * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        release(L);
        delete L;
        return fail(e == hipErrorOutOfMemory ? GF_E_NOMEM : GF_E_HIP, "allocation failed: %s", hipGetErrorString(e));
    }
    L->bytes = z.total;
    L->cfg64 = SweepConfig{4, 256};
    L->cfg32 = SweepConfig{4, 256};
    // The heat bath samples each subgroup element in every lane of a site's
    // group, so its arithmetic grows with the lanes per site: one lane is the
    // fastest shape on MI355X (32^4: float32 with g 175 us per sweep at 1 lane
    // vs 282 us at 4; float64 414 us vs 544 us at 2).
    L->cfg_hb64 = SweepConfig{1, 128, 2};
    L->cfg_hb32 = SweepConfig{1, 256, 0};
    if (group == 2) {
        // one lane per site: the SU(2) site update is a few quaternion products
        L->cfg64 = SweepConfig{1, 256, 0};
        L->cfg32 = SweepConfig{1, 256, 0};
        L->cfg_hb64 = SweepConfig{1, 256, 0};
    }
    *out = L;
    return GF_OK;
}

}  // namespace detail
}  // namespace gf

extern "C" {

gf_status gf_create_lattice(const int32_t dims[4], gf_prec prec, void* hip_stream, gf_lattice* out)
{
    return create_lattice(dims, prec, 3, false, hip_stream, out);
}

gf_status gf_create_lattice_su2(const int32_t dims[4], gf_prec prec, void* hip_stream, gf_lattice* out)
{
    return create_lattice(dims, prec, 2, false, hip_stream, out);
}

gf_status gf_create_lattice_min8(const int32_t dims[4], void* hip_stream, gf_lattice* out)
{
    return create_lattice(dims, GF_FP64, 3, true, hip_stream, out);
}

gf_status gf_lattice_storage(gf_lattice L, int32_t* reals_per_link)
{
    if (!L || !reals_per_link) return fail(GF_E_ARG, "null argument");
    *reals_per_link = L->group == 2 ? 4 : (L->min8 ? 8 : 12);
    return GF_OK;
}

gf_status gf_set_storage(gf_lattice L, int32_t reals_per_link)
{
    if (!L) return fail(GF_E_ARG, "null lattice");
    if (reals_per_link != 8 && reals_per_link != 12)
        return fail(GF_E_ARG, "reals per link must be 8 or 12 (got %d)", reals_per_link);
    return do_set_storage(L, reals_per_link == 8);
}

gf_status gf_lattice_group(gf_lattice L, int32_t* nc)
{
    if (!L || !nc) return fail(GF_E_ARG, "null argument");
    *nc = L->group;
    return GF_OK;
}

gf_status gf_destroy_lattice(gf_lattice L)
{
    if (!L) return GF_OK;
    hipError_t e = hipStreamSynchronize(L->stream);
    release(L);
    delete L;
    if (e != hipSuccess) return fail(GF_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return GF_OK;
}

gf_status gf_lattice_info(gf_lattice L, int64_t* volume, int64_t* device_bytes)
{
    if (!L) return fail(GF_E_ARG, "null lattice");
    if (volume) *volume = L->volume;
    if (device_bytes) *device_bytes = L->bytes;
    return GF_OK;
}

namespace {

gf_status set_config(gf_lattice L, gf_prec kernel, int32_t tps, int32_t block, int32_t nontemporal, int32_t min_waves,
                     bool heat_bath)
{
    if (!L) return fail(GF_E_ARG, "null lattice");
    if (kernel != GF_FP64 && kernel != GF_FP32) return fail(GF_E_ARG, "kernel precision must be GF_FP64 or GF_FP32");
    SweepConfig c{tps, block, nontemporal, min_waves};
    if (L->group == 2) {
        if (!gf::su2_config_valid(c))
            return fail(GF_E_ARG,
                        "SU(2) sweep config tps=%d block=%d policy=%d: one lane per site, block 64, 128, 256 or 512, "
                        "cache policy 0, 1 or 2",
                        tps, block, nontemporal);
    } else if (!gf::sweep_config_valid(c))
        return fail(GF_E_ARG,
                    "sweep config tps=%d block=%d policy=%d min_waves=%d: tps must be 1, 2, 4 or 8, block 64, 128, "
                    "256 or 512 (not 512 with tps 1), cache policy 0, 1 or 2 (1 and 2 only with tps <= 4 and block "
                    "<= 256), min_waves 0 or 2 (2 only with tps 1)",
                    tps, block, nontemporal, min_waves);
    if ((kernel == GF_FP64 ? min8_64(L) : L->min8) && min_waves != 0)
        return fail(GF_E_ARG, "8-real links: min_waves must be 0 (the register cap is an axis of the 12-real kernel)");
    if (heat_bath)
        (kernel == GF_FP32 ? L->cfg_hb32 : L->cfg_hb64) = c;
    else
        (kernel == GF_FP32 ? L->cfg32 : L->cfg64) = c;
    return GF_OK;
}

}  // namespace

gf_status gf_set_sweep_config(gf_lattice L, gf_prec kernel, int32_t tps, int32_t block, int32_t nontemporal,
                              int32_t min_waves)
{
    return set_config(L, kernel, tps, block, nontemporal, min_waves, false);
}

gf_status gf_set_anneal_config(gf_lattice L, gf_prec kernel, int32_t tps, int32_t block, int32_t nontemporal,
                               int32_t min_waves)
{
    return set_config(L, kernel, tps, block, nontemporal, min_waves, true);
}

gf_status gf_promote_fp64(gf_lattice L)
{
    GF_TRY(check_ready(L));
    return do_promote(L);
}

gf_status gf_set_links_device(gf_lattice L, const double* dev)
{
    if (!L || !dev) return fail(GF_E_ARG, "null argument");
    return upload_canonical(L, dev);
}

gf_status gf_set_links(gf_lattice L, const double* host)
{
    if (!L || !host) return fail(GF_E_ARG, "null argument");
    const size_t bytes = (size_t)L->volume * 4 * canon_per_link(L) * sizeof(double);
    double* stage = nullptr;
    GF_HIP(hipMalloc((void**)&stage, bytes));
    hipError_t e = hipMemcpyAsync(stage, host, bytes, hipMemcpyHostToDevice, L->stream);
    gf_status st = GF_OK;
    if (e == hipSuccess) st = upload_canonical(L, stage);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    (void)hipFree(stage);
    if (e != hipSuccess) return fail(GF_E_HIP, "set_links: %s", hipGetErrorString(e));
    return st;
}

gf_status gf_get_links_device(gf_lattice L, double* dev)
{
    GF_TRY(check_ready(L));
    if (!dev) return fail(GF_E_ARG, "null argument");
    return download_canonical(L, dev);
}

gf_status gf_get_links(gf_lattice L, double* host)
{
    GF_TRY(check_ready(L));
    if (!host) return fail(GF_E_ARG, "null argument");
    const size_t bytes = (size_t)L->volume * 4 * canon_per_link(L) * sizeof(double);
    double* stage = nullptr;
    GF_HIP(hipMalloc((void**)&stage, bytes));
    gf_status st = download_canonical(L, stage);
    hipError_t e = hipSuccess;
    if (st == GF_OK) e = hipMemcpyAsync(host, stage, bytes, hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    (void)hipFree(stage);
    if (e != hipSuccess) return fail(GF_E_HIP, "get_links: %s", hipGetErrorString(e));
    return st;
}

gf_status gf_sweep_or(gf_lattice L, int32_t n_sweeps, double omega, gf_or_mode mode)
{
    GF_TRY(check_ready(L));
    GF_TRY(check_omega(omega, (int)mode));
    if (n_sweeps < 0) return fail(GF_E_ARG, "n_sweeps = %d < 0", n_sweeps);
    return do_sweeps(L, n_sweeps, omega, (int)mode);
}

gf_status gf_half_sweep_or(gf_lattice L, int32_t colour, double omega, gf_or_mode mode)
{
    GF_TRY(check_ready(L));
    GF_TRY(check_omega(omega, (int)mode));
    if (colour != 0 && colour != 1) return fail(GF_E_ARG, "colour must be 0 (black) or 1 (white)");
    return do_half_sweep(L, colour, omega, (int)mode);
}

gf_status gf_get_anneal_counter(gf_lattice L, uint32_t* sweeps_done)
{
    if (!L || !sweeps_done) return fail(GF_E_ARG, "null argument");
    if (L->prec == GF_MIXED) return fail(GF_E_STATE, "a GF_MIXED lattice cannot be checkpointed by its links");
    *sweeps_done = L->anneal_sweeps;
    return GF_OK;
}

gf_status gf_set_anneal_counter(gf_lattice L, uint32_t sweeps_done)
{
    GF_TRY(check_ready(L));
    if (L->prec == GF_MIXED) return fail(GF_E_STATE, "a GF_MIXED lattice cannot be checkpointed by its links");
    L->anneal_sweeps = sweeps_done;
    return GF_OK;
}

gf_status gf_anneal(gf_lattice L, int32_t n_sweeps, double T_start, double T_end, uint64_t seed)
{
    TraceRange range("gf_anneal");
    GF_TRY(check_ready(L));
    if (n_sweeps < 0) return fail(GF_E_ARG, "n_sweeps = %d < 0", n_sweeps);
    if (!(T_end > 0.0) || !(T_start >= T_end) || !std::isfinite(T_start))
        return fail(GF_E_ARG, "need T_start >= T_end > 0 (got %g, %g)", T_start, T_end);
    for (int32_t s = 0; s < n_sweeps; ++s) {
        const double T = anneal_temperature(s, n_sweeps, T_start, T_end);
        const uint32_t sweep = L->anneal_sweeps + (uint32_t)s;
        for (int parity = 0; parity < 2; ++parity) {
            if (L->group == 2 && is_fp32(L))
                GF_HIP(gf::launch_su2_hb(su2_32(L), L->geom, parity, (float)T, seed, sweep, L->cfg_hb32, L->stream,
                                         L->gauge));
            else if (L->group == 2)
                GF_HIP(gf::launch_su2_hb(su2_64(L), L->geom, parity, T, seed, sweep, L->cfg_hb64, L->stream,
                                         L->gauge));
            else if (min8_64(L))
                GF_HIP(gf::launch_hb_half_sweep(field8(L), L->geom, parity, T, seed, sweep, L->cfg_hb64, L->stream,
                                                L->gauge));
            else if (is_fp32(L) && L->min8)
                GF_HIP(gf::launch_hb_half_sweep(field8f(L), L->geom, parity, (float)T, seed, sweep, L->cfg_hb32,
                                                g_tracking(L), L->stream, L->gauge));
            else if (is_fp32(L))
                GF_HIP(gf::launch_hb_half_sweep(field32(L), L->geom, parity, (float)T, seed, sweep, L->cfg_hb32,
                                                g_tracking(L), L->stream, L->gauge));
            else
                GF_HIP(gf::launch_hb_half_sweep(field64(L), L->geom, parity, T, seed, sweep, L->cfg_hb64,
                                                L->stream, L->gauge));
        }
    }
    L->anneal_sweeps += (uint32_t)n_sweeps;
    return GF_OK;
}

gf_status gf_measure_theta_F(gf_lattice L, double* theta, double* F)
{
    GF_TRY(check_ready(L));
    if (!theta || !F) return fail(GF_E_ARG, "null argument");
    return do_measure(L, theta, F);
}

gf_status gf_set_gauge(gf_lattice L, gf_gauge gauge)
{
    if (!L) return fail(GF_E_ARG, "null lattice");
    if (gauge != GF_LANDAU && gauge != GF_COULOMB) return fail(GF_E_ARG, "unknown gauge %d", (int)gauge);
    if (gauge == GF_COULOMB && L->dims[3] > 65535)
        return fail(GF_E_ARG, "Coulomb gauge supports at most 65535 timeslices (Nt = %d)", L->dims[3]);
    L->gauge = gauge == GF_COULOMB ? gf::GAUGE_COULOMB : gf::GAUGE_LANDAU;
    return GF_OK;
}

gf_status gf_get_gauge(gf_lattice L, gf_gauge* gauge)
{
    if (!L || !gauge) return fail(GF_E_ARG, "null argument");
    *gauge = L->gauge == gf::GAUGE_COULOMB ? GF_COULOMB : GF_LANDAU;
    return GF_OK;
}

gf_status gf_measure_timeslices(gf_lattice L, double* theta_t, double* F_t)
{
    GF_TRY(check_ready(L));
    if (!theta_t || !F_t) return fail(GF_E_ARG, "null argument");
    if (L->gauge != gf::GAUGE_COULOMB) return fail(GF_E_STATE, "per-timeslice values need a Coulomb-gauge lattice");
    double th = 0.0, f = 0.0;
    GF_TRY(measure_enqueue(L, L->stream));
    GF_HIP(hipStreamSynchronize(L->stream));
    GF_TRY(measure_read(L, &th, &f));
    for (int t = 0; t < L->dims[3]; ++t) {
        theta_t[t] = L->hslices[2 * t];
        F_t[t] = L->hslices[2 * t + 1];
    }
    return GF_OK;
}

gf_status gf_set_check_policy(gf_lattice L, int32_t adaptive, double margin)
{
    if (!L) return fail(GF_E_ARG, "null lattice");
    if (adaptive && !(margin >= 1.0 && std::isfinite(margin)))
        return fail(GF_E_ARG, "margin = %g must be finite and >= 1", margin);
    L->adaptive = adaptive != 0;
    if (adaptive) L->margin = margin;
    return GF_OK;
}

gf_status gf_sweep_estimate(gf_lattice L, double omega, gf_or_mode mode, double* theta_est)
{
    GF_TRY(check_ready(L));
    GF_TRY(check_omega(omega, (int)mode));
    if (!theta_est) return fail(GF_E_ARG, "null argument");
    GF_TRY(do_est_sweep(L, omega, (int)mode, theta_est));
    if (std::isnan(*theta_est)) return fail(GF_E_NUMERIC, "theta estimate is NaN");
    return GF_OK;
}

gf_status gf_lattice_counters(gf_lattice L, int64_t* measures, int64_t* estimates)
{
    if (!L) return fail(GF_E_ARG, "null lattice");
    if (measures) *measures = L->n_measures;
    if (estimates) *estimates = L->n_estimates;
    return GF_OK;
}

gf_status gf_reunitarize(gf_lattice L)
{
    GF_TRY(check_ready(L));
    return do_reunitarize(L);
}

gf_status gf_plaquette(gf_lattice L, double* P)
{
    GF_TRY(check_ready(L));
    if (!P) return fail(GF_E_ARG, "null argument");
    if (L->group == 2 && is_fp32(L))
        GF_HIP(gf::launch_su2_plaquette(su2_32(L), L->geom, L->partial, L->dres, L->stream));
    else if (L->group == 2)
        GF_HIP(gf::launch_su2_plaquette(su2_64(L), L->geom, L->partial, L->dres, L->stream));
    else if (min8_64(L))
        GF_HIP(gf::launch_plaquette(field8(L), L->geom, L->partial, L->dres, L->stream));
    else if (is_fp32(L) && L->min8)
        GF_HIP(gf::launch_plaquette(field8f(L), L->geom, L->partial, L->dres, L->stream));
    else if (is_fp32(L))
        GF_HIP(gf::launch_plaquette(field32(L), L->geom, L->partial, L->dres, L->stream));
    else
        GF_HIP(gf::launch_plaquette(field64(L), L->geom, L->partial, L->dres, L->stream));
    GF_HIP(hipMemcpyAsync(L->hres, L->dres, sizeof(double), hipMemcpyDeviceToHost, L->stream));
    GF_HIP(hipStreamSynchronize(L->stream));
    *P = L->hres[0];
    if (!std::isfinite(*P)) return fail(GF_E_NUMERIC, "plaquette is not finite");
    return GF_OK;
}

gf_status gf_tune_switch(gf_lattice L, double theta_target, double* floor, double* theta_switch)
{
    GF_TRY(check_ready(L));
    if (!floor || !theta_switch) return fail(GF_E_ARG, "null argument");
    if (!(theta_target >= 0.0)) return fail(GF_E_ARG, "theta_target must be >= 0");
    GF_TRY(do_fp32_floor(L, floor));
    *theta_switch = std::max(theta_target, kFloorMargin * *floor);
    return GF_OK;
}

gf_status gf_fix_until(gf_lattice L, const gf_fix_params* p, gf_fix_result* res)
{
    TraceRange range("gf_fix_until");
    GF_TRY(check_ready(L));
    if (!p || !res) return fail(GF_E_ARG, "null argument");
    GF_TRY(check_omega(p->omega, p->mode));
    if (p->max_sweeps < 0 || p->check_every < 1 || p->reunit_every < 0)
        return fail(GF_E_ARG, "need max_sweeps >= 0, check_every >= 1, reunit_every >= 0");
    if (!(p->theta_target >= 0.0)) return fail(GF_E_ARG, "theta_target must be >= 0");
    if (std::isnan(p->theta_switch)) return fail(GF_E_ARG, "theta_switch is NaN");
    std::memset(res, 0, sizeof *res);
    double theta_switch = 0.0;
    GF_TRY(resolve_switch(L, p->theta_target, p->theta_switch, &theta_switch));
    double theta = 0.0, F = 0.0;
    GF_TRY(do_measure(L, &theta, &F));
    int32_t sweeps = 0;
    double best = theta;
    int stall = 0;
    for (;;) {
        const bool finished = !(theta >= p->theta_target && sweeps < p->max_sweeps);
        // GF_MIXED ends in float64: the float32 phase is left at the switch
        // point, at a stall below kStallTheta, and when the loop would end.
        if (L->prec == GF_MIXED && L->phase == 0 && (finished || leave_fp32(theta, theta_switch, best, stall))) {
            TraceRange promote("promote_fp64");
            GF_TRY(do_promote(L));
            GF_TRY(do_measure(L, &theta, &F));
            continue;
        }
        if (finished) break;
        TraceRange check(is_fp32(L) ? "fix_check_fp32" : "fix_check_fp64");
        const bool fp32 = is_fp32(L);
        const bool mixed32 = L->prec == GF_MIXED && L->phase == 0;
        const int32_t n = std::min(p->check_every, p->max_sweeps - sweeps);
        // n sweeps, reunitarising after every sweep whose count is a multiple of
        // reunit_every; adaptive checks take the last one with the fused estimate
        double est = 0.0;
        int32_t done = 0;
        while (done < n) {
            int32_t run = n - done;
            if (p->reunit_every > 0) {
                const int32_t to_reunit = p->reunit_every - (sweeps % p->reunit_every);
                run = std::min(run, to_reunit);
            }
            if (L->adaptive && done + run == n) {
                GF_TRY(do_sweeps(L, run - 1, p->omega, p->mode));
                GF_TRY(do_est_sweep(L, p->omega, p->mode, &est));
            } else {
                GF_TRY(do_sweeps(L, run, p->omega, p->mode));
            }
            sweeps += run;
            done += run;
            if (p->reunit_every > 0 && sweeps % p->reunit_every == 0) GF_TRY(do_reunitarize(L));
        }
        if (fp32)
            res->sweeps_fp32 += n;
        else
            res->sweeps_fp64 += n;
        // Adaptive checks measure exactly only where a decision can be taken: at the
        // last sweep, once the estimate is below margin x the smallest threshold that
        // could decide (the target; in the float32 phase of GF_MIXED also the switch
        // point and the stall level), and at every check of the float32 phase once
        // theta has been below the stall level (the stall rule counts every check
        // from the first check below it on).  Elsewhere theta is above every
        // threshold, so skipping the measurement changes no decision: the sweep
        // count, links, theta and F are those of checking every time.
        bool exact = true;
        if (L->adaptive) {
            double thr = p->theta_target;
            if (mixed32) thr = std::max(thr, std::max(theta_switch, kStallTheta));
            exact = sweeps >= p->max_sweeps || !(est >= L->margin * thr) || (mixed32 && best < kStallTheta);
        }
        if (exact) {
            GF_TRY(do_measure(L, &theta, &F));
            update_stall(theta, &best, &stall);
        } else {
            theta = est;  // >= margin x every threshold: no decision at this check
        }
    }
    res->converged = theta < p->theta_target;
    res->sweeps = sweeps;
    res->theta = theta;
    res->F = F;
    return GF_OK;
}

}  // extern "C"
