// gf_sweep_impl.h -- the single-lattice checkerboard half-sweep kernel
// (overrelaxation and heat bath, Sec. 2 and the abstract of arXiv:1412.3655)
// and its launch dispatch, instantiated per gauge and per estimate flag in
// translation units of their own (compiled in parallel): gf_sweep.hip
// (Landau gauge, K over 4 directions), gf_sweep_coulomb.hip (Coulomb gauge, K
// over x, y, z), gf_sweep_est.hip and gf_sweep_coulomb_est.hip (the sweeps
// that also sum the estimate of theta).  The per-site body lives in gf_site.h.  The loop over
// sites is over the half index of one colour: every link is read once and
// written once per half-sweep (per site update in FP64 with 12-real links:
// 768 B read and 768 B written; with 8-real links 512 B and 512 B), whatever
// the gauge.  The 8-real instantiations are compiled in gf_sweep_min8*.hip
// (float64) and gf_sweep_min8f*.hip (float32: 256 B read and 256 B written).
#pragma once

#include "gf_kernels.h"
#include "gf_site.h"

namespace gf {
namespace sweep_impl {

// EST: the block also sums tr[Delta Delta^dag] of its sites' K before their
// update into est[2 (parity gridDim.x + b)] (b the block's tile, second double
// 0), which a fixed-order pass turns into an estimate of theta.  A template
// parameter, so the plain sweep carries none of it.
template <typename R, int TPS, int MODE, int BLOCK, bool TRACKG, int CP, int NDIR, bool EST, typename F>
__device__ __forceinline__ void half_sweep_body(const F& f, const Geom& g, int parity, const Rule<R>& rule,
                                                const GField& gacc, double* est)
{
    // With cached loads the white half-sweep takes the blocks in reverse
    // order, so it starts on the links the black half-sweep touched last,
    // which are still in the Infinity Cache (a 32^4 float64 field is 402 MB
    // against 256 MB of cache), and ends where the next black half-sweep
    // starts; non-temporal loads leave nothing there to reuse.  Sites of one
    // colour are independent, so the result does not depend on the order.
    const uint32_t b = (parity && !nt_loads(CP)) ? gridDim.x - 1u - blockIdx.x : blockIdx.x;
    const uint32_t gid = b * (uint32_t)BLOCK + threadIdx.x;
    const uint32_t h = gid / TPS;
    const int r = (int)(gid % TPS);
    // whole groups of TPS lanes leave or skip together, so every DPP partner is live
    if constexpr (!EST) {
        if (h >= g.vh) return;
        site_update<R, TPS, MODE, TRACKG, CP, NDIR, F>(f, g, parity, h, r, rule, gacc);
    } else {
        double th = 0.0;
        if (h < g.vh) th = site_update<R, TPS, MODE, TRACKG, CP, NDIR, F>(f, g, parity, h, r, rule, gacc, true);
        block_sum2<BLOCK>(th, 0.0, est + 2 * ((size_t)parity * gridDim.x + b));
    }
}

template <typename R, int TPS, int MODE, int BLOCK, bool TRACKG, int CP, int NDIR, bool EST, typename F>
__global__ void __launch_bounds__(BLOCK) k_or_half_sweep(F f, Geom g, int parity, Rule<R> rule, GField gacc,
                                                         double* est)
{
    half_sweep_body<R, TPS, MODE, BLOCK, TRACKG, CP, NDIR, EST, F>(f, g, parity, rule, gacc, est);
}

// The same kernel held to at least 2 waves per SIMD (at most 256 registers per
// lane): the register-limit axis of run-time tuning, for the one-lane float64
// shape.
template <typename R, int TPS, int MODE, int BLOCK, bool TRACKG, int CP, int NDIR, bool EST, typename F>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_or_half_sweep_w2(F f, Geom g, int parity, Rule<R> rule, GField gacc, double* est)
{
    half_sweep_body<R, TPS, MODE, BLOCK, TRACKG, CP, NDIR, EST, F>(f, g, parity, rule, gacc, est);
}

// Blocks of one half-sweep launch in configuration c (the estimate buffer
// holds 2 pairs per block of each colour).
inline uint32_t sweep_grid(const Geom& g, const SweepConfig& c)
{
    return (uint32_t)(((uint64_t)g.vh * (uint64_t)c.tps + (uint64_t)c.block - 1) / (uint64_t)c.block);
}

template <int NDIR, bool EST, typename R, int TPS, int MODE, bool TRACKG, typename F>
hipError_t launch_tps(const F& f, const Geom& g, int parity, const Rule<R>& rule, const SweepConfig& c,
                      const GField& gacc, hipStream_t st, double* est)
{
    const int block = c.block;
    const uint32_t grid = sweep_grid(g, c);
    if (grid == 0) return hipSuccess;
    // minw = 2 selects the register-capped kernel for the one-lane float64 shape
    // of the 12-real layout (other shapes already run 2 or more waves per SIMD)
    constexpr bool kCap = sizeof(R) == 8 && TPS == 1 && std::is_same<F, LinkField<R>>::value;
    const bool cap = kCap && c.minw == 2;
#define GF_LAUNCH(B, CPV)                                                                                         \
    do {                                                                                                          \
        if constexpr (kCap) {                                                                                     \
            if (cap) {                                                                                            \
                hipLaunchKernelGGL((k_or_half_sweep_w2<R, TPS, MODE, B, TRACKG, CPV, NDIR, EST, F>), dim3(grid),  \
                                   dim3(B), 0, st, f, g, parity, rule, gacc, est);                                \
                break;                                                                                            \
            }                                                                                                     \
        }                                                                                                         \
        hipLaunchKernelGGL((k_or_half_sweep<R, TPS, MODE, B, TRACKG, CPV, NDIR, EST, F>), dim3(grid), dim3(B), 0,  \
                           st, f, g, parity, rule, gacc, est);                                                    \
    } while (0)
#define GF_LAUNCH_SMALL_BLOCKS(CPV)                  \
    switch (block) {                                 \
        case 64: GF_LAUNCH(64, CPV); break;          \
        case 128: GF_LAUNCH(128, CPV); break;        \
        case 256: GF_LAUNCH(256, CPV); break;        \
        default: return hipErrorInvalidValue;        \
    }
    if (c.nt == 1 || c.nt == 2) {
        if constexpr (TPS <= 4) {
            if (c.nt == 1) {
                GF_LAUNCH_SMALL_BLOCKS(1)
            } else {
                GF_LAUNCH_SMALL_BLOCKS(2)
            }
        } else {
            return hipErrorInvalidValue;
        }
    } else if (c.nt == 0) {
        switch (block) {
            case 64: GF_LAUNCH(64, 0); break;
            case 128: GF_LAUNCH(128, 0); break;
            case 256: GF_LAUNCH(256, 0); break;
            default:
                if constexpr (TPS > 1)
                    GF_LAUNCH(512, 0);
                else
                    return hipErrorInvalidValue;
                break;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef GF_LAUNCH_SMALL_BLOCKS
#undef GF_LAUNCH
    return hipGetLastError();
}

template <int NDIR, bool EST, typename R, int MODE, bool TRACKG, typename F>
hipError_t launch_mode(const F& f, const Geom& g, int parity, const Rule<R>& rule, const SweepConfig& c,
                       const GField& gacc, hipStream_t st, double* est)
{
    switch (c.tps) {
        case 1: return launch_tps<NDIR, EST, R, 1, MODE, TRACKG>(f, g, parity, rule, c, gacc, st, est);
        case 2: return launch_tps<NDIR, EST, R, 2, MODE, TRACKG>(f, g, parity, rule, c, gacc, st, est);
        case 8: return launch_tps<NDIR, EST, R, 8, MODE, TRACKG>(f, g, parity, rule, c, gacc, st, est);
        default: return launch_tps<NDIR, EST, R, 4, MODE, TRACKG>(f, g, parity, rule, c, gacc, st, est);
    }
}

// EST = true needs est != nullptr; EST = false ignores est.
template <int NDIR, bool EST>
hipError_t or_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double omega, int mode,
                         const SweepConfig& cfg, hipStream_t st, double* est)
{
    const GField none{nullptr, 0};
    const Rule<double> rule{omega, 1.0, 0u, 0u, 0u};
    return mode == OR_EXACT ? launch_mode<NDIR, EST, double, 0, false>(f, g, parity, rule, cfg, none, st, est)
                            : launch_mode<NDIR, EST, double, 1, false>(f, g, parity, rule, cfg, none, st, est);
}

template <int NDIR, bool EST>
hipError_t or_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float omega, int mode,
                         const SweepConfig& cfg, const GField& gacc, hipStream_t st, double* est)
{
    const Rule<float> rule{omega, 1.0f, 0u, 0u, 0u};
    if (gacc.base)
        return mode == OR_EXACT ? launch_mode<NDIR, EST, float, 0, true>(f, g, parity, rule, cfg, gacc, st, est)
                                : launch_mode<NDIR, EST, float, 1, true>(f, g, parity, rule, cfg, gacc, st, est);
    return mode == OR_EXACT ? launch_mode<NDIR, EST, float, 0, false>(f, g, parity, rule, cfg, gacc, st, est)
                            : launch_mode<NDIR, EST, float, 1, false>(f, g, parity, rule, cfg, gacc, st, est);
}

template <int NDIR>
hipError_t hb_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double T, uint64_t seed,
                         uint32_t sweep, const SweepConfig& cfg, hipStream_t st)
{
    const GField none{nullptr, 0};
    const Rule<double> rule{1.0, T, (uint32_t)seed, (uint32_t)(seed >> 32), sweep};
    return launch_mode<NDIR, false, double, HEATBATH, false>(f, g, parity, rule, cfg, none, st, nullptr);
}

template <int NDIR>
hipError_t hb_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float T, uint64_t seed,
                         uint32_t sweep, const SweepConfig& cfg, const GField& gacc, hipStream_t st)
{
    const Rule<float> rule{1.0f, T, (uint32_t)seed, (uint32_t)(seed >> 32), sweep};
    if (gacc.base) return launch_mode<NDIR, false, float, HEATBATH, true>(f, g, parity, rule, cfg, gacc, st, nullptr);
    return launch_mode<NDIR, false, float, HEATBATH, false>(f, g, parity, rule, cfg, gacc, st, nullptr);
}

// Float64 links stored in 8 reals (Link8Field): the same kernel, decoding on
// load and encoding on store.
template <int NDIR, bool EST>
hipError_t or_half_sweep(const Link8Field& f, const Geom& g, int parity, double omega, int mode,
                         const SweepConfig& cfg, hipStream_t st, double* est)
{
    const GField none{nullptr, 0};
    const Rule<double> rule{omega, 1.0, 0u, 0u, 0u};
    return mode == OR_EXACT ? launch_mode<NDIR, EST, double, 0, false>(f, g, parity, rule, cfg, none, st, est)
                            : launch_mode<NDIR, EST, double, 1, false>(f, g, parity, rule, cfg, none, st, est);
}

template <int NDIR>
hipError_t hb_half_sweep(const Link8Field& f, const Geom& g, int parity, double T, uint64_t seed, uint32_t sweep,
                         const SweepConfig& cfg, hipStream_t st)
{
    const GField none{nullptr, 0};
    const Rule<double> rule{1.0, T, (uint32_t)seed, (uint32_t)(seed >> 32), sweep};
    return launch_mode<NDIR, false, double, HEATBATH, false>(f, g, parity, rule, cfg, none, st, nullptr);
}

// Float32 links stored in 8 reals (Link8Field32): the float32 sweeps, g(x)
// tracked when gacc.base is set.
template <int NDIR, bool EST>
hipError_t or_half_sweep(const Link8Field32& f, const Geom& g, int parity, float omega, int mode,
                         const SweepConfig& cfg, const GField& gacc, hipStream_t st, double* est)
{
    const Rule<float> rule{omega, 1.0f, 0u, 0u, 0u};
    if (gacc.base)
        return mode == OR_EXACT ? launch_mode<NDIR, EST, float, 0, true>(f, g, parity, rule, cfg, gacc, st, est)
                                : launch_mode<NDIR, EST, float, 1, true>(f, g, parity, rule, cfg, gacc, st, est);
    return mode == OR_EXACT ? launch_mode<NDIR, EST, float, 0, false>(f, g, parity, rule, cfg, gacc, st, est)
                            : launch_mode<NDIR, EST, float, 1, false>(f, g, parity, rule, cfg, gacc, st, est);
}

template <int NDIR>
hipError_t hb_half_sweep(const Link8Field32& f, const Geom& g, int parity, float T, uint64_t seed, uint32_t sweep,
                         const SweepConfig& cfg, const GField& gacc, hipStream_t st)
{
    const Rule<float> rule{1.0f, T, (uint32_t)seed, (uint32_t)(seed >> 32), sweep};
    if (gacc.base) return launch_mode<NDIR, false, float, HEATBATH, true>(f, g, parity, rule, cfg, gacc, st, nullptr);
    return launch_mode<NDIR, false, float, HEATBATH, false>(f, g, parity, rule, cfg, gacc, st, nullptr);
}

}  // namespace sweep_impl
}  // namespace gf
