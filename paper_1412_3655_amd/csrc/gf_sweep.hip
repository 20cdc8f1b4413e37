// gf_sweep.hip -- the single-lattice checkerboard half-sweep kernels
// (overrelaxation and heat bath, Sec. 2 and the abstract of arXiv:1412.3655)
// for gfx950.  The per-site body lives in gf_site.h.  The loop over sites is
// over the half index of one colour: every link is read once and written once
// per half-sweep (per site update in FP64 with 12-real links: 768 B read and
// 768 B written).
#include "gf_kernels.h"
#include "gf_site.h"

namespace gf {

namespace {

template <typename R, int TPS, int MODE, int BLOCK, bool TRACKG, int CP>
__global__ void __launch_bounds__(BLOCK) k_or_half_sweep(LinkField<R> f, Geom g, int parity, Rule<R> rule,
                                                         GField gacc)
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
    // whole groups of TPS lanes leave together, so every DPP partner is live
    if (h >= g.vh) return;
    site_update<R, TPS, MODE, TRACKG, CP>(f, g, parity, h, r, rule, gacc);
}

template <typename R, int TPS, int MODE, bool TRACKG>
hipError_t launch_tps(const LinkField<R>& f, const Geom& g, int parity, const Rule<R>& rule, const SweepConfig& c,
                      const GField& gacc, hipStream_t st)
{
    const int block = c.block;
    const uint64_t threads = (uint64_t)g.vh * TPS;
    const uint32_t grid = (uint32_t)((threads + block - 1) / block);
    if (grid == 0) return hipSuccess;
#define GF_LAUNCH(B, CPV) \
    hipLaunchKernelGGL((k_or_half_sweep<R, TPS, MODE, B, TRACKG, CPV>), dim3(grid), dim3(B), 0, st, f, g, parity, rule, gacc)
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

template <typename R, int MODE, bool TRACKG>
hipError_t launch_mode(const LinkField<R>& f, const Geom& g, int parity, const Rule<R>& rule, const SweepConfig& c,
                       const GField& gacc, hipStream_t st)
{
    switch (c.tps) {
        case 1: return launch_tps<R, 1, MODE, TRACKG>(f, g, parity, rule, c, gacc, st);
        case 2: return launch_tps<R, 2, MODE, TRACKG>(f, g, parity, rule, c, gacc, st);
        case 8: return launch_tps<R, 8, MODE, TRACKG>(f, g, parity, rule, c, gacc, st);
        default: return launch_tps<R, 4, MODE, TRACKG>(f, g, parity, rule, c, gacc, st);
    }
}

}  // namespace

bool sweep_config_valid(const SweepConfig& c)
{
    const bool tps_ok = c.tps == 1 || c.tps == 2 || c.tps == 4 || c.tps == 8;
    const bool blk_ok = c.block == 64 || c.block == 128 || c.block == 256 || c.block == 512;
    const bool nt_ok = c.nt == 0 || ((c.nt == 1 || c.nt == 2) && c.tps <= 4 && c.block <= 256);
    // one lane per site needs more than the 256 registers a 512-thread block allows
    return tps_ok && blk_ok && nt_ok && !(c.tps == 1 && c.block == 512);
}

hipError_t launch_or_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double omega, int mode,
                                const SweepConfig& cfg, hipStream_t st)
{
    const GField none{nullptr, 0};
    const Rule<double> rule{omega, 1.0, 0u, 0u, 0u};
    return mode == OR_EXACT ? launch_mode<double, 0, false>(f, g, parity, rule, cfg, none, st)
                            : launch_mode<double, 1, false>(f, g, parity, rule, cfg, none, st);
}

hipError_t launch_or_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float omega, int mode,
                                const SweepConfig& cfg, const GField& gacc, hipStream_t st)
{
    const Rule<float> rule{omega, 1.0f, 0u, 0u, 0u};
    if (gacc.base)
        return mode == OR_EXACT ? launch_mode<float, 0, true>(f, g, parity, rule, cfg, gacc, st)
                                : launch_mode<float, 1, true>(f, g, parity, rule, cfg, gacc, st);
    return mode == OR_EXACT ? launch_mode<float, 0, false>(f, g, parity, rule, cfg, gacc, st)
                            : launch_mode<float, 1, false>(f, g, parity, rule, cfg, gacc, st);
}

hipError_t launch_hb_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, hipStream_t st)
{
    const GField none{nullptr, 0};
    const Rule<double> rule{1.0, T, (uint32_t)seed, (uint32_t)(seed >> 32), sweep};
    return launch_mode<double, HEATBATH, false>(f, g, parity, rule, cfg, none, st);
}

hipError_t launch_hb_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, const GField& gacc, hipStream_t st)
{
    const Rule<float> rule{1.0f, T, (uint32_t)seed, (uint32_t)(seed >> 32), sweep};
    if (gacc.base) return launch_mode<float, HEATBATH, true>(f, g, parity, rule, cfg, gacc, st);
    return launch_mode<float, HEATBATH, false>(f, g, parity, rule, cfg, gacc, st);
}

}  // namespace gf
