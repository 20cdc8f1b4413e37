// gf_sweep.hip -- the single-lattice half-sweep launchers of libgf on gfx950:
// Landau gauge here (K over all 4 directions, Eq. localfunctional of
// arXiv:1412.3655); the Coulomb instantiation of the same kernel is compiled
// in gf_sweep_coulomb.hip and reached through the gauge argument, the
// estimating sweeps in gf_sweep_est.hip / gf_sweep_coulomb_est.hip.
#include "gf_sweep_impl.h"

namespace gf {

bool sweep_config_valid(const SweepConfig& c)
{
    const bool tps_ok = c.tps == 1 || c.tps == 2 || c.tps == 4 || c.tps == 8;
    const bool blk_ok = c.block == 64 || c.block == 128 || c.block == 256 || c.block == 512;
    const bool nt_ok = c.nt == 0 || ((c.nt == 1 || c.nt == 2) && c.tps <= 4 && c.block <= 256);
    const bool minw_ok = c.minw == 0 || (c.minw == 2 && c.tps == 1);
    // one lane per site needs more than the 256 registers a 512-thread block allows
    return tps_ok && blk_ok && nt_ok && minw_ok && !(c.tps == 1 && c.block == 512);
}

hipError_t launch_or_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double omega, int mode,
                                const SweepConfig& cfg, hipStream_t st, int gauge, double* est)
{
    if (gauge == GAUGE_COULOMB) return launch_or_half_sweep_coulomb(f, g, parity, omega, mode, cfg, st, est);
    if (est) return launch_or_half_sweep_est(f, g, parity, omega, mode, cfg, st, est);
    return sweep_impl::or_half_sweep<NDIR_LANDAU, false>(f, g, parity, omega, mode, cfg, st, nullptr);
}

hipError_t launch_or_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float omega, int mode,
                                const SweepConfig& cfg, const GField& gacc, hipStream_t st, int gauge, double* est)
{
    if (gauge == GAUGE_COULOMB)
        return launch_or_half_sweep_coulomb(f, g, parity, omega, mode, cfg, gacc, st, est);
    if (est) return launch_or_half_sweep_est(f, g, parity, omega, mode, cfg, gacc, st, est);
    return sweep_impl::or_half_sweep<NDIR_LANDAU, false>(f, g, parity, omega, mode, cfg, gacc, st, nullptr);
}

uint32_t sweep_blocks(const Geom& g, const SweepConfig& cfg)
{
    return sweep_impl::sweep_grid(g, cfg);
}

hipError_t launch_hb_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, hipStream_t st, int gauge)
{
    if (gauge == GAUGE_COULOMB) return launch_hb_half_sweep_coulomb(f, g, parity, T, seed, sweep, cfg, st);
    return sweep_impl::hb_half_sweep<NDIR_LANDAU>(f, g, parity, T, seed, sweep, cfg, st);
}

hipError_t launch_hb_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, const GField& gacc, hipStream_t st, int gauge)
{
    if (gauge == GAUGE_COULOMB) return launch_hb_half_sweep_coulomb(f, g, parity, T, seed, sweep, cfg, gacc, st);
    return sweep_impl::hb_half_sweep<NDIR_LANDAU>(f, g, parity, T, seed, sweep, cfg, gacc, st);
}

}  // namespace gf
