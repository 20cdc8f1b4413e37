// gf_sweep_min8.hip -- the overrelaxation half-sweep over float64 links stored
// in 8 reals (the minimal representation named in Sec. 4.1 of
// arXiv:1412.3655; codec in gf_min8.h), Landau gauge.  The kernel of
// gf_sweep_impl.h with the 8-real field: every link is decoded on load and
// encoded on store, so a site update moves 512 B read + 512 B written instead
// of 768 B + 768 B.  Coulomb gauge, the estimating sweeps and the heat bath of
// this layout are compiled in gf_sweep_min8_coulomb.hip, gf_sweep_min8_est.hip
// and gf_sweep_min8_hb.hip.
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_or_half_sweep(const Link8Field& f, const Geom& g, int parity, double omega, int mode,
                                const SweepConfig& cfg, hipStream_t st, int gauge, double* est)
{
    if (gauge == GAUGE_COULOMB) return launch_or_half_sweep_min8_coulomb(f, g, parity, omega, mode, cfg, st, est);
    if (est) return launch_or_half_sweep_min8_est(f, g, parity, omega, mode, cfg, st, est, GAUGE_LANDAU);
    return sweep_impl::or_half_sweep<NDIR_LANDAU, false>(f, g, parity, omega, mode, cfg, st, nullptr);
}

}  // namespace gf
