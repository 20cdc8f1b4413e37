// gf_sweep_min8_coulomb.hip -- the Coulomb-gauge overrelaxation half-sweep
// (K over x, y, z; abstract and Sec. 1 of arXiv:1412.3655) over float64 links
// stored in 8 reals (gf_min8.h).
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_or_half_sweep_min8_coulomb(const Link8Field& f, const Geom& g, int parity, double omega, int mode,
                                             const SweepConfig& cfg, hipStream_t st, double* est)
{
    if (est) return launch_or_half_sweep_min8_est(f, g, parity, omega, mode, cfg, st, est, GAUGE_COULOMB);
    return sweep_impl::or_half_sweep<NDIR_COULOMB, false>(f, g, parity, omega, mode, cfg, st, nullptr);
}

}  // namespace gf
