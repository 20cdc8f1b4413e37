// gf_sweep_min8_est.hip -- the estimating overrelaxation half-sweeps (they also
// sum tr[Delta Delta^dag] of every site's K before its update, per block) over
// float64 links stored in 8 reals (gf_min8.h), Landau and Coulomb gauge.
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_or_half_sweep_min8_est(const Link8Field& f, const Geom& g, int parity, double omega, int mode,
                                         const SweepConfig& cfg, hipStream_t st, double* est, int gauge)
{
    if (gauge == GAUGE_COULOMB)
        return sweep_impl::or_half_sweep<NDIR_COULOMB, true>(f, g, parity, omega, mode, cfg, st, est);
    return sweep_impl::or_half_sweep<NDIR_LANDAU, true>(f, g, parity, omega, mode, cfg, st, est);
}

}  // namespace gf
