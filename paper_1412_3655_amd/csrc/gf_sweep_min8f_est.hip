// gf_sweep_min8f_est.hip -- the estimating float32 overrelaxation half-sweeps
// (they also sum tr[Delta Delta^dag] of every site's K before its update, per
// block) over links stored in 8 reals (gf_min8.h), Landau and Coulomb gauge.
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_or_half_sweep_min8f_est(const Link8Field32& f, const Geom& g, int parity, float omega, int mode,
                                          const SweepConfig& cfg, const GField& gacc, hipStream_t st, double* est,
                                          int gauge)
{
    if (gauge == GAUGE_COULOMB)
        return sweep_impl::or_half_sweep<NDIR_COULOMB, true>(f, g, parity, omega, mode, cfg, gacc, st, est);
    return sweep_impl::or_half_sweep<NDIR_LANDAU, true>(f, g, parity, omega, mode, cfg, gacc, st, est);
}

}  // namespace gf
