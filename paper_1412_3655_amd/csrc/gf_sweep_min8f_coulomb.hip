// gf_sweep_min8f_coulomb.hip -- the Coulomb-gauge float32 overrelaxation
// half-sweep (K over x, y, z; abstract and Sec. 1 of arXiv:1412.3655) over
// links stored in 8 reals (gf_min8.h).
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_or_half_sweep_min8f_coulomb(const Link8Field32& f, const Geom& g, int parity, float omega,
                                              int mode, const SweepConfig& cfg, const GField& gacc, hipStream_t st,
                                              double* est)
{
    if (est) return launch_or_half_sweep_min8f_est(f, g, parity, omega, mode, cfg, gacc, st, est, GAUGE_COULOMB);
    return sweep_impl::or_half_sweep<NDIR_COULOMB, false>(f, g, parity, omega, mode, cfg, gacc, st, nullptr);
}

}  // namespace gf
