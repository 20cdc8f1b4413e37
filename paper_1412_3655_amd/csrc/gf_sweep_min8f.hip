// gf_sweep_min8f.hip -- the float32 overrelaxation half-sweep (the bulk sweeps
// of GF_FP32 and GF_MIXED lattices) over links stored in 8 reals (the minimal
// representation named in Sec. 4.1 of arXiv:1412.3655; codec in gf_min8.h),
// Landau gauge, with or without g(x) tracking.  A site update moves 256 B read
// + 256 B written of links instead of 384 B + 384 B.  Coulomb gauge, the
// estimating sweeps and the heat bath of this layout are compiled in
// gf_sweep_min8f_coulomb.hip, gf_sweep_min8f_est.hip and gf_sweep_min8f_hb.hip.
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_or_half_sweep(const Link8Field32& f, const Geom& g, int parity, float omega, int mode,
                                const SweepConfig& cfg, const GField& gacc, hipStream_t st, int gauge, double* est)
{
    if (gauge == GAUGE_COULOMB)
        return launch_or_half_sweep_min8f_coulomb(f, g, parity, omega, mode, cfg, gacc, st, est);
    if (est) return launch_or_half_sweep_min8f_est(f, g, parity, omega, mode, cfg, gacc, st, est, GAUGE_LANDAU);
    return sweep_impl::or_half_sweep<NDIR_LANDAU, false>(f, g, parity, omega, mode, cfg, gacc, st, nullptr);
}

}  // namespace gf
