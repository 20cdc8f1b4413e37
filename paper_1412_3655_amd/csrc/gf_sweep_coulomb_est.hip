// gf_sweep_coulomb_est.hip -- the Coulomb gauge overrelaxation half-sweeps that also sum
// tr[Delta Delta^dag] of every site's K before its update, per block (the
// fused estimate of the gauge condition, used to decide where the exact
// measurement of Sec. 2's stopping test is needed).  The kernel of
// gf_sweep_impl.h with EST = true, in a translation unit of its own so it
// compiles beside the plain sweeps.
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_or_half_sweep_coulomb_est(const LinkField<double>& f, const Geom& g, int parity, double omega, int mode,
                                            const SweepConfig& cfg, hipStream_t st, double* est)
{
    return sweep_impl::or_half_sweep<NDIR_COULOMB, true>(f, g, parity, omega, mode, cfg, st, est);
}

hipError_t launch_or_half_sweep_coulomb_est(const LinkField<float>& f, const Geom& g, int parity, float omega, int mode,
                                            const SweepConfig& cfg, const GField& gacc, hipStream_t st, double* est)
{
    return sweep_impl::or_half_sweep<NDIR_COULOMB, true>(f, g, parity, omega, mode, cfg, gacc, st, est);
}

}  // namespace gf
