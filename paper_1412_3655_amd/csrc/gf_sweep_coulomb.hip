// gf_sweep_coulomb.hip -- the Coulomb-gauge half-sweep launchers of libgf
// (Coulomb gauge is listed beside Landau gauge in the abstract and Sec. 1 of
// arXiv:1412.3655).  The kernel is the Landau one of gf_sweep_impl.h with K(x)
// summed over the spatial directions only, so each site maximises its share of
// sum_x sum_i Re tr[g(x) U_i(x) g(x+i^)^dag], one independent problem per
// timeslice; g(x) still transforms all 8 links at x (the temporal ones too),
// which keeps the configuration on its gauge orbit.  Traffic per site update is
// that of the Landau sweep.
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_or_half_sweep_coulomb(const LinkField<double>& f, const Geom& g, int parity, double omega,
                                        int mode, const SweepConfig& cfg, hipStream_t st, double* est)
{
    if (est) return launch_or_half_sweep_coulomb_est(f, g, parity, omega, mode, cfg, st, est);
    return sweep_impl::or_half_sweep<NDIR_COULOMB, false>(f, g, parity, omega, mode, cfg, st, nullptr);
}

hipError_t launch_or_half_sweep_coulomb(const LinkField<float>& f, const Geom& g, int parity, float omega,
                                        int mode, const SweepConfig& cfg, const GField& gacc, hipStream_t st,
                                        double* est)
{
    if (est) return launch_or_half_sweep_coulomb_est(f, g, parity, omega, mode, cfg, gacc, st, est);
    return sweep_impl::or_half_sweep<NDIR_COULOMB, false>(f, g, parity, omega, mode, cfg, gacc, st, nullptr);
}

hipError_t launch_hb_half_sweep_coulomb(const LinkField<double>& f, const Geom& g, int parity, double T,
                                        uint64_t seed, uint32_t sweep, const SweepConfig& cfg, hipStream_t st)
{
    return sweep_impl::hb_half_sweep<NDIR_COULOMB>(f, g, parity, T, seed, sweep, cfg, st);
}

hipError_t launch_hb_half_sweep_coulomb(const LinkField<float>& f, const Geom& g, int parity, float T,
                                        uint64_t seed, uint32_t sweep, const SweepConfig& cfg, const GField& gacc,
                                        hipStream_t st)
{
    return sweep_impl::hb_half_sweep<NDIR_COULOMB>(f, g, parity, T, seed, sweep, cfg, gacc, st);
}

}  // namespace gf
