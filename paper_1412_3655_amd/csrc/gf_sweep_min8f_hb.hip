// gf_sweep_min8f_hb.hip -- the float32 heat-bath half-sweep of the annealing
// prelude (abstract of arXiv:1412.3655) over links stored in 8 reals
// (gf_min8.h), Landau and Coulomb gauge, with or without g(x) tracking.
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_hb_half_sweep(const Link8Field32& f, const Geom& g, int parity, float T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, const GField& gacc, hipStream_t st, int gauge)
{
    if (gauge == GAUGE_COULOMB)
        return sweep_impl::hb_half_sweep<NDIR_COULOMB>(f, g, parity, T, seed, sweep, cfg, gacc, st);
    return sweep_impl::hb_half_sweep<NDIR_LANDAU>(f, g, parity, T, seed, sweep, cfg, gacc, st);
}

}  // namespace gf
