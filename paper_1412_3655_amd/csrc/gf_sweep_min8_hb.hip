// gf_sweep_min8_hb.hip -- the heat-bath half-sweep of the annealing prelude
// (abstract of arXiv:1412.3655) over float64 links stored in 8 reals
// (gf_min8.h), Landau and Coulomb gauge.  Decoding yields SU(3) to rounding,
// so the 12-real layout's re-orthonormalisation on load is not needed here.
#include "gf_sweep_impl.h"

namespace gf {

hipError_t launch_hb_half_sweep(const Link8Field& f, const Geom& g, int parity, double T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, hipStream_t st, int gauge)
{
    if (gauge == GAUGE_COULOMB) return sweep_impl::hb_half_sweep<NDIR_COULOMB>(f, g, parity, T, seed, sweep, cfg, st);
    return sweep_impl::hb_half_sweep<NDIR_LANDAU>(f, g, parity, T, seed, sweep, cfg, st);
}

}  // namespace gf
