// gf_su2.h -- SU(2) link fields and the launchers of gf_su2.hip (internal C++ API).
#pragma once

#include "gf_kernels.h"

namespace gf {

// 16-byte chunks per SU(2) link (a quaternion of 4 reals)
template <typename R>
struct Su2Chunks;
template <>
struct Su2Chunks<double> {
    using T = double2;
    static constexpr int N = 2;
};
template <>
struct Su2Chunks<float> {
    using T = float4;
    static constexpr int N = 1;
};

// Quaternion links in the tiled checkerboard layout of the SU(3) fields:
// chunk c of U_mu at (parity, h) at base[(((parity 4 + mu) ld/64 + h/64) N + c) 64 + h mod 64].
template <typename R>
struct Su2Field {
    typename Su2Chunks<R>::T* base;
    uint32_t ld;
};

// Sweep configurations of the SU(2) kernel: one lane per site, block 64..512, cache policy 0..2.
bool su2_config_valid(const SweepConfig& c);
uint32_t su2_sweep_blocks(const Geom& g, const SweepConfig& c);
// Partial-sum pairs the SU(2) reductions need (Landau or per timeslice).
uint32_t su2_partials(const Geom& g);

// One overrelaxation half-sweep (est as for launch_or_half_sweep: 2 pairs per block of each colour).
hipError_t launch_su2_or(const Su2Field<double>& f, const Geom& g, int parity, double omega, int mode,
                         const SweepConfig& c, hipStream_t st, int gauge, double* est);
hipError_t launch_su2_or(const Su2Field<float>& f, const Geom& g, int parity, float omega, int mode,
                         const SweepConfig& c, hipStream_t st, int gauge, double* est);
// One heat-bath half-sweep at temperature T (Philox key seed, sweep counter sweep).
hipError_t launch_su2_hb(const Su2Field<double>& f, const Geom& g, int parity, double T, uint64_t seed,
                         uint32_t sweep, const SweepConfig& c, hipStream_t st, int gauge);
hipError_t launch_su2_hb(const Su2Field<float>& f, const Geom& g, int parity, float T, uint64_t seed,
                         uint32_t sweep, const SweepConfig& c, hipStream_t st, int gauge);
// Landau: out[0] = theta, out[1] = F.  Coulomb: out[2t] = theta_C(t), out[2t+1] = F_C(t).
hipError_t launch_su2_measure(const Su2Field<double>& f, const Geom& g, int gauge, double* partial, double* out,
                              hipStream_t st);
hipError_t launch_su2_measure(const Su2Field<float>& f, const Geom& g, int gauge, double* partial, double* out,
                              hipStream_t st);
hipError_t launch_su2_plaquette(const Su2Field<double>& f, const Geom& g, double* partial, double* out,
                                hipStream_t st);
hipError_t launch_su2_plaquette(const Su2Field<float>& f, const Geom& g, double* partial, double* out,
                                hipStream_t st);
hipError_t launch_su2_reunitarize(const Su2Field<double>& f, const Geom& g, hipStream_t st);
hipError_t launch_su2_reunitarize(const Su2Field<float>& f, const Geom& g, hipStream_t st);
// Canonical float64 [site][mu][2][2][re,im] (device) <-> quaternion layout.
hipError_t launch_su2_pack(const double* canon, const Su2Field<double>& f, const Geom& g, hipStream_t st);
hipError_t launch_su2_pack(const double* canon, const Su2Field<float>& f, const Geom& g, hipStream_t st);
hipError_t launch_su2_unpack(const Su2Field<double>& f, const Geom& g, double* canon, hipStream_t st);
hipError_t launch_su2_unpack(const Su2Field<float>& f, const Geom& g, double* canon, hipStream_t st);

}  // namespace gf
