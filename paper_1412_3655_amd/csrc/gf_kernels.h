// gf_kernels.h -- host-side launchers of the libgf kernels (internal C++ API).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf_device.h"
#include "gf_min8.h"

namespace gf {

// Sweep kernel configuration: lanes per site (1, 2, 4 or 8), block size
// (64, 128, 256 or 512 threads), cache policy of the link accesses (0 =
// plain, 1 = non-temporal loads and stores, 2 = plain loads and non-temporal
// stores; 1 and 2 with tps <= 4 and block <= 256) and register limit (minw:
// 0 = the compiler's allocation, 2 = at least 2 waves per SIMD, i.e. at most
// 256 registers per lane; only with tps 1, where a float64 site update
// otherwise takes 256 VGPRs + 68 AGPRs and 1 wave per SIMD).
struct SweepConfig {
    int tps = 4;
    int block = 256;
    int nt = 0;
    int minw = 0;
};

bool sweep_config_valid(const SweepConfig& c);

// Gauge of a lattice's functional: Landau (K over all 4 directions) or
// Coulomb (K over x, y, z; one independent problem per timeslice).
constexpr int GAUGE_LANDAU = 0;
constexpr int GAUGE_COULOMB = 1;

// One overrelaxation half-sweep over the sites of colour `parity`.  est !=
// nullptr: the launch also writes its per-block sums of tr[Delta Delta^dag]
// before the update as pairs at est + 2 * parity * sweep_blocks(g, cfg)
// (colour 0 first, then colour 1: 4 * sweep_blocks doubles for a sweep).
hipError_t launch_or_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double omega, int mode,
                                const SweepConfig& cfg, hipStream_t st, int gauge = GAUGE_LANDAU,
                                double* est = nullptr);
// float32; with gacc.base != nullptr the sweep also accumulates g(x) <- G g(x).
hipError_t launch_or_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float omega, int mode,
                                const SweepConfig& cfg, const GField& gacc, hipStream_t st,
                                int gauge = GAUGE_LANDAU, double* est = nullptr);
uint32_t sweep_blocks(const Geom& g, const SweepConfig& cfg);

// One heat-bath half-sweep at temperature T: Philox key = seed, sweep counter
// `sweep` (float32 with gacc.base != nullptr also accumulates g).
hipError_t launch_hb_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, hipStream_t st, int gauge = GAUGE_LANDAU);
hipError_t launch_hb_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, const GField& gacc, hipStream_t st,
                                int gauge = GAUGE_LANDAU);

// The Coulomb instantiations (gf_sweep_coulomb.hip) behind gauge = GAUGE_COULOMB.
hipError_t launch_or_half_sweep_coulomb(const LinkField<double>& f, const Geom& g, int parity, double omega,
                                        int mode, const SweepConfig& cfg, hipStream_t st, double* est);
hipError_t launch_or_half_sweep_coulomb(const LinkField<float>& f, const Geom& g, int parity, float omega,
                                        int mode, const SweepConfig& cfg, const GField& gacc, hipStream_t st,
                                        double* est);
// The estimating overrelaxation sweeps (gf_sweep_est.hip, gf_sweep_coulomb_est.hip); est != nullptr.
hipError_t launch_or_half_sweep_est(const LinkField<double>& f, const Geom& g, int parity, double omega, int mode,
                                    const SweepConfig& cfg, hipStream_t st, double* est);
hipError_t launch_or_half_sweep_est(const LinkField<float>& f, const Geom& g, int parity, float omega, int mode,
                                    const SweepConfig& cfg, const GField& gacc, hipStream_t st, double* est);
hipError_t launch_or_half_sweep_coulomb_est(const LinkField<double>& f, const Geom& g, int parity, double omega,
                                            int mode, const SweepConfig& cfg, hipStream_t st, double* est);
hipError_t launch_or_half_sweep_coulomb_est(const LinkField<float>& f, const Geom& g, int parity, float omega,
                                            int mode, const SweepConfig& cfg, const GField& gacc, hipStream_t st,
                                            double* est);
hipError_t launch_hb_half_sweep_coulomb(const LinkField<double>& f, const Geom& g, int parity, double T,
                                        uint64_t seed, uint32_t sweep, const SweepConfig& cfg, hipStream_t st);
hipError_t launch_hb_half_sweep_coulomb(const LinkField<float>& f, const Geom& g, int parity, float T,
                                        uint64_t seed, uint32_t sweep, const SweepConfig& cfg, const GField& gacc,
                                        hipStream_t st);

// Float64 links stored in 8 reals (gf_min8.h): the same sweeps, decoding on
// load and encoding on store; est as above.
hipError_t launch_or_half_sweep(const Link8Field& f, const Geom& g, int parity, double omega, int mode,
                                const SweepConfig& cfg, hipStream_t st, int gauge = GAUGE_LANDAU,
                                double* est = nullptr);
hipError_t launch_hb_half_sweep(const Link8Field& f, const Geom& g, int parity, double T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, hipStream_t st, int gauge = GAUGE_LANDAU);
hipError_t launch_or_half_sweep_min8_coulomb(const Link8Field& f, const Geom& g, int parity, double omega, int mode,
                                             const SweepConfig& cfg, hipStream_t st, double* est);
hipError_t launch_or_half_sweep_min8_est(const Link8Field& f, const Geom& g, int parity, double omega, int mode,
                                         const SweepConfig& cfg, hipStream_t st, double* est, int gauge);

// Float32 links stored in 8 reals (gf_min8.h): the float32 sweeps (g tracked
// when gacc.base is set), decoding and encoding in float32; est as above.
hipError_t launch_or_half_sweep(const Link8Field32& f, const Geom& g, int parity, float omega, int mode,
                                const SweepConfig& cfg, const GField& gacc, hipStream_t st, int gauge = GAUGE_LANDAU,
                                double* est = nullptr);
hipError_t launch_hb_half_sweep(const Link8Field32& f, const Geom& g, int parity, float T, uint64_t seed,
                                uint32_t sweep, const SweepConfig& cfg, const GField& gacc, hipStream_t st,
                                int gauge = GAUGE_LANDAU);
hipError_t launch_or_half_sweep_min8f_coulomb(const Link8Field32& f, const Geom& g, int parity, float omega,
                                              int mode, const SweepConfig& cfg, const GField& gacc, hipStream_t st,
                                              double* est);
hipError_t launch_or_half_sweep_min8f_est(const Link8Field32& f, const Geom& g, int parity, float omega, int mode,
                                          const SweepConfig& cfg, const GField& gacc, hipStream_t st, double* est,
                                          int gauge);

// theta / F: per-block partial sums (2 doubles per block) then one finalize
// block; out[0] = theta, out[1] = F.  partial must hold measure_partials(g).
uint32_t measure_blocks(const Geom& g);
// out[0] = s0 * sum of the n pairs' first halves, out[1] = s1 * second halves,
// in index order (one block).
hipError_t launch_finalize(const double* partial, uint32_t n, double s0, double s1, double* out, hipStream_t st);
hipError_t launch_measure(const LinkField<double>& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_measure(const LinkField<float>& f, const Geom& g, double* partial, double* out, hipStream_t st);
// The same over links in the ABI's canonical float64 array (device), read in
// place; bitwise equal to launch_measure over the packed float64 field.
hipError_t launch_measure_canonical(const double* canon, const Geom& g, double* partial, double* out, hipStream_t st);

// Coulomb gauge, per timeslice t = 0 .. Nt-1: out[2t] = theta_C(t) =
// (1/(3 V3)) sum_{x in t} tr[Delta_C Delta_C^dag], out[2t+1] = F_C(t) =
// (1/(9 V3)) sum_{x in t} sum_i Re tr U_i(x), with V3 = Nx Ny Nz; every
// timeslice's per-block partials are added in index order by one block.
// partial must hold slice_partials(g) pairs.
uint32_t slice_partials(const Geom& g);
hipError_t launch_measure_slices(const LinkField<double>& f, const Geom& g, double* partial, double* out,
                                 hipStream_t st);
hipError_t launch_measure_slices(const LinkField<float>& f, const Geom& g, double* partial, double* out,
                                 hipStream_t st);

// out[0] = (1/(3V)) sum_x tr[E E^dag], E = Delta computed in float32 from the
// float32-rounded links minus Delta in float64: the float32 rounding floor of
// theta for this configuration.  min8: the links rounded through the 8-real
// float32 storage instead of rows 0, 1 rounded.  partial as for launch_measure.
hipError_t launch_fp32_floor(const LinkField<double>& f, const Geom& g, double* partial, double* out, hipStream_t st,
                             bool min8 = false);

// Average plaquette into out[0]; partial as for launch_measure.
hipError_t launch_plaquette(const LinkField<double>& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_plaquette(const LinkField<float>& f, const Geom& g, double* partial, double* out, hipStream_t st);

// Gram-Schmidt of rows 0, 1 of every link.
hipError_t launch_reunitarize(const LinkField<double>& f, const Geom& g, hipStream_t st);
hipError_t launch_reunitarize(const LinkField<float>& f, const Geom& g, hipStream_t st);

// The reductions and layout conversion of links stored in 8 reals (pack
// encodes, unpack decodes; float32 values are decoded and encoded in float64,
// the encoded values rounded to float32).
hipError_t launch_measure(const Link8Field& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_measure_slices(const Link8Field& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_plaquette(const Link8Field& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_pack(const double* canon, const Link8Field& f, const Geom& g, hipStream_t st);
hipError_t launch_unpack(const Link8Field& f, const Geom& g, double* canon, hipStream_t st);
hipError_t launch_measure(const Link8Field32& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_measure_slices(const Link8Field32& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_plaquette(const Link8Field32& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_pack(const double* canon, const Link8Field32& f, const Geom& g, hipStream_t st);
hipError_t launch_unpack(const Link8Field32& f, const Geom& g, double* canon, hipStream_t st);
hipError_t launch_pack_range(const double* canon, const Link8Field32& f, const Geom& g, uint64_t first, uint64_t n,
                             hipStream_t st);
hipError_t launch_unpack_range(const Link8Field32& f, const Geom& g, double* canon, uint64_t first, uint64_t n,
                               hipStream_t st);

// Every link of a float64 field converted to the other storage (12 -> 8 reals
// projects rows 0, 1 onto SU(3) like a store; 8 -> 12 writes the decoded rows).
hipError_t launch_convert(const LinkField<double>& from, const Link8Field& to, const Geom& g, hipStream_t st);
hipError_t launch_convert(const Link8Field& from, const LinkField<double>& to, const Geom& g, hipStream_t st);
hipError_t launch_convert(const LinkField<float>& from, const Link8Field32& to, const Geom& g, hipStream_t st);
hipError_t launch_convert(const Link8Field32& from, const LinkField<float>& to, const Geom& g, hipStream_t st);

// Canonical float64 [site][mu][3][3][2] (device) <-> device layout.
hipError_t launch_pack(const double* canon, const LinkField<double>& f, const Geom& g, hipStream_t st);
hipError_t launch_pack(const double* canon, const LinkField<float>& f, const Geom& g, hipStream_t st);
hipError_t launch_unpack(const LinkField<double>& f, const Geom& g, double* canon, hipStream_t st);
hipError_t launch_unpack(const LinkField<float>& f, const Geom& g, double* canon, hipStream_t st);
// The same for the canonical links first .. first+n-1 (4 per site, lexicographic
// site order), held at canon[0 .. 18 n): a lattice moves through a staging
// buffer smaller than itself.  The range must lie inside the lattice.
hipError_t launch_pack_range(const double* canon, const LinkField<double>& f, const Geom& g, uint64_t first,
                             uint64_t n, hipStream_t st);
hipError_t launch_pack_range(const double* canon, const LinkField<float>& f, const Geom& g, uint64_t first,
                             uint64_t n, hipStream_t st);
hipError_t launch_unpack_range(const LinkField<double>& f, const Geom& g, double* canon, uint64_t first, uint64_t n,
                               hipStream_t st);
hipError_t launch_unpack_range(const LinkField<float>& f, const Geom& g, double* canon, uint64_t first, uint64_t n,
                               hipStream_t st);

// Mixed precision: g(x) <- 1; Gram-Schmidt of g; and the float64 rebuild
// U_mu(x) <- g(x) U0_mu(x) g(x+mu^)^dag in place over the float64 field that
// holds U0 (g re-orthonormalised in float64 first).
hipError_t launch_g_identity(const GField& gacc, const Geom& g, hipStream_t st);
hipError_t launch_g_reunitarize(const GField& gacc, const Geom& g, hipStream_t st);
hipError_t launch_rebuild_from_g(const LinkField<double>& u0, const GField& gacc, const Geom& g, hipStream_t st);

}  // namespace gf
