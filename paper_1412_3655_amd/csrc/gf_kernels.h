// gf_kernels.h -- host-side launchers of the libgf kernels (internal C++ API).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf_device.h"

namespace gf {

// Sweep kernel configuration: lanes per site (1, 2, 4 or 8) and block size
// (64, 128, 256 or 512 threads).
struct SweepConfig {
    int tps = 4;
    int block = 256;
};

bool sweep_config_valid(const SweepConfig& c);

// One overrelaxation half-sweep over the sites of colour `parity`.
hipError_t launch_or_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double omega, int mode,
                                const SweepConfig& cfg, hipStream_t st);
hipError_t launch_or_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float omega, int mode,
                                const SweepConfig& cfg, hipStream_t st);

// theta / F: per-block partial sums (2 doubles per block) then one finalize
// block; out[0] = theta, out[1] = F.  partial must hold measure_partials(g).
uint32_t measure_blocks(const Geom& g);
hipError_t launch_measure(const LinkField<double>& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_measure(const LinkField<float>& f, const Geom& g, double* partial, double* out, hipStream_t st);

// Average plaquette into out[0]; partial as for launch_measure.
hipError_t launch_plaquette(const LinkField<double>& f, const Geom& g, double* partial, double* out, hipStream_t st);
hipError_t launch_plaquette(const LinkField<float>& f, const Geom& g, double* partial, double* out, hipStream_t st);

// Gram-Schmidt of rows 0, 1 of every link.
hipError_t launch_reunitarize(const LinkField<double>& f, const Geom& g, hipStream_t st);
hipError_t launch_reunitarize(const LinkField<float>& f, const Geom& g, hipStream_t st);

// Canonical float64 [site][mu][3][3][2] (device) <-> device layout.
hipError_t launch_pack(const double* canon, const LinkField<double>& f, const Geom& g, hipStream_t st);
hipError_t launch_pack(const double* canon, const LinkField<float>& f, const Geom& g, hipStream_t st);
hipError_t launch_unpack(const LinkField<double>& f, const Geom& g, double* canon, hipStream_t st);
hipError_t launch_unpack(const LinkField<float>& f, const Geom& g, double* canon, hipStream_t st);

}  // namespace gf
