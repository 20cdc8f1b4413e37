// gf_noalloc.hip -- gf_measure_theta_F_noalloc: the theta / F measurement of
// gf_measure_theta_F over links the caller holds in the canonical float64
// layout on the device, for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops).  Its only scratch, the
// per-block partial sums of the reduction, lives in a fixed device array of
// this file; nothing is allocated or freed.
#include <mutex>

#include "gf_internal.h"

using namespace gf::detail;

namespace {

// Partial sums of the theta / F reduction: 2 doubles per block, 2 blocks per
// 256 sites of each colour, so 1 MiB serves lattices of up to 2^24 sites.
constexpr size_t kScratchDoubles = (size_t)1 << 17;

static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` per device (each GPU holds its own copy of the
// array).  The host symbol `scratch` is not a device address: only these
// pointers are passed to kernels.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

gf_status scratch_of_current_device(double** out)
{
    int dev = 0;
    GF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GF_E_ARG, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        GF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GF_E_HIP, "hipGetSymbolAddress returned a null address");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return GF_OK;
}

}  // namespace

extern "C" {

gf_status gf_measure_theta_F_noalloc(const int32_t dims[4], const double* dev_links, double* dev_out,
                                     void* hip_stream)
{
    if (!dims || !dev_links || !dev_out) return fail(GF_E_ARG, "null argument");
    int64_t V = 0;
    GF_TRY(check_dims(dims, &V));
    gf::Geom g{};
    if (!make_geom(dims, &g)) return fail(GF_E_ARG, "internal: index division check failed");
    const size_t need = 2 * (size_t)gf::measure_blocks(g);
    if (need > kScratchDoubles)
        return fail(GF_E_ARG,
                    "lattice of %lld sites needs %zu doubles of reduction scratch; the allocation-free "
                    "measurement holds %zu (at most %lld sites)",
                    (long long)V, need, kScratchDoubles, (long long)(kScratchDoubles / 2 * 256));
    double* partial = nullptr;
    GF_TRY(scratch_of_current_device(&partial));
    GF_HIP(gf::launch_measure_canonical(dev_links, g, partial, dev_out, (hipStream_t)hip_stream));
    return GF_OK;
}

}  // extern "C"
