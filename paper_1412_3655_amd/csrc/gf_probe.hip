// gf_probe.hip -- a plain streaming copy of known traffic (gf_probe_copy),
// used to put the achieved bandwidth of the sweep in context and to calibrate
// hardware traffic counters: it reads `bytes` and writes `bytes`, nothing else.
#include "gf_internal.h"

using namespace gf::detail;

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void __launch_bounds__(256) k_probe_copy(const v4f* __restrict__ src, v4f* __restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        if constexpr (NT) {
            const v4f v = __builtin_nontemporal_load(src + i);
            __builtin_nontemporal_store(v, dst + i);
        } else {
            dst[i] = src[i];
        }
    }
}

}  // namespace

extern "C" gf_status gf_probe_copy(size_t bytes, int32_t reps, int32_t nontemporal, int32_t blocks, double* gbps)
{
    if (bytes < 4096 || bytes % 16 || reps < 1 || blocks < 1 || !gbps) return fail(GF_E_ARG, "bad arguments");
    const size_t n = bytes / 16;
    v4f *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void**)&a, bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&b, bytes);
    if (e == hipSuccess) e = hipMemset(a, 0, bytes);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.f;
    if (e == hipSuccess) {
        auto launch = [&]() {
            if (nontemporal)
                hipLaunchKernelGGL(k_probe_copy<true>, dim3(blocks), dim3(256), 0, nullptr, a, b, n);
            else
                hipLaunchKernelGGL(k_probe_copy<false>, dim3(blocks), dim3(256), 0, nullptr, a, b, n);
            return hipGetLastError();
        };
        e = launch();
        if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e != hipSuccess) return fail(GF_E_HIP, "probe: %s", hipGetErrorString(e));
    *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return GF_OK;
}
