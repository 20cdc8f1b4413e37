// gf_pool.hip -- batched sweeps of many resident lattices and the job pool
// behind gf_pool_* (include/gf.h).
//
// Each job owns an ordinary lattice object; the pool keeps a device table
// with one descriptor per slot (field pointers, geometry, rule parameters)
// and, per pool step of C = check_every sweeps, device work lists:
// for sweep k of the step and each kernel kind (heat bath / OR in float32
// with g tracking / OR in float64 / reunitarisation / measurement /
// finalisation) the list of slots that take part, as (slot, first tile)
// prefix entries, so one launch per (sweep, kind) covers every lattice of
// every shape.  Work lists and the slot table live in device memory and are
// refreshed by one host-to-device copy per step; the launches of a step are
// captured in a hipGraph once per work structure (which (k, kind) lists are
// non-empty) and replayed.  A sweep launch has one block per tile of its
// list: before each replay the grid of every captured sweep node is set to
// its list's tile count (hipGraphExecKernelNodeSetParams).  The other kinds
// (reunitarisation, measurement, finalisation) keep persistent grids that
// stride over their tiles.  A persistent sweep was measured ~13 % slower on
// MI355X: across the loop the compiler keeps the math library's polynomial
// coefficients of the exact power in registers, which pushes the float64
// sweep over the register file into accumulation-register spills.
//
// A step may be left running while the host admits, polls, fetches and
// releases jobs (gf_pool_step_async): those touch only lattices that the step
// in flight does not use, on a second stream, so the host's work (copying a
// job's links from pageable memory through a fixed staging buffer, packing
// them, its first measurement) overlaps the GPU's.  Lattices released while a
// step runs are freed when it has been completed (freeing synchronises the
// device).
//
// The per-site bodies are the same functions the single-lattice kernels use
// (gf_site.h) and the block decomposition of the measurement is the same, so
// every job's links, theta and F are bitwise those of the same job run alone
// through gf_anneal / gf_fix_until.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "gf_internal.h"
#include "gf_site.h"

namespace gf {
namespace pool {

constexpr int PBLOCK = 256;  // threads per block of the reunitarisation / measurement kernels
constexpr int kHeatBathTps = 1;  // lanes per site of the heat-bath sweeps (its sampling is per lane)
constexpr int kHeatBathBlock = 128;  // threads per block of the heat-bath sweeps
// Default shape of the overrelaxation sweeps (lanes per site, threads per
// block): the fastest over 64 lattices of 12^4 to 24^3x48 on MI355X (float32
// with g: 2 lanes with 12-real links, 1 lane with 8-real links, 5 % ahead of
// 2; float64: 1 lane, 3 % ahead of 2; 128 threads for all) and cache policy
// (non-temporal for float32 in 8 reals, 1-4 % ahead of plain at one lane;
// plain for float32 in 12 reals; non-temporal for float64); gf_pool_autotune
// picks them for the resident mix.
constexpr int kDefaultTps32 = 2, kDefaultTps32Min8 = 1, kDefaultTps64 = 1, kDefaultBlock = 128;
// Staging buffer through which admissions and fetches move a job's canonical
// links (18 doubles per link) in chunks; a multiple of one site's 4 links.
constexpr size_t kStageLinks = (size_t)4 * 58254;  // 33.6 MB

struct SlotDev {
    LinkField<double> f64;
    LinkField<float> f32;
    GField gacc;
    Geom g;
    double omega;
    double T0, T1;
    int32_t n_anneal;
    uint32_t key0, key1;
    uint32_t anneal_base;  // heat-bath sweeps done before this step
    double scale_theta, scale_F;
    double* partial;
    double* result;
};

// (slot, first tile) prefix entries; entry n (the sentinel) holds the tile total.
struct Entry {
    uint32_t slot;
    uint32_t first;
};

enum Kind { K_HB32 = 0, K_OR32, K_OR64, K_HB64, K_R32, K_R64, K_M32, K_M64, K_FIN, NKIND };

__device__ __forceinline__ uint32_t find_entry(const Entry* e, uint32_t n, uint32_t t)
{
    uint32_t lo = 0, hi = n;  // e[lo].first <= t < e[hi].first
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (e[mid].first <= t)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// The entry of tile t found by one wave in one pass of independent loads:
// every lane reads a strided share of the segment's `stride` entries while
// the count is read, and the wave counts the entries j < n with
// first <= t (first is a prefix sum from 0, so that count minus one is the
// entry).  A binary search would chain log2(n) dependent loads before the
// block could issue its first link load.  Lists of up to 64 * kWaveEntries
// entries; *slot and *first receive the entry's fields (false: empty list).
constexpr uint32_t kWaveEntries = 8;

__device__ __forceinline__ bool find_entry_wave(const Entry* e, const uint32_t* count, uint32_t stride, uint32_t t,
                                                uint32_t* slot, uint32_t* first)
{
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t fs[kWaveEntries], ss[kWaveEntries];
#pragma unroll
    for (uint32_t q = 0; q < kWaveEntries; ++q) {
        const uint32_t j = lane + 64u * q;
        fs[q] = 0xFFFFFFFFu;
        ss[q] = 0u;
        if (j < stride) {
            fs[q] = e[j].first;
            ss[q] = e[j].slot;
        }
    }
    const uint32_t n = *count;
    uint32_t cnt = 0;
#pragma unroll
    for (uint32_t q = 0; q < kWaveEntries; ++q) {
        const uint32_t j = lane + 64u * q;
        cnt += (uint32_t)__popcll(__ballot(j < n && fs[q] <= t));
    }
    if (cnt == 0u) return false;  // empty list (never launched)
    const uint32_t i = cnt - 1u;
    uint32_t my_slot = 0u, my_first = 0u;
#pragma unroll
    for (uint32_t q = 0; q < kWaveEntries; ++q)
        if (q == i / 64u) {
            my_slot = ss[q];
            my_first = fs[q];
        }
    *slot = (uint32_t)__shfl((int)my_slot, (int)(i % 64u), 64);
    *first = (uint32_t)__shfl((int)my_first, (int)(i % 64u), 64);
    return true;
}

template <typename R>
__device__ __forceinline__ LinkField<R> field_of(const SlotDev& sd);
template <>
__device__ __forceinline__ LinkField<double> field_of<double>(const SlotDev& sd)
{
    return sd.f64;
}
template <>
__device__ __forceinline__ LinkField<float> field_of<float>(const SlotDev& sd)
{
    return sd.f32;
}

// The float32 links of a pool whose float32 links are stored in 8 reals.
__device__ __forceinline__ Link8Field32 field8_of(const SlotDev& sd)
{
    return Link8Field32{sd.f32.base, sd.f32.ld};
}

// Linear schedule of gf_anneal: T_start at sweep 0, T_end at sweep n - 1,
// both endpoints exact (float64).
__device__ __forceinline__ double schedule_T(const SlotDev& sd, uint32_t s)
{
    if (sd.n_anneal <= 1 || s == 0) return sd.T0;
    if (s == (uint32_t)(sd.n_anneal - 1)) return sd.T1;
    return sd.T0 + (sd.T1 - sd.T0) * (double)s / (double)(sd.n_anneal - 1);
}

// CP: cache policy of the link accesses (gf_device.h: 0 plain, 1 non-temporal),
// a pool setting per precision (defaults above) and an axis of
// gf_pool_autotune.
// Block t sweeps tile t of the list (the host launches one block per tile of
// the list; a block past the tile total lands past the last lattice's sites
// and leaves).  With plain loads the white half-sweep takes the tiles in
// reverse order, so it starts on the links the black sweep touched last
// (still in the Infinity Cache); with non-temporal loads it keeps the forward
// order (on MI355X the reverse order made non-temporal float64 sweeps 1-2 %
// slower and plain float32 ones 3 % faster).  The order inside a colour does
// not change the result.  stride = entries per list segment.  A tile is
// BLOCK / TPS sites.  M8: float32 links stored in 8 reals.
template <typename R, int TPS, int MODE, bool TRACKG, int BLOCK, bool M8, int CP>
__global__ void __launch_bounds__(BLOCK) k_pool_sweep(const SlotDev* __restrict__ slots,
                                                      const Entry* __restrict__ list,
                                                      const uint32_t* __restrict__ count, uint32_t stride,
                                                      int parity, uint32_t k)
{
    constexpr uint32_t SPB = BLOCK / TPS;
    const uint32_t t = (parity && !nt_loads(CP)) ? gridDim.x - 1u - blockIdx.x : blockIdx.x;
    uint32_t slot, first;
    if (stride <= 64u * kWaveEntries) {
        if (!find_entry_wave(list, count, stride, t, &slot, &first)) return;
    } else {
        const uint32_t n = *count;
        if (t >= list[n].first) return;
        const uint32_t i = find_entry(list, n, t);
        slot = list[i].slot;
        first = list[i].first;
    }
    // The tile, hence its entry, is the block's: moving slot and first to scalar
    // registers lets the slot descriptor load through the scalar cache and keeps
    // the geometry's index arithmetic on the scalar unit, as in the
    // single-lattice kernel, whose geometry is a kernel argument.
    slot = __builtin_amdgcn_readfirstlane(slot);
    first = __builtin_amdgcn_readfirstlane(first);
    const SlotDev sd = slots[slot];
    const uint32_t h = (t - first) * SPB + threadIdx.x / TPS;
    const int r = (int)(threadIdx.x % TPS);
    if (h >= sd.g.vh) return;  // whole TPS groups leave together
    Rule<R> rule;
    if constexpr (MODE == HEATBATH) {
        const uint32_t s = sd.anneal_base + k;
        rule = Rule<R>{R(1), (R)schedule_T(sd, s), sd.key0, sd.key1, s};
    } else {
        rule = Rule<R>{(R)sd.omega, R(1), 0u, 0u, 0u};
    }
    if constexpr (M8)
        site_update<R, TPS, MODE, TRACKG, CP, NDIR_LANDAU, Link8Field32>(field8_of(sd), sd.g, parity, h, r, rule,
                                                                         sd.gacc);
    else
        site_update<R, TPS, MODE, TRACKG, CP>(field_of<R>(sd), sd.g, parity, h, r, rule, sd.gacc);
}

// M8: 8-real links are SU(3) at every store; only g(x) is reunitarised.
template <typename R, bool WITH_G, bool M8>
__global__ void __launch_bounds__(PBLOCK) k_pool_reunit(const SlotDev* __restrict__ slots,
                                                        const Entry* __restrict__ list,
                                                        const uint32_t* __restrict__ count)
{
    const uint32_t n = *count;
    const uint32_t total = list[n].first;
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        const uint32_t i = find_entry(list, n, t);
        const SlotDev sd = slots[list[i].slot];
        const uint32_t h = (t - list[i].first) * PBLOCK + threadIdx.x;
        if (h >= sd.g.vh) continue;
        const LinkField<R> f = field_of<R>(sd);
        for (int pm = 0; pm < 8 && !M8; ++pm) {
            M3<R> u;
            load_rows01(f, pm >> 2, pm & 3, h, u);
            gram_schmidt_rows01(u);
            store_rows01(f, pm >> 2, pm & 3, h, u);
        }
        if constexpr (WITH_G) {
            for (int p = 0; p < 2; ++p) {
                M3<float> u;
                load_g(sd.gacc, p, h, u);
                gram_schmidt_rows01(u);
#pragma unroll
                for (int c = 0; c < 3; ++c) store_g_chunk(sd.gacc, p, h, c, u);
            }
        }
    }
}

// Tile b of a slot = measurement block (parity = b / nb, block = b % nb) of the
// single-lattice measurement, writing the same partial.
template <typename R, bool M8>
__global__ void __launch_bounds__(PBLOCK) k_pool_measure(const SlotDev* __restrict__ slots,
                                                         const Entry* __restrict__ list,
                                                         const uint32_t* __restrict__ count)
{
    const uint32_t n = *count;
    const uint32_t total = list[n].first;
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        const uint32_t i = find_entry(list, n, t);
        const SlotDev sd = slots[list[i].slot];
        const uint32_t b = t - list[i].first;
        const uint32_t nb = (sd.g.vh + PBLOCK - 1) / PBLOCK;
        const int parity = (int)(b / nb);
        const uint32_t h = (b % nb) * PBLOCK + threadIdx.x;
        double th = 0.0, fr = 0.0;
        if constexpr (M8) {
            if (h < sd.g.vh) measure_site(field8_of(sd), sd.g, parity, h, th, fr);
        } else {
            if (h < sd.g.vh) measure_site(field_of<R>(sd), sd.g, parity, h, th, fr);
        }
        block_sum2<PBLOCK>(th, fr, sd.partial + 2 * (size_t)b);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(PBLOCK) k_pool_finalize(const SlotDev* __restrict__ slots,
                                                          const Entry* __restrict__ list,
                                                          const uint32_t* __restrict__ count)
{
    const uint32_t n = *count;
    for (uint32_t t = blockIdx.x; t < n; t += gridDim.x) {
        const SlotDev sd = slots[list[t].slot];
        const uint32_t nb = (sd.g.vh + PBLOCK - 1) / PBLOCK;
        finalize_pairs<PBLOCK>(sd.partial, 2 * nb, sd.scale_theta, sd.scale_F, sd.result);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host --

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum JobState { J_ANNEAL = 0, J_FIX = 1, J_DONE = 2 };

struct Job {
    uint64_t id = 0;
    gf_lattice lat = nullptr;
    int slot = -1;
    JobState state = J_FIX;
    gf_fix_params p{};
    int32_t anneal_total = 0, anneal_done = 0;
    double T0 = 1.0, T1 = 1.0;
    uint64_t seed = 0;
    gf_fix_result res{};
    double theta = 0.0, F = 0.0, best = 0.0;
    double theta_switch = 0.0;  // resolved switch point (p.theta_switch < 0: chosen for the lattice)
    int stall = 0;
    gf_status status = GF_OK;
    double t_admit = 0.0, t_done = 0.0;
    bool polled = false;
    int64_t bytes = 0;
    // plan of the current step
    int plan_kind = -1, plan_n = 0, plan_measure_k = -1;
};

}  // namespace pool
}  // namespace gf

using namespace gf;
using namespace gf::pool;
using namespace gf::detail;

// A captured step: the graph (kept for its node handles) and, for every sweep
// launch, its node, its captured parameters and its (k, kind) segment.
struct StepGraph {
    struct SweepNode {
        hipGraphNode_t node;
        hipKernelNodeParams params;
        size_t seg;
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<SweepNode> sweeps;
};

void destroy_step_graph(StepGraph& g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
    g.sweeps.clear();
}

struct gf_pool_ {
    gf_pool_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int chunk = 1;
    std::vector<Job> jobs;           // indexed by slot (slot == index); id 0 with lat == nullptr = free
    std::vector<SlotDev> slot_host;  // mirror of the device slot table
    int64_t bytes_in_use = 0;
    // device buffers
    SlotDev* slots_dev = nullptr;
    Entry* lists_dev = nullptr;
    uint32_t* counts_dev = nullptr;
    double* results_dev = nullptr;
    // pinned host staging
    SlotDev* slots_pin = nullptr;
    Entry* lists_pin = nullptr;
    uint32_t* counts_pin = nullptr;
    double* results_pin = nullptr;
    size_t list_stride = 0;  // entries per (k, kind) segment = max_slots + 1
    std::map<std::string, StepGraph> graphs;
    std::vector<gf_pool_done> finished;  // not yet polled
    std::vector<uint32_t> seg_tiles;     // tiles per (k, kind) list of the step being launched
    std::vector<size_t> launch_log;      // (k, kind) segment of every launch while capturing
    int grid_other = 0;                  // persistent grid of the reunitarisation / measurement kernels
    // transfers of admitted / fetched jobs, beside a step in flight
    hipStream_t xfer = nullptr;
    double* stage = nullptr;  // kStageLinks canonical links
    bool in_flight = false;   // a launched step has not been completed
    std::vector<std::pair<gf_lattice, int64_t>> deferred;  // released while a step ran: freed at its completion
};

namespace {

gf_status pool_check(gf_pool P)
{
    if (!P) return fail(GF_E_ARG, "null pool");
    return GF_OK;
}

gf_status check_pool_shape(int tps, int block)
{
    if ((tps != 1 && tps != 2 && tps != 4) || (block != 64 && block != 128 && block != 256))
        return fail(GF_E_ARG, "pool sweep shape tps=%d block=%d: tps must be 1, 2 or 4 and block 64, 128 or 256",
                    tps, block);
    return GF_OK;
}

// Device bytes of a job's lattice: what gf_create_lattice allocates for it.
int64_t lattice_bytes(const int32_t dims[4], int32_t prec, bool min8)
{
    Geom g{};
    if (!make_geom(dims, &g)) return -1;
    return lattice_sizes(g, (gf_prec)prec, 3, min8).total;
}

Entry* seg(gf_pool P, Entry* base, int k, int kind)
{
    return base + ((size_t)k * NKIND + kind) * P->list_stride;
}

uint32_t tiles_of(const Geom& g, int kind, int tps, int block)
{
    switch (kind) {
        case K_HB32:
        case K_OR32:
        case K_OR64:
        case K_HB64: {
            const uint32_t spb = (uint32_t)block / (uint32_t)tps;
            return (g.vh + spb - 1) / spb;
        }
        case K_R32:
        case K_R64: return (g.vh + PBLOCK - 1) / PBLOCK;
        case K_M32:
        case K_M64: return 2 * ((g.vh + PBLOCK - 1) / PBLOCK);
        default: return 1;
    }
}

template <typename R, int TPS, int MODE, bool TRACKG, bool M8, int CP>
hipError_t launch_sweep_tps(hipStream_t st, const SlotDev* slots, int block, uint32_t tiles, const Entry* list,
                            const uint32_t* count, uint32_t stride, int parity, uint32_t k)
{
    const dim3 grid(tiles);
    switch (block) {
        case 64:
            hipLaunchKernelGGL((k_pool_sweep<R, TPS, MODE, TRACKG, 64, M8, CP>), grid, dim3(64), 0, st, slots, list,
                               count, stride, parity, k);
            break;
        case 256:
            hipLaunchKernelGGL((k_pool_sweep<R, TPS, MODE, TRACKG, 256, M8, CP>), grid, dim3(256), 0, st, slots, list,
                               count, stride, parity, k);
            break;
        default:
            hipLaunchKernelGGL((k_pool_sweep<R, TPS, MODE, TRACKG, 128, M8, CP>), grid, dim3(128), 0, st, slots, list,
                               count, stride, parity, k);
            break;
    }
    return hipGetLastError();
}

template <typename R, int MODE, bool TRACKG, bool M8, int CP>
hipError_t launch_sweep_shape_cp(hipStream_t st, const SlotDev* slots, int tps, int block, uint32_t tiles,
                                 const Entry* list, const uint32_t* count, uint32_t stride, int parity, uint32_t k)
{
    switch (tps) {
        case 1:
            return launch_sweep_tps<R, 1, MODE, TRACKG, M8, CP>(st, slots, block, tiles, list, count, stride, parity,
                                                                k);
        case 2:
            return launch_sweep_tps<R, 2, MODE, TRACKG, M8, CP>(st, slots, block, tiles, list, count, stride, parity,
                                                                k);
        default:
            return launch_sweep_tps<R, 4, MODE, TRACKG, M8, CP>(st, slots, block, tiles, list, count, stride, parity,
                                                                k);
    }
}

// One sweep launch of kind (R, MODE, TRACKG, M8) over `tiles` tiles of block /
// tps sites (tps 1, 2 or 4; block 64, 128 or 256) with cache policy cp (0
// plain loads and stores, 1 non-temporal; gf_device.h).  The heat-bath kinds
// keep the fixed policy: plain for float32, non-temporal for float64.
template <typename R, int MODE, bool TRACKG, bool M8>
hipError_t launch_sweep_shape(hipStream_t st, const SlotDev* slots, int tps, int block, int cp, uint32_t tiles,
                              const Entry* list, const uint32_t* count, uint32_t stride, int parity, uint32_t k)
{
    if constexpr (MODE == HEATBATH) {
        constexpr int CPH = sizeof(R) == 8 ? 1 : 0;
        return launch_sweep_shape_cp<R, MODE, TRACKG, M8, CPH>(st, slots, tps, block, tiles, list, count, stride,
                                                               parity, k);
    } else {
        return cp == 1 ? launch_sweep_shape_cp<R, MODE, TRACKG, M8, 1>(st, slots, tps, block, tiles, list, count,
                                                                       stride, parity, k)
                       : launch_sweep_shape_cp<R, MODE, TRACKG, M8, 0>(st, slots, tps, block, tiles, list, count,
                                                                       stride, parity, k);
    }
}

// The float32 kinds take the pool's float32 storage (M8: 8 reals per link).
template <typename R, int MODE, bool TRACKG>
hipError_t launch_sweep_kind(gf_pool P, int tps, int block, int cp, uint32_t tiles, const Entry* list,
                             const uint32_t* count, int parity, uint32_t k)
{
    if constexpr (sizeof(R) == 4) {
        if (P->cfg.reals32 == 8)
            return launch_sweep_shape<R, MODE, TRACKG, true>(P->stream, P->slots_dev, tps, block, cp, tiles, list,
                                                             count, (uint32_t)P->list_stride, parity, k);
    }
    return launch_sweep_shape<R, MODE, TRACKG, false>(P->stream, P->slots_dev, tps, block, cp, tiles, list, count,
                                                      (uint32_t)P->list_stride, parity, k);
}

bool is_sweep_kind(int kind)
{
    return kind == K_HB32 || kind == K_OR32 || kind == K_OR64 || kind == K_HB64;
}

hipError_t launch_kind(gf_pool P, int k, int kind, int parity)
{
    const size_t sgi = (size_t)k * NKIND + kind;
    const Entry* list = seg(P, P->lists_dev, k, kind);
    const uint32_t* count = P->counts_dev + sgi;
    const uint32_t tiles = P->seg_tiles[sgi];
    const uint32_t kk = (uint32_t)k;
    const int mode = P->cfg.mode;
    const int t32 = P->cfg.tps32, t64 = P->cfg.tps64, b32 = P->cfg.block32, b64 = P->cfg.block64;
    const int c32 = P->cfg.cache32 - 1, c64 = P->cfg.cache64 - 1;  // kernel cache policy codes
    P->launch_log.push_back(sgi);
    switch (kind) {
        case K_HB32:
            return launch_sweep_kind<float, HEATBATH, true>(P, kHeatBathTps, kHeatBathBlock, 0, tiles, list, count,
                                                            parity, kk);
        case K_HB64:
            return launch_sweep_kind<double, HEATBATH, false>(P, kHeatBathTps, kHeatBathBlock, 1, tiles, list, count,
                                                              parity, kk);
        case K_OR32:
            return mode == GF_OR_EXACT
                       ? launch_sweep_kind<float, 0, true>(P, t32, b32, c32, tiles, list, count, parity, kk)
                       : launch_sweep_kind<float, 1, true>(P, t32, b32, c32, tiles, list, count, parity, kk);
        case K_OR64:
            return mode == GF_OR_EXACT
                       ? launch_sweep_kind<double, 0, false>(P, t64, b64, c64, tiles, list, count, parity, kk)
                       : launch_sweep_kind<double, 1, false>(P, t64, b64, c64, tiles, list, count, parity, kk);
        case K_R32:
            if (P->cfg.reals32 == 8)
                hipLaunchKernelGGL((k_pool_reunit<float, true, true>), dim3(P->grid_other), dim3(PBLOCK), 0, P->stream,
                                   P->slots_dev, list, count);
            else
                hipLaunchKernelGGL((k_pool_reunit<float, true, false>), dim3(P->grid_other), dim3(PBLOCK), 0,
                                   P->stream, P->slots_dev, list, count);
            break;
        case K_R64:
            hipLaunchKernelGGL((k_pool_reunit<double, false, false>), dim3(P->grid_other), dim3(PBLOCK), 0, P->stream,
                               P->slots_dev, list, count);
            break;
        case K_M32:
            if (P->cfg.reals32 == 8)
                hipLaunchKernelGGL((k_pool_measure<float, true>), dim3(P->grid_other), dim3(PBLOCK), 0, P->stream,
                                   P->slots_dev, list, count);
            else
                hipLaunchKernelGGL((k_pool_measure<float, false>), dim3(P->grid_other), dim3(PBLOCK), 0, P->stream,
                                   P->slots_dev, list, count);
            break;
        case K_M64:
            hipLaunchKernelGGL((k_pool_measure<double, false>), dim3(P->grid_other), dim3(PBLOCK), 0, P->stream,
                               P->slots_dev, list, count);
            break;
        default:
            hipLaunchKernelGGL(k_pool_finalize, dim3(P->grid_other), dim3(PBLOCK), 0, P->stream, P->slots_dev, list,
                               count);
            break;
    }
    return hipGetLastError();
}

// Enqueue the whole step for the work structure `sig` (one char per (k, kind)).
gf_status enqueue_step(gf_pool P, const std::string& sig)
{
    static const int sweep_kinds[4] = {K_HB32, K_OR32, K_OR64, K_HB64};
    for (int k = 0; k < P->chunk; ++k) {
        const char* row = sig.c_str() + (size_t)k * NKIND;
        for (int parity = 0; parity < 2; ++parity)
            for (int kind : sweep_kinds)
                if (row[kind] == '1') GF_HIP(launch_kind(P, k, kind, parity));
        for (int kind : {K_R32, K_R64, K_M32, K_M64, K_FIN})
            if (row[kind] == '1') GF_HIP(launch_kind(P, k, kind, 0));
    }
    return GF_OK;
}

// Capture the step for `sig` (launches in the order enqueue_step issues them)
// and record the node of every sweep launch: a stream capture is a chain, so
// the nodes are walked from the root along their single dependents.
gf_status capture_step(gf_pool P, const std::string& sig, StepGraph& out)
{
    P->launch_log.clear();
    GF_HIP(hipStreamBeginCapture(P->stream, hipStreamCaptureModeRelaxed));
    gf_status st = enqueue_step(P, sig);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(P->stream, &graph);
    if (st != GF_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(GF_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    out.graph = graph;
    const size_t n = P->launch_log.size();
    std::vector<hipGraphNode_t> chain;
    size_t cnt = 0;
    hipGraphNode_t node = nullptr;
    e = hipGraphGetRootNodes(graph, nullptr, &cnt);
    if (e == hipSuccess && cnt == 1) e = hipGraphGetRootNodes(graph, &node, &cnt);
    while (e == hipSuccess && cnt == 1 && chain.size() <= n) {
        chain.push_back(node);
        cnt = 0;
        e = hipGraphNodeGetDependentNodes(node, nullptr, &cnt);
        if (e != hipSuccess || cnt != 1) break;
        e = hipGraphNodeGetDependentNodes(node, &node, &cnt);
    }
    if (e != hipSuccess || chain.size() != n) {
        destroy_step_graph(out);
        return fail(GF_E_HIP, "captured step is not a chain of %zu launches (%zu nodes)", n, chain.size());
    }
    for (size_t i = 0; i < n; ++i) {
        const size_t sgi = P->launch_log[i];
        if (!is_sweep_kind((int)(sgi % NKIND))) continue;
        StepGraph::SweepNode sn{chain[i], {}, sgi};
        e = hipGraphKernelNodeGetParams(chain[i], &sn.params);
        if (e != hipSuccess) {
            destroy_step_graph(out);
            return fail(GF_E_HIP, "hipGraphKernelNodeGetParams: %s", hipGetErrorString(e));
        }
        out.sweeps.push_back(sn);
    }
    e = hipGraphInstantiate(&out.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        destroy_step_graph(out);
        return fail(GF_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return GF_OK;
}

gf_status run_graph(gf_pool P, const std::string& sig)
{
    auto it = P->graphs.find(sig);
    if (it == P->graphs.end()) {
        if (P->graphs.size() >= 64) {
            for (auto& kv : P->graphs) destroy_step_graph(kv.second);
            P->graphs.clear();
        }
        StepGraph g;
        GF_TRY(capture_step(P, sig, g));
        it = P->graphs.emplace(sig, g).first;
    } else {
        // one block per tile of this step's lists
        for (auto& sn : it->second.sweeps) {
            const uint32_t tiles = P->seg_tiles[sn.seg];
            if (sn.params.gridDim.x == tiles) continue;
            sn.params.gridDim = dim3(tiles);
            GF_HIP(hipGraphExecKernelNodeSetParams(it->second.exec, sn.node, &sn.params));
        }
    }
    GF_HIP(hipGraphLaunch(it->second.exec, P->stream));
    return GF_OK;
}

void fill_slot(gf_pool P, int slot)
{
    Job& j = P->jobs[slot];
    gf_lattice L = j.lat;
    SlotDev& d = P->slot_host[slot];
    std::memset(&d, 0, sizeof d);
    d.f64 = LinkField<double>{L->f64, L->geom.ld};
    d.f32 = LinkField<float>{L->f32, L->geom.ld};
    d.gacc = L->gacc;
    d.g = L->geom;
    d.omega = j.p.omega;
    d.T0 = j.T0;
    d.T1 = j.T1;
    d.n_anneal = j.anneal_total;
    d.key0 = (uint32_t)j.seed;
    d.key1 = (uint32_t)(j.seed >> 32);
    d.anneal_base = L->anneal_sweeps;
    const double V = 2.0 * (double)L->geom.vh;
    d.scale_theta = 1.0 / (3.0 * V);
    d.scale_F = 1.0 / (12.0 * V);
    d.partial = L->partial;
    d.result = P->results_dev + 2 * (size_t)slot;
}

void finish(gf_pool P, Job& j, gf_status status)
{
    j.state = J_DONE;
    j.status = status;
    j.t_done = now_s();
    j.res.converged = j.theta < j.p.theta_target && status == GF_OK;
    j.res.theta = j.theta;
    j.res.F = j.F;
    gf_pool_done d{};
    d.job_id = j.id;
    d.result = j.res;
    d.status = status;
    d.t_admit = j.t_admit;
    d.t_done = j.t_done;
    P->finished.push_back(d);
}

// The loop head of gf_fix_until for a job in the fix phase: finish, or promote
// and measure again, until the job needs sweeps.
// The loop head of gf_fix_until for a job in the fix phase: promote a GF_MIXED
// job at its switch point (or when it would end), finish it when done.
gf_status fix_head(gf_pool P, Job& j)
{
    gf_lattice L = j.lat;
    for (;;) {
        const bool finished = !(j.theta >= j.p.theta_target && j.res.sweeps < j.p.max_sweeps);
        const bool in_fp32 = L->prec == GF_MIXED && L->phase == 0;
        if (in_fp32 && (finished || leave_fp32(j.theta, j.theta_switch, j.best, j.stall))) {
            GF_TRY(do_promote(L));
            gf_status st = do_measure(L, &j.theta, &j.F);
            if (st != GF_OK) {
                finish(P, j, st);
                return GF_OK;
            }
            continue;
        }
        if (finished) finish(P, j, GF_OK);
        return GF_OK;
    }
}

// Entering the fix phase (at admission, or after the anneal): the measured
// theta starts the stall record and the switch point is resolved, as at the
// start of gf_fix_until.
void enter_fix(gf_pool P, Job& j)
{
    j.state = J_FIX;
    j.best = j.theta;
    j.stall = 0;
    const gf_status st = resolve_switch(j.lat, j.p.theta_target, j.p.theta_switch, &j.theta_switch);
    if (st != GF_OK) finish(P, j, st);
}

// A finished job's lattice is not used by a step in flight, but freeing device
// memory synchronises the device: while a step runs, the lattice waits (its
// bytes still counted) until the step is completed.
void release_job(gf_pool P, Job& j)
{
    if (j.lat && P->in_flight) {
        P->deferred.emplace_back(j.lat, j.bytes);
    } else if (j.lat) {
        (void)gf_destroy_lattice(j.lat);
        P->bytes_in_use -= j.bytes;
    }
    j = Job();
}

void free_deferred(gf_pool P)
{
    for (auto& d : P->deferred) {
        (void)gf_destroy_lattice(d.first);
        P->bytes_in_use -= d.second;
    }
    P->deferred.clear();
}

// A job's canonical links in from host memory, chunk by chunk through the
// staging buffer, on the transfer stream; returns once the host buffer has been
// read and the lattice is packed.
gf_status upload_job(gf_pool P, gf_lattice L, const double* host)
{
    const uint64_t nlinks = (uint64_t)L->volume * 4;
    hipError_t e = hipSuccess;
    for (uint64_t first = 0; first < nlinks && e == hipSuccess; first += kStageLinks) {
        const uint64_t n = std::min<uint64_t>(kStageLinks, nlinks - first);
        e = hipMemcpyAsync(P->stage, host + first * 18, n * 18 * sizeof(double), hipMemcpyHostToDevice, P->xfer);
        if (e == hipSuccess && L->f32 && L->min8)
            e = gf::launch_pack_range(P->stage, field8f(L), L->geom, first, n, P->xfer);
        else if (e == hipSuccess && L->f32)
            e = gf::launch_pack_range(P->stage, field32(L), L->geom, first, n, P->xfer);
        if (e == hipSuccess && L->f64) e = gf::launch_pack_range(P->stage, field64(L), L->geom, first, n, P->xfer);
    }
    if (e == hipSuccess && L->gacc.base) e = gf::launch_g_identity(L->gacc, L->geom, P->xfer);
    const hipError_t es = hipStreamSynchronize(P->xfer);  // also after a failed enqueue: nothing stays queued
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return fail(GF_E_HIP, "admission upload: %s", hipGetErrorString(e));
    L->phase = 0;
    L->has_links = true;
    L->anneal_sweeps = 0;
    return GF_OK;
}

// A finished job's links out to host memory the same way (the field its
// result is in: float64 once promoted).
gf_status download_job(gf_pool P, gf_lattice L, double* host)
{
    const uint64_t nlinks = (uint64_t)L->volume * 4;
    hipError_t e = hipSuccess;
    for (uint64_t first = 0; first < nlinks && e == hipSuccess; first += kStageLinks) {
        const uint64_t n = std::min<uint64_t>(kStageLinks, nlinks - first);
        if (is_fp32(L) && L->min8)
            e = gf::launch_unpack_range(field8f(L), L->geom, P->stage, first, n, P->xfer);
        else if (is_fp32(L))
            e = gf::launch_unpack_range(field32(L), L->geom, P->stage, first, n, P->xfer);
        else
            e = gf::launch_unpack_range(field64(L), L->geom, P->stage, first, n, P->xfer);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host + first * 18, P->stage, n * 18 * sizeof(double), hipMemcpyDeviceToHost, P->xfer);
    }
    const hipError_t es = hipStreamSynchronize(P->xfer);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return fail(GF_E_HIP, "fetch: %s", hipGetErrorString(e));
    return GF_OK;
}

// Loop heads of the jobs in the fix phase, then the plan of the next step:
// work lists, slot table, the graph launch and the copy of the results, all
// enqueued; the step is in flight until complete_step.
gf_status launch_step(gf_pool P)
{
    const int C = P->chunk;
    // loop heads (finish / promote) of jobs in the fix phase
    for (auto& j : P->jobs)
        if (j.lat && j.state == J_FIX) GF_TRY(fix_head(P, j));

    // plan the step
    const size_t nseg = (size_t)C * NKIND;
    std::vector<uint32_t> n_entries(nseg, 0), n_tiles(nseg, 0);
    auto add = [&](int k, int kind, int slot, const Geom& g) {
        const size_t sgi = (size_t)k * NKIND + kind;
        Entry* e = seg(P, P->lists_pin, k, kind);
        e[n_entries[sgi]] = Entry{(uint32_t)slot, n_tiles[sgi]};
        n_entries[sgi]++;
        const int tps = kind == K_OR32 ? P->cfg.tps32 : kind == K_OR64 ? P->cfg.tps64 : kHeatBathTps;
        const int blk = kind == K_OR32 ? P->cfg.block32 : kind == K_OR64 ? P->cfg.block64 : kHeatBathBlock;
        n_tiles[sgi] += tiles_of(g, kind, tps, blk);
    };
    bool any = false;
    for (auto& j : P->jobs) {
        j.plan_kind = -1;
        j.plan_n = 0;
        j.plan_measure_k = -1;
        if (!j.lat || j.state == J_DONE) continue;
        gf_lattice L = j.lat;
        const bool fp32 = is_fp32(L);
        if (j.state == J_ANNEAL) {
            const int a = std::min(j.anneal_total - j.anneal_done, C);
            const int kind = fp32 ? K_HB32 : K_HB64;
            for (int k = 0; k < a; ++k) add(k, kind, j.slot, L->geom);
            j.plan_kind = kind;
            j.plan_n = a;
            if (j.anneal_done + a == j.anneal_total) j.plan_measure_k = a - 1;
        } else {
            const int n = std::min(j.p.check_every, j.p.max_sweeps - j.res.sweeps);
            const int kind = fp32 ? K_OR32 : K_OR64;
            for (int k = 0; k < n; ++k) {
                add(k, kind, j.slot, L->geom);
                const int32_t done = j.res.sweeps + k + 1;
                if (j.p.reunit_every > 0 && done % j.p.reunit_every == 0) add(k, fp32 ? K_R32 : K_R64, j.slot, L->geom);
            }
            j.plan_kind = kind;
            j.plan_n = n;
            j.plan_measure_k = n - 1;
        }
        if (j.plan_measure_k >= 0) {
            add(j.plan_measure_k, fp32 ? K_M32 : K_M64, j.slot, L->geom);
            add(j.plan_measure_k, K_FIN, j.slot, L->geom);
        }
        any = any || j.plan_n > 0;
    }
    if (!any) return GF_OK;

    std::string sig(nseg, '0');
    for (size_t i = 0; i < nseg; ++i) {
        const int k = (int)(i / NKIND), kind = (int)(i % NKIND);
        seg(P, P->lists_pin, k, kind)[n_entries[i]] = Entry{0u, n_tiles[i]};  // sentinel
        P->counts_pin[i] = n_entries[i];
        P->seg_tiles[i] = n_tiles[i];
        if (n_entries[i]) sig[i] = '1';
    }
    for (int s = 0; s < (int)P->jobs.size(); ++s) P->slots_pin[s] = P->slot_host[s];

    GF_HIP(hipMemcpyAsync(P->slots_dev, P->slots_pin, sizeof(SlotDev) * P->jobs.size(), hipMemcpyHostToDevice,
                          P->stream));
    GF_HIP(hipMemcpyAsync(P->lists_dev, P->lists_pin, sizeof(Entry) * nseg * P->list_stride, hipMemcpyHostToDevice,
                          P->stream));
    GF_HIP(hipMemcpyAsync(P->counts_dev, P->counts_pin, sizeof(uint32_t) * nseg, hipMemcpyHostToDevice, P->stream));
    GF_TRY(run_graph(P, sig));
    GF_HIP(hipMemcpyAsync(P->results_pin, P->results_dev, sizeof(double) * 2 * P->jobs.size(), hipMemcpyDeviceToHost,
                          P->stream));
    P->in_flight = true;
    return GF_OK;
}

// Wait for the step in flight (if any), free what was released meanwhile, and
// apply the step's outcome to its jobs.
gf_status complete_step(gf_pool P)
{
    if (!P->in_flight) return GF_OK;
    P->in_flight = false;
    GF_HIP(hipStreamSynchronize(P->stream));
    free_deferred(P);
    for (auto& j : P->jobs) {
        if (!j.lat || j.state == J_DONE || j.plan_n == 0) continue;
        gf_lattice L = j.lat;
        if (j.state == J_ANNEAL) {
            j.anneal_done += j.plan_n;
            L->anneal_sweeps += (uint32_t)j.plan_n;
            P->slot_host[j.slot].anneal_base = L->anneal_sweeps;
            if (j.plan_measure_k >= 0) {
                j.theta = P->results_pin[2 * j.slot];
                j.F = P->results_pin[2 * j.slot + 1];
                if (std::isfinite(j.theta) && std::isfinite(j.F)) enter_fix(P, j);
            }
        } else {
            j.res.sweeps += j.plan_n;
            if (j.plan_kind == K_OR32)
                j.res.sweeps_fp32 += j.plan_n;
            else
                j.res.sweeps_fp64 += j.plan_n;
            j.theta = P->results_pin[2 * j.slot];
            j.F = P->results_pin[2 * j.slot + 1];
            update_stall(j.theta, &j.best, &j.stall);
        }
        if (j.plan_measure_k >= 0 && (!std::isfinite(j.theta) || !std::isfinite(j.F))) {
            finish(P, j, GF_E_NUMERIC);
            continue;
        }
        if (j.state == J_FIX) GF_TRY(fix_head(P, j));
    }
    return GF_OK;
}

}  // namespace

extern "C" {

double gf_clock(void)
{
    return now_s();
}

gf_status gf_pool_job_bytes(const int32_t dims[4], int32_t prec, int32_t reals32, int64_t* bytes)
{
    if (!dims || !bytes) return fail(GF_E_ARG, "null argument");
    for (int m = 0; m < 4; ++m)
        if (dims[m] < 2 || dims[m] % 2) return fail(GF_E_ARG, "extents must be even and >= 2");
    if (prec != GF_FP64 && prec != GF_MIXED && prec != GF_FP32) return fail(GF_E_ARG, "bad precision");
    if (reals32 != 0 && reals32 != 12 && reals32 != 8) return fail(GF_E_ARG, "reals32 must be 0, 12 or 8");
    if (reals32 == 8 && prec == GF_FP64) return fail(GF_E_ARG, "a GF_FP64 job has no float32 links");
    int64_t V = 1;
    GF_TRY(check_dims(dims, &V));
    *bytes = lattice_bytes(dims, prec, reals32 == 8);
    if (*bytes < 0) return fail(GF_E_ARG, "internal: index division check failed");
    return GF_OK;
}

gf_status gf_pool_create(const gf_pool_config* cfg, void* hip_stream, gf_pool* out)
{
    if (!cfg || !out) return fail(GF_E_ARG, "null argument");
    *out = nullptr;
    if (cfg->max_slots < 1 || cfg->max_slots > 4096) return fail(GF_E_ARG, "max_slots must be 1..4096");
    if (cfg->prec != GF_MIXED && cfg->prec != GF_FP64) return fail(GF_E_ARG, "pool precision must be GF_MIXED or GF_FP64");
    if (cfg->check_every < 1 || cfg->check_every > 1000) return fail(GF_E_ARG, "check_every must be 1..1000");
    if (cfg->mode != GF_OR_EXACT && cfg->mode != GF_OR_BINOMIAL1) return fail(GF_E_ARG, "unknown mode");
    gf_pool_config c = *cfg;
    if (c.reals32 == 0) c.reals32 = 12;
    if (c.reals32 != 12 && c.reals32 != 8) return fail(GF_E_ARG, "reals32 must be 0, 12 or 8");
    if (c.reals32 == 8 && c.prec != GF_MIXED) return fail(GF_E_ARG, "8-real float32 links need a GF_MIXED pool");
    if (c.tps32 == 0) c.tps32 = c.reals32 == 8 ? kDefaultTps32Min8 : kDefaultTps32;
    if (c.tps64 == 0) c.tps64 = kDefaultTps64;
    if (c.block32 == 0) c.block32 = kDefaultBlock;
    if (c.block64 == 0) c.block64 = kDefaultBlock;
    if (c.cache32 == 0) c.cache32 = c.reals32 == 8 ? 2 : 1;  // 8 reals: non-temporal; 12: plain
    if (c.cache64 == 0) c.cache64 = 2;  // non-temporal
    GF_TRY(check_pool_shape(c.tps32, c.block32));
    GF_TRY(check_pool_shape(c.tps64, c.block64));
    if (c.cache32 < 1 || c.cache32 > 2 || c.cache64 < 1 || c.cache64 > 2)
        return fail(GF_E_ARG, "cache32 / cache64 must be 0 (default), 1 (plain) or 2 (non-temporal)");

    gf_pool_* P = new (std::nothrow) gf_pool_();
    if (!P) return fail(GF_E_NOMEM, "host allocation failed");
    P->cfg = c;
    P->chunk = c.check_every;
    if (hip_stream) {
        P->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete P;
            return fail(GF_E_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        P->own_stream = true;
    }
    P->jobs.resize(c.max_slots);
    P->slot_host.resize(c.max_slots);
    P->list_stride = (size_t)c.max_slots + 1;
    const size_t nseg = (size_t)P->chunk * NKIND;
    hipError_t e = hipMalloc((void**)&P->slots_dev, sizeof(SlotDev) * c.max_slots);
    if (e == hipSuccess) e = hipMalloc((void**)&P->lists_dev, sizeof(Entry) * nseg * P->list_stride);
    if (e == hipSuccess) e = hipMalloc((void**)&P->counts_dev, sizeof(uint32_t) * nseg);
    if (e == hipSuccess) e = hipMalloc((void**)&P->results_dev, sizeof(double) * 2 * c.max_slots);
    if (e == hipSuccess) e = hipHostMalloc((void**)&P->slots_pin, sizeof(SlotDev) * c.max_slots, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&P->lists_pin, sizeof(Entry) * nseg * P->list_stride, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&P->counts_pin, sizeof(uint32_t) * nseg, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&P->results_pin, sizeof(double) * 2 * c.max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&P->stage, kStageLinks * 18 * sizeof(double));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->xfer, hipStreamNonBlocking);
    int dev = 0, ncu = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        gf_pool_destroy(P);
        return fail(GF_E_HIP, "pool allocation failed: %s", hipGetErrorString(e));
    }
    // persistent grid of the reunitarisation / measurement kernels: a few resident blocks per compute unit
    P->grid_other = 4 * ncu;
    P->seg_tiles.assign(nseg, 0);
    std::memset(P->slots_pin, 0, sizeof(SlotDev) * c.max_slots);
    *out = P;
    return GF_OK;
}

gf_status gf_pool_destroy(gf_pool P)
{
    if (!P) return GF_OK;
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    if (P->xfer) (void)hipStreamSynchronize(P->xfer);
    P->in_flight = false;
    free_deferred(P);
    for (auto& j : P->jobs) release_job(P, j);
    for (auto& kv : P->graphs) destroy_step_graph(kv.second);
    if (P->slots_dev) (void)hipFree(P->slots_dev);
    if (P->lists_dev) (void)hipFree(P->lists_dev);
    if (P->counts_dev) (void)hipFree(P->counts_dev);
    if (P->results_dev) (void)hipFree(P->results_dev);
    if (P->slots_pin) (void)hipHostFree(P->slots_pin);
    if (P->lists_pin) (void)hipHostFree(P->lists_pin);
    if (P->counts_pin) (void)hipHostFree(P->counts_pin);
    if (P->results_pin) (void)hipHostFree(P->results_pin);
    if (P->stage) (void)hipFree(P->stage);
    if (P->xfer) (void)hipStreamDestroy(P->xfer);
    if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
    delete P;
    return GF_OK;
}

gf_status gf_pool_admit(gf_pool P, uint64_t job_id, const int32_t dims[4], const double* host_links,
                        const gf_fix_params* params, int32_t anneal_sweeps, double T_start, double T_end,
                        uint64_t seed)
{
    GF_TRY(pool_check(P));
    if (!dims || !host_links || !params) return fail(GF_E_ARG, "null argument");
    GF_TRY(check_omega(params->omega, params->mode));
    if (params->mode != P->cfg.mode) return fail(GF_E_ARG, "job mode %d differs from the pool's %d", params->mode,
                                                 P->cfg.mode);
    if (params->check_every != P->cfg.check_every)
        return fail(GF_E_ARG, "job check_every %d differs from the pool's %d", params->check_every, P->cfg.check_every);
    if (params->max_sweeps < 0 || params->reunit_every < 0 || !(params->theta_target >= 0.0) ||
        std::isnan(params->theta_switch))
        return fail(GF_E_ARG, "bad fix parameters");
    if (anneal_sweeps < 0) return fail(GF_E_ARG, "anneal_sweeps < 0");
    if (anneal_sweeps > 0 && (!(T_end > 0.0) || !(T_start >= T_end) || !std::isfinite(T_start)))
        return fail(GF_E_ARG, "need T_start >= T_end > 0");
    for (auto& j : P->jobs)
        if (j.lat && j.id == job_id) return fail(GF_E_ARG, "job id %llu is already in the pool", (unsigned long long)job_id);
    int64_t bytes = 0;
    GF_TRY(gf_pool_job_bytes(dims, P->cfg.prec, P->cfg.reals32, &bytes));
    int slot = -1;
    for (int s = 0; s < (int)P->jobs.size(); ++s)
        if (!P->jobs[s].lat) {
            slot = s;
            break;
        }
    if (slot < 0) return fail(GF_E_FULL, "all %d slots are taken", P->cfg.max_slots);
    if ((size_t)(P->bytes_in_use + bytes) > P->cfg.hbm_budget)
        return fail(GF_E_FULL, "job needs %lld bytes, %lld of %zu in use", (long long)bytes,
                    (long long)P->bytes_in_use, P->cfg.hbm_budget);

    gf_lattice L = nullptr;
    GF_TRY(create_lattice(dims, (gf_prec)P->cfg.prec, 3, P->cfg.reals32 == 8, P->stream, &L));
    // the job's own lattice object takes the pool's shape (its solo kernels
    // are not used for sweeps while it is in the pool)
    L->cfg32 = SweepConfig{P->cfg.tps32, P->cfg.block32, P->cfg.cache32 - 1};
    L->cfg64 = SweepConfig{P->cfg.tps64, P->cfg.block64, P->cfg.cache64 - 1};
    gf_status st = upload_job(P, L, host_links);
    double theta = 0.0, F = 0.0;
    if (st == GF_OK && anneal_sweeps == 0) {
        // the first measurement of gf_fix_until, beside a step in flight
        ++L->n_measures;
        st = measure_enqueue(L, P->xfer);
        const hipError_t e = hipStreamSynchronize(P->xfer);
        if (st == GF_OK && e != hipSuccess) st = fail(GF_E_HIP, "admission measurement: %s", hipGetErrorString(e));
        if (st == GF_OK) {
            st = measure_read(L, &theta, &F);
            if (st == GF_E_NUMERIC) st = GF_OK;  // admitted: the job finishes with GF_E_NUMERIC below
        }
    }
    if (st != GF_OK) {
        if (P->in_flight)
            P->deferred.emplace_back(L, 0);
        else
            gf_destroy_lattice(L);
        return st;
    }
    Job& j = P->jobs[slot];
    j = Job();
    j.id = job_id;
    j.lat = L;
    j.slot = slot;
    j.p = *params;
    j.anneal_total = anneal_sweeps;
    j.T0 = T_start;
    j.T1 = T_end;
    j.seed = seed;
    j.t_admit = now_s();
    j.bytes = L->bytes;
    P->bytes_in_use += j.bytes;
    if (anneal_sweeps > 0) {
        j.state = J_ANNEAL;
    } else {
        j.state = J_FIX;
        j.theta = theta;
        j.F = F;
        if (!std::isfinite(theta) || !std::isfinite(F))
            finish(P, j, GF_E_NUMERIC);
        else
            enter_fix(P, j);
    }
    fill_slot(P, slot);
    return GF_OK;
}

gf_status gf_pool_step(gf_pool P)
{
    TraceRange range("gf_pool_step");
    GF_TRY(pool_check(P));
    GF_TRY(complete_step(P));
    GF_TRY(launch_step(P));
    return complete_step(P);
}

gf_status gf_pool_step_async(gf_pool P)
{
    TraceRange range("gf_pool_step_async");
    GF_TRY(pool_check(P));
    GF_TRY(complete_step(P));
    return launch_step(P);
}

gf_status gf_pool_sync(gf_pool P)
{
    GF_TRY(pool_check(P));
    return complete_step(P);
}

gf_status gf_pool_poll(gf_pool P, gf_pool_done* out, int32_t cap, int32_t* n)
{
    GF_TRY(pool_check(P));
    if (!n || (cap > 0 && !out) || cap < 0) return fail(GF_E_ARG, "bad arguments");
    const int32_t m = std::min<int32_t>(cap, (int32_t)P->finished.size());
    for (int32_t i = 0; i < m; ++i) out[i] = P->finished[i];
    P->finished.erase(P->finished.begin(), P->finished.begin() + m);
    *n = m;
    return GF_OK;
}

gf_status gf_pool_fetch_links(gf_pool P, uint64_t job_id, double* host)
{
    GF_TRY(pool_check(P));
    if (!host) return fail(GF_E_ARG, "null argument");
    for (auto& j : P->jobs)
        if (j.lat && j.id == job_id) {
            if (j.state != J_DONE) return fail(GF_E_STATE, "job %llu has not finished", (unsigned long long)job_id);
            GF_TRY(check_ready(j.lat));
            GF_TRY(download_job(P, j.lat, host));
            release_job(P, j);
            return GF_OK;
        }
    return fail(GF_E_ARG, "no job %llu in the pool", (unsigned long long)job_id);
}

gf_status gf_pool_release(gf_pool P, uint64_t job_id)
{
    GF_TRY(pool_check(P));
    for (auto& j : P->jobs)
        if (j.lat && j.id == job_id) {
            if (j.state != J_DONE) return fail(GF_E_STATE, "job %llu has not finished", (unsigned long long)job_id);
            release_job(P, j);
            return GF_OK;
        }
    return fail(GF_E_ARG, "no job %llu in the pool", (unsigned long long)job_id);
}

gf_status gf_pool_cancel(gf_pool P, uint64_t job_id)
{
    GF_TRY(pool_check(P));
    GF_TRY(complete_step(P));  // the job may be in the step in flight
    for (auto& j : P->jobs)
        if (j.lat && j.id == job_id) {
            if (j.state == J_DONE) return fail(GF_E_STATE, "job %llu has already finished", (unsigned long long)job_id);
            finish(P, j, GF_E_CANCELLED);
            return GF_OK;
        }
    return fail(GF_E_ARG, "no job %llu in the pool", (unsigned long long)job_id);
}

gf_status gf_pool_autotune(gf_pool P, int32_t kernel, int32_t n_sweeps, size_t scratch_bytes, gf_tune_entry* table,
                           int32_t cap, int32_t* n_out, gf_tune_entry* chosen)
{
    TraceRange range("gf_pool_autotune");
    GF_TRY(pool_check(P));
    GF_TRY(complete_step(P));  // it times launches of the resident jobs' fields
    if (kernel != GF_FP32 && kernel != GF_FP64) return fail(GF_E_ARG, "kernel must be GF_FP32 or GF_FP64");
    if (kernel == GF_FP32 && P->cfg.prec != GF_MIXED)
        return fail(GF_E_ARG, "a GF_FP64 pool has no float32 sweeps to tune");
    if (n_sweeps < 1 || cap < 0 || (cap > 0 && !table)) return fail(GF_E_ARG, "bad arguments");
    if (n_out) *n_out = 0;
    const bool f32 = kernel == GF_FP32;

    // scratch copies of the resident jobs' fields, in slot order, up to scratch_bytes
    struct Copy {
        SlotDev sd;
        void* field;
        void* g;
    };
    std::vector<Copy> copies;
    size_t used = 0;
    gf_status st = GF_OK;
    hipError_t e = hipSuccess;
    for (auto& j : P->jobs) {
        if (!j.lat) continue;
        gf_lattice L = j.lat;
        const size_t fb = (size_t)2 * 4 * L->geom.ld * 16 * (f32 ? (P->cfg.reals32 == 8 ? kMin8Chunks32 : 3) : 6);
        const size_t gb = f32 ? (size_t)2 * 3 * L->geom.ld * 16 : 0;
        if (used + fb + gb > scratch_bytes) break;
        Copy c{P->slot_host[j.slot], nullptr, nullptr};
        e = hipMalloc(&c.field, fb);
        if (e == hipSuccess && gb) e = hipMalloc(&c.g, gb);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c.field, f32 ? (void*)L->f32 : (void*)L->f64, fb, hipMemcpyDeviceToDevice, P->stream);
        if (e == hipSuccess && gb) e = hipMemcpyAsync(c.g, L->gacc.base, gb, hipMemcpyDeviceToDevice, P->stream);
        if (f32) {
            c.sd.f32 = LinkField<float>{(float4*)c.field, L->geom.ld};
            c.sd.gacc = GField{(float4*)c.g, L->geom.ld};
        } else {
            c.sd.f64 = LinkField<double>{(double2*)c.field, L->geom.ld};
        }
        copies.push_back(c);
        if (e != hipSuccess) break;
        used += fb + gb;
    }
    if (e == hipSuccess && copies.empty())
        st = fail(GF_E_STATE, "no resident job fits the scratch budget of %zu bytes", scratch_bytes);

    const size_t n = copies.size();
    SlotDev* slots_d = nullptr;
    Entry* list_d = nullptr;
    uint32_t* count_d = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<SlotDev> sd(n);
    std::vector<Entry> list(n + 1);
    for (size_t i = 0; i < n; ++i) sd[i] = copies[i].sd;
    const uint32_t count = (uint32_t)n;
    if (st == GF_OK && e == hipSuccess) e = hipMalloc((void**)&slots_d, sizeof(SlotDev) * n);
    if (st == GF_OK && e == hipSuccess) e = hipMalloc((void**)&list_d, sizeof(Entry) * (n + 1));
    if (st == GF_OK && e == hipSuccess) e = hipMalloc((void**)&count_d, sizeof(uint32_t));
    if (st == GF_OK && e == hipSuccess)
        e = hipMemcpyAsync(slots_d, sd.data(), sizeof(SlotDev) * n, hipMemcpyHostToDevice, P->stream);
    if (st == GF_OK && e == hipSuccess)
        e = hipMemcpyAsync(count_d, &count, sizeof(uint32_t), hipMemcpyHostToDevice, P->stream);
    if (st == GF_OK && e == hipSuccess) e = hipEventCreate(&e0);
    if (st == GF_OK && e == hipSuccess) e = hipEventCreate(&e1);
    if (st == GF_OK && e == hipSuccess) e = hipStreamSynchronize(P->stream);

    const int mode = P->cfg.mode;
    // Two rounds over every shape (lanes per site, block, cache policy), each
    // shape keeping its faster time: a single round favours the shapes timed
    // after the clocks have settled.
    constexpr int kNShapes = 18;
    int shapes[kNShapes][3];
    {
        int q = 0;
        for (int tps : {1, 2, 4})
            for (int block : {64, 128, 256})
                for (int cp : {0, 1}) {
                    shapes[q][0] = tps;
                    shapes[q][1] = block;
                    shapes[q][2] = cp;
                    ++q;
                }
    }
    double shape_us[kNShapes];
    for (double& x : shape_us) x = 1e300;
    for (int round = 0; round < 2; ++round) {
        for (int si = 0; si < kNShapes; ++si) {
            if (st != GF_OK || e != hipSuccess) break;
            const int tps = shapes[si][0], block = shapes[si][1], cp = shapes[si][2];
            uint32_t tiles = 0;
            for (size_t i = 0; i < n; ++i) {
                list[i] = Entry{(uint32_t)i, tiles};
                tiles += tiles_of(sd[i].g, f32 ? K_OR32 : K_OR64, tps, block);
            }
            list[n] = Entry{0u, tiles};
            // ordered before this shape's launches; the previous shape's launches
            // have finished (event synchronised), so list_d and `list` are free
            e = hipMemcpyAsync(list_d, list.data(), sizeof(Entry) * (n + 1), hipMemcpyHostToDevice, P->stream);
            auto sweep = [&]() -> hipError_t {
                for (int parity = 0; parity < 2; ++parity) {
                    hipError_t r;
                    const uint32_t ns = (uint32_t)(n + 1);
                    if (f32 && P->cfg.reals32 == 8)
                        r = mode == GF_OR_EXACT
                                ? launch_sweep_shape<float, 0, true, true>(P->stream, slots_d, tps, block, cp, tiles,
                                                                           list_d, count_d, ns, parity, 0u)
                                : launch_sweep_shape<float, 1, true, true>(P->stream, slots_d, tps, block, cp, tiles,
                                                                           list_d, count_d, ns, parity, 0u);
                    else if (f32)
                        r = mode == GF_OR_EXACT
                                ? launch_sweep_shape<float, 0, true, false>(P->stream, slots_d, tps, block, cp, tiles,
                                                                            list_d, count_d, ns, parity, 0u)
                                : launch_sweep_shape<float, 1, true, false>(P->stream, slots_d, tps, block, cp, tiles,
                                                                            list_d, count_d, ns, parity, 0u);
                    else
                        r = mode == GF_OR_EXACT
                                ? launch_sweep_shape<double, 0, false, false>(P->stream, slots_d, tps, block, cp, tiles,
                                                                              list_d, count_d, ns, parity, 0u)
                                : launch_sweep_shape<double, 1, false, false>(P->stream, slots_d, tps, block, cp, tiles,
                                                                              list_d, count_d, ns, parity, 0u);
                    if (r != hipSuccess) return r;
                }
                return hipSuccess;
            };
            if (e == hipSuccess) e = sweep();  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, P->stream);
            for (int k = 0; k < n_sweeps && e == hipSuccess; ++k) e = sweep();
            if (e == hipSuccess) e = hipEventRecord(e1, P->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            shape_us[si] = std::min(shape_us[si], 1e3 * (double)ms / n_sweeps);
        }
    }
    int best_tps = 0, best_block = 0, best_cp = 0, m = 0;
    double best_us = 1e300;
    for (int si = 0; si < kNShapes && st == GF_OK && e == hipSuccess; ++si) {
        const int tps = shapes[si][0], block = shapes[si][1], cp = shapes[si][2];
        if (m < cap) table[m] = gf_tune_entry{tps, block, cp, 0, shape_us[si]};
        ++m;
        if (shape_us[si] < best_us) {
            best_us = shape_us[si];
            best_tps = tps;
            best_block = block;
            best_cp = cp;
        }
    }
    if (st == GF_OK && e != hipSuccess) st = fail(GF_E_HIP, "pool autotune: %s", hipGetErrorString(e));
    (void)hipStreamSynchronize(P->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (slots_d) (void)hipFree(slots_d);
    if (list_d) (void)hipFree(list_d);
    if (count_d) (void)hipFree(count_d);
    for (auto& c : copies) {
        if (c.field) (void)hipFree(c.field);
        if (c.g) (void)hipFree(c.g);
    }
    if (st != GF_OK) return st;
    if (f32) {
        P->cfg.tps32 = best_tps;
        P->cfg.block32 = best_block;
        P->cfg.cache32 = best_cp + 1;
    } else {
        P->cfg.tps64 = best_tps;
        P->cfg.block64 = best_block;
        P->cfg.cache64 = best_cp + 1;
    }
    // captured steps hold the previous shape's kernels
    for (auto& kv : P->graphs) destroy_step_graph(kv.second);
    P->graphs.clear();
    if (n_out) *n_out = std::min(m, cap);
    if (chosen) *chosen = gf_tune_entry{best_tps, best_block, best_cp, 0, best_us};
    return GF_OK;
}

gf_status gf_pool_get_shape(gf_pool P, int32_t* tps32, int32_t* block32, int32_t* tps64, int32_t* block64)
{
    GF_TRY(pool_check(P));
    if (tps32) *tps32 = P->cfg.tps32;
    if (block32) *block32 = P->cfg.block32;
    if (tps64) *tps64 = P->cfg.tps64;
    if (block64) *block64 = P->cfg.block64;
    return GF_OK;
}

gf_status gf_pool_get_cache(gf_pool P, int32_t* cache32, int32_t* cache64)
{
    GF_TRY(pool_check(P));
    if (cache32) *cache32 = P->cfg.cache32;
    if (cache64) *cache64 = P->cfg.cache64;
    return GF_OK;
}

gf_status gf_pool_stats(gf_pool P, int32_t* active, int32_t* finished, int64_t* bytes_in_use)
{
    GF_TRY(pool_check(P));
    int32_t a = 0, f = 0;
    for (auto& j : P->jobs) {
        if (!j.lat) continue;
        if (j.state == J_DONE)
            ++f;
        else
            ++a;
    }
    if (active) *active = a;
    if (finished) *finished = f;
    if (bytes_in_use) *bytes_in_use = P->bytes_in_use;
    return GF_OK;
}

}  // extern "C"
