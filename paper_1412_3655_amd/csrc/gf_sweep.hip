// gf_sweep.hip -- the checkerboard overrelaxation half-sweep (Sec. 2 of
// arXiv:1412.3655) for gfx950.
//
// One site update: K(x) = sum_mu [U_mu(x) + U_mu(x-mu^)^dag]
// (Eq. localfunctional); for the SU(2) subgroups (0,1), (0,2), (1,2) the
// maximiser of the SU(2)-span projection of the 2x2 block of K is raised to
// the power omega and rotates K and the accumulated G; finally U_mu(x) <-
// G U_mu(x) and U_mu(x-mu^) <- U_mu(x-mu^) G^dag (the gauge transformation
// of Sec. 2 with g(x) = G and g = 1 elsewhere).  The paper recomputes
// nothing between subgroups; rotating K by the subgroup element is the same
// as recomputing it from the rotated links (forward links become S U,
// backward links U S^dag, so K -> S K).
//
// Work split (Sec. 3.2 and 4.2 of the paper use 8 or 4 threads per site):
// TPS lanes of one wavefront share a site, lane r owning the 8/TPS links
// with leaf index r*(8/TPS) .. (r+1)*(8/TPS)-1 in the leaf order
// U_0(x), U_0(x-0^)^dag, U_1(x), U_1(x-1^)^dag, ...  Each lane sums its
// leaves in the fixed pairwise tree ((L0+L1)+(L2+L3))+((L4+L5)+(L6+L7)) and
// the lanes finish the same tree with DPP butterflies (no LDS), so K is
// bitwise the same for every TPS.  The subgroup algebra then runs
// redundantly in every lane of the group, and each lane applies G to the
// links it loaded and stores them.  The loop over sites is over the half
// index of one colour: every link is read once and written once per
// half-sweep (768 B per site update in FP64 with 12-real links).
#include "gf_kernels.h"

namespace gf {

namespace {

constexpr int OR_EXACT = 0;

// The SU(2) element applied for the projected block quaternion a (unnormalised,
// a0 + i(a1 s1 + a2 s2 + a3 s3)): the maximiser b = (a0, -a1, -a2, -a3)/|a|
// raised to the power omega.  EXACT: with phi = atan2(|a_vec|, a0), b^omega =
// (cos(omega phi), -sin(omega phi) a_vec/|a_vec|).  BINOMIAL1: normalise
// (1 - omega) + omega b.  |a| = 0 leaves the subgroup alone.
template <int MODE, typename R>
__device__ __forceinline__ Quat<R> or_element(const Quat<R>& a, R omega)
{
    Quat<R> b;
    if constexpr (MODE == OR_EXACT) {
        const R v2 = fmad(a.b1, a.b1, fmad(a.b2, a.b2, a.b3 * a.b3));
        if (v2 > R(0)) {
            const R v = sqrt(v2);
            const R phi = atan2(v, a.b0);
            R s, c;
            sin_cos(omega * phi, &s, &c);
            const R f = -s / v;
            b.b0 = c;
            b.b1 = f * a.b1;
            b.b2 = f * a.b2;
            b.b3 = f * a.b3;
        } else {
            b.b0 = a.b0 < R(0) ? R(-1) : R(1);
            b.b1 = R(0);
            b.b2 = R(0);
            b.b3 = R(0);
        }
    } else {
        const R n2 = fmad(a.b0, a.b0, fmad(a.b1, a.b1, fmad(a.b2, a.b2, a.b3 * a.b3)));
        if (n2 > R(0)) {
            const R inv = R(1) / sqrt(n2);
            const R t0 = fmad(omega, a.b0 * inv, R(1) - omega);
            const R t1 = -omega * (a.b1 * inv);
            const R t2 = -omega * (a.b2 * inv);
            const R t3 = -omega * (a.b3 * inv);
            const R tn = R(1) / sqrt(fmad(t0, t0, fmad(t1, t1, fmad(t2, t2, t3 * t3))));
            b.b0 = t0 * tn;
            b.b1 = t1 * tn;
            b.b2 = t2 * tn;
            b.b3 = t3 * tn;
        } else {
            b.b0 = R(1);
            b.b1 = R(0);
            b.b2 = R(0);
            b.b3 = R(0);
        }
    }
    return b;
}

// Leaf k of this lane: U (forward, bwd = false) or U^dagger (backward).
// Sum of NL consecutive leaves in the fixed pairwise tree.
template <int NL, typename R>
__device__ __forceinline__ void leaf_tree(const M3<R>* U, const bool* bwd, M3<R>& out)
{
    if constexpr (NL == 1) {
        m_leaf(out, U[0], bwd[0]);
    } else {
        M3<R> right;
        leaf_tree<NL / 2>(U, bwd, out);
        leaf_tree<NL / 2>(U + NL / 2, bwd + NL / 2, right);
        m_add(out, right);
    }
}

template <typename R, int TPS, int MODE, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_or_half_sweep(LinkField<R> f, Geom g, int parity, R omega)
{
    constexpr int NL = 8 / TPS;
    const uint32_t gid = blockIdx.x * (uint32_t)BLOCK + threadIdx.x;
    const uint32_t h = gid / TPS;
    const int r = (int)(gid % TPS);
    // whole groups of TPS lanes leave together, so every DPP partner below is live
    if (h >= g.vh) return;
    const Site s = decode_site(g, parity, h);

    M3<R> U[NL];
    bool bwd[NL];
    int mu_of[NL];
    uint32_t at[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int li = r * NL + k;
        mu_of[k] = li >> 1;
        bwd[k] = (li & 1) != 0;
        at[k] = bwd[k] ? back_h(g, h, s, mu_of[k]) : h;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) load_rows01(f, bwd[k] ? 1 - parity : parity, mu_of[k], at[k], U[k]);
#pragma unroll
    for (int k = 0; k < NL; ++k) rebuild_row2(U[k]);

    M3<R> K;
    leaf_tree<NL>(U, bwd, K);
    if constexpr (TPS >= 2) dpp_accumulate<DPP_XOR1>(K);
    if constexpr (TPS >= 4) dpp_accumulate<DPP_XOR2>(K);
    if constexpr (TPS >= 8) dpp_accumulate<DPP_HALF_MIRROR>(K);

    M3<R> G;
    {
        const Quat<R> b = or_element<MODE>(block_quaternion<0, 1>(K), omega);
        set_embedding<0, 1>(b, G);
        rotate_rows<0, 1>(b, K);
    }
    {
        const Quat<R> b = or_element<MODE>(block_quaternion<0, 2>(K), omega);
        rotate_rows<0, 2>(b, G);
        rotate_rows<0, 2>(b, K);
    }
    {
        const Quat<R> b = or_element<MODE>(block_quaternion<1, 2>(K), omega);
        rotate_rows<1, 2>(b, G);
    }

#pragma unroll
    for (int k = 0; k < NL; ++k) {
        if (bwd[k])
            right_mul_dag_rows01(G, U[k]);
        else
            left_mul_rows01(G, U[k]);
        store_rows01(f, bwd[k] ? 1 - parity : parity, mu_of[k], at[k], U[k]);
    }
}

template <typename R, int TPS, int MODE>
hipError_t launch_tps(const LinkField<R>& f, const Geom& g, int parity, R omega, int block, hipStream_t st)
{
    const uint64_t threads = (uint64_t)g.vh * TPS;
    const uint32_t grid = (uint32_t)((threads + block - 1) / block);
    if (grid == 0) return hipSuccess;
    switch (block) {
        case 64:
            hipLaunchKernelGGL((k_or_half_sweep<R, TPS, MODE, 64>), dim3(grid), dim3(64), 0, st, f, g, parity, omega);
            break;
        case 128:
            hipLaunchKernelGGL((k_or_half_sweep<R, TPS, MODE, 128>), dim3(grid), dim3(128), 0, st, f, g, parity, omega);
            break;
        case 256:
            hipLaunchKernelGGL((k_or_half_sweep<R, TPS, MODE, 256>), dim3(grid), dim3(256), 0, st, f, g, parity, omega);
            break;
        default:
            if constexpr (TPS > 1)
                hipLaunchKernelGGL((k_or_half_sweep<R, TPS, MODE, 512>), dim3(grid), dim3(512), 0, st, f, g, parity,
                                   omega);
            else
                return hipErrorInvalidValue;
            break;
    }
    return hipGetLastError();
}

template <typename R, int MODE>
hipError_t launch_mode(const LinkField<R>& f, const Geom& g, int parity, R omega, const SweepConfig& c, hipStream_t st)
{
    switch (c.tps) {
        case 1: return launch_tps<R, 1, MODE>(f, g, parity, omega, c.block, st);
        case 2: return launch_tps<R, 2, MODE>(f, g, parity, omega, c.block, st);
        case 8: return launch_tps<R, 8, MODE>(f, g, parity, omega, c.block, st);
        default: return launch_tps<R, 4, MODE>(f, g, parity, omega, c.block, st);
    }
}

}  // namespace

bool sweep_config_valid(const SweepConfig& c)
{
    const bool tps_ok = c.tps == 1 || c.tps == 2 || c.tps == 4 || c.tps == 8;
    const bool blk_ok = c.block == 64 || c.block == 128 || c.block == 256 || c.block == 512;
    // one lane per site needs more than the 256 registers a 512-thread block allows
    return tps_ok && blk_ok && !(c.tps == 1 && c.block == 512);
}

hipError_t launch_or_half_sweep(const LinkField<double>& f, const Geom& g, int parity, double omega, int mode,
                                const SweepConfig& cfg, hipStream_t st)
{
    return mode == OR_EXACT ? launch_mode<double, 0>(f, g, parity, omega, cfg, st)
                            : launch_mode<double, 1>(f, g, parity, omega, cfg, st);
}

hipError_t launch_or_half_sweep(const LinkField<float>& f, const Geom& g, int parity, float omega, int mode,
                                const SweepConfig& cfg, hipStream_t st)
{
    return mode == OR_EXACT ? launch_mode<float, 0>(f, g, parity, omega, cfg, st)
                            : launch_mode<float, 1>(f, g, parity, omega, cfg, st);
}

}  // namespace gf
