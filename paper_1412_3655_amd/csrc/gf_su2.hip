// gf_su2.hip -- the gauge group SU(2) on gfx950 (arXiv:1412.3655: the
// abstract lists SU(2) beside SU(3); Sec. 2 gives the maximiser
// g = K^dag / sqrt(det K^dag), exact for SU(2), so a site update needs no
// subgroup iteration; Sec. 4.1 changes the group by the link
// parameterisation alone).
//
// A link is the quaternion (q0, q1, q2, q3) of U = q0 + i (q1 s1 + q2 s2 + q3 s3)
// = [[q0 + i q3, q2 + i q1], [-q2 + i q1, q0 - i q3]]: 4 reals, the minimal
// storage (SU(2) has 3 parameters and the unit norm keeps the representation
// exact under products).  Layout as for SU(3): colour, direction, 64-site
// tiles, 16-byte chunks (float64: 2 chunks (q0, q1), (q2, q3); float32: 1),
// so a site update reads and writes 8 x 32 B = 512 B in float64.
//
// Products: (p o q) = (p0 q0 - p.q, p0 q + q0 p - p x q) is the matrix product
// of the two elements; U^dag = (q0, -q).  K(x) = sum_mu [U_mu(x) +
// U_mu(x-mu^)^dag] is the element of the real span with quaternion c (sum of
// the links' quaternions, the backward ones conjugated); the maximiser is
// (c0, -c)/|c| raised to omega (or_element of the SU(3) subgroups, whose
// quaternion argument is 2c), and the heat bath draws from
// exp(Re tr[g K]/T) with the SU(3) subgroup sampler (kappa = 2|c|/T).
//
// theta = (1/(2V)) sum_x tr[Delta Delta^dag] with Delta = [(K - K^dag)/(2i)]
// = c.s, so tr[Delta Delta^dag] = 2|c|^2; F = (1/(8V)) sum_x sum_mu 2 q0.
// Coulomb gauge: K over x, y, z, per timeslice (1/(2 V3)) and (1/(6 V3)).
#include "gf_kernels.h"
#include "gf_site.h"
#include "gf_su2.h"

namespace gf {
namespace {

constexpr int RB = 256;  // threads per block of the reductions and layout kernels

template <typename R>
__device__ __forceinline__ size_t chunk2_index(const Su2Field<R>& f, int parity, int mu, int c, uint32_t h)
{
    const size_t tile = (size_t)(parity * 4 + mu) * (f.ld / kLinkTile) + h / kLinkTile;
    return (tile * Su2Chunks<R>::N + c) * kLinkTile + h % kLinkTile;
}

template <bool NT>
__device__ __forceinline__ Quat<double> load_q(const Su2Field<double>& f, int parity, int mu, uint32_t h)
{
    const double2 a = ld16<NT>(f.base + chunk2_index(f, parity, mu, 0, h));
    const double2 b = ld16<NT>(f.base + chunk2_index(f, parity, mu, 1, h));
    return Quat<double>{a.x, a.y, b.x, b.y};
}

template <bool NT>
__device__ __forceinline__ Quat<float> load_q(const Su2Field<float>& f, int parity, int mu, uint32_t h)
{
    const float4 a = ld16<NT>(f.base + chunk2_index(f, parity, mu, 0, h));
    return Quat<float>{a.x, a.y, a.z, a.w};
}

template <bool NT>
__device__ __forceinline__ void store_q(const Su2Field<double>& f, int parity, int mu, uint32_t h,
                                        const Quat<double>& q)
{
    st16<NT>(f.base + chunk2_index(f, parity, mu, 0, h), make_double2(q.b0, q.b1));
    st16<NT>(f.base + chunk2_index(f, parity, mu, 1, h), make_double2(q.b2, q.b3));
}

template <bool NT>
__device__ __forceinline__ void store_q(const Su2Field<float>& f, int parity, int mu, uint32_t h,
                                        const Quat<float>& q)
{
    st16<NT>(f.base + chunk2_index(f, parity, mu, 0, h), make_float4(q.b0, q.b1, q.b2, q.b3));
}

// p o q (matrix product of the two elements)
template <typename R>
__device__ __forceinline__ Quat<R> qmul(const Quat<R>& p, const Quat<R>& q)
{
    Quat<R> r;
    r.b0 = fmad(p.b0, q.b0, -fmad(p.b1, q.b1, fmad(p.b2, q.b2, p.b3 * q.b3)));
    r.b1 = fmad(p.b0, q.b1, fmad(q.b0, p.b1, -fmad(p.b2, q.b3, -(p.b3 * q.b2))));
    r.b2 = fmad(p.b0, q.b2, fmad(q.b0, p.b2, -fmad(p.b3, q.b1, -(p.b1 * q.b3))));
    r.b3 = fmad(p.b0, q.b3, fmad(q.b0, p.b3, -fmad(p.b1, q.b2, -(p.b2 * q.b1))));
    return r;
}

template <typename R>
__device__ __forceinline__ Quat<R> qdag(const Quat<R>& q)
{
    return Quat<R>{q.b0, -q.b1, -q.b2, -q.b3};
}

// Quaternion c of K(x) over the first NDIR directions, summed in the fixed
// order ((f0 + b0) + (f1 + b1)) + ((f2 + b2) + (f3 + b3)).
template <int NDIR, typename R>
__device__ __forceinline__ Quat<R> k_of(const Quat<R>* f, const Quat<R>* b)
{
    Quat<R> leaf[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        if (mu < NDIR) {
            leaf[mu] = Quat<R>{f[mu].b0 + b[mu].b0, f[mu].b1 - b[mu].b1, f[mu].b2 - b[mu].b2, f[mu].b3 - b[mu].b3};
        } else {
            leaf[mu] = Quat<R>{R(0), R(0), R(0), R(0)};
        }
    }
    auto add = [](const Quat<R>& a, const Quat<R>& c) {
        return Quat<R>{a.b0 + c.b0, a.b1 + c.b1, a.b2 + c.b2, a.b3 + c.b3};
    };
    return add(add(leaf[0], leaf[1]), add(leaf[2], leaf[3]));
}

template <typename R, int MODE, int BLOCK, int CP, int NDIR>
__global__ void __launch_bounds__(BLOCK) k_su2_half_sweep(Su2Field<R> f, Geom g, int parity, Rule<R> rule,
                                                          double* est)
{
    // white half-sweeps with cached loads take the blocks in reverse order (as the SU(3) sweep)
    const uint32_t b = (parity && !nt_loads(CP)) ? gridDim.x - 1u - blockIdx.x : blockIdx.x;
    const uint32_t h = b * (uint32_t)BLOCK + threadIdx.x;
    double th = 0.0;
    if (h < g.vh) {
        const Site s = decode_site(g, parity, h);
        const uint32_t lex = 2 * h + (uint32_t)(s.x & 1);
        Quat<R> fw[4], bw[4];
        uint32_t at[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) at[mu] = back_h(g, h, s, mu);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            fw[mu] = load_q<nt_loads(CP)>(f, parity, mu, h);
            bw[mu] = load_q<nt_loads(CP)>(f, 1 - parity, mu, at[mu]);
        }
        const Quat<R> c = k_of<NDIR>(fw, bw);
        if (est) th = 2.0 * ((double)c.b1 * (double)c.b1 + (double)c.b2 * (double)c.b2 + (double)c.b3 * (double)c.b3);
        const Quat<R> a2{R(2) * c.b0, R(2) * c.b1, R(2) * c.b2, R(2) * c.b3};
        const Quat<R> gx = subgroup_element<MODE>(a2, rule, lex, 0u);
        const Quat<R> gd = qdag(gx);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            store_q<nt_stores(CP)>(f, parity, mu, h, qmul(gx, fw[mu]));
            store_q<nt_stores(CP)>(f, 1 - parity, mu, at[mu], qmul(bw[mu], gd));
        }
    }
    if (est) block_sum2<BLOCK>(th, 0.0, est + 2 * ((size_t)parity * gridDim.x + b));
}

// Landau: per-block (theta, F) partial sums over both colours (blocks alternate colours tile by tile).
// Coulomb: the same per timeslice t = blockIdx.y.
template <typename R, int NDIR>
__global__ void __launch_bounds__(RB) k_su2_measure(Su2Field<R> f, Geom g, double* partial)
{
    const int parity = (int)(blockIdx.x & 1u);
    const uint32_t k = (blockIdx.x >> 1) * RB + threadIdx.x;
    const uint32_t span = NDIR == 4 ? g.vh : g.hs3;
    double th = 0.0, fr = 0.0;
    if (k < span) {
        const uint32_t h = (NDIR == 4 ? 0u : blockIdx.y * g.hs3) + k;
        const Site s = decode_site(g, parity, h);
        double c1 = 0.0, c2 = 0.0, c3 = 0.0;
#pragma unroll
        for (int mu = 0; mu < NDIR; ++mu) {
            const Quat<R> a = load_q<false>(f, parity, mu, h);
            const Quat<R> b = load_q<false>(f, 1 - parity, mu, back_h(g, h, s, mu));
            fr += 2.0 * (double)a.b0;
            c1 += (double)a.b1 - (double)b.b1;
            c2 += (double)a.b2 - (double)b.b2;
            c3 += (double)a.b3 - (double)b.b3;
        }
        th = 2.0 * (c1 * c1 + c2 * c2 + c3 * c3);
    }
    block_sum2<RB>(th, fr, partial + 2 * ((size_t)blockIdx.y * gridDim.x + blockIdx.x));
}

__global__ void __launch_bounds__(RB) k_su2_finalize(const double* partial, uint32_t n, double s0, double s1,
                                                     double* out)
{
    finalize_pairs<RB>(partial + 2 * (size_t)blockIdx.x * n, n, s0, s1, out + 2 * (size_t)blockIdx.x);
}

template <typename R>
__global__ void __launch_bounds__(RB) k_su2_plaquette(Su2Field<R> f, Geom g, double* partial)
{
    const int parity = blockIdx.y;
    const uint32_t h = blockIdx.x * RB + threadIdx.x;
    double acc = 0.0;
    if (h < g.vh) {
        const Site s = decode_site(g, parity, h);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int nu = mu + 1; nu < 4; ++nu) {
                const Quat<R> a = load_q<false>(f, parity, mu, h);
                const Quat<R> b = load_q<false>(f, 1 - parity, nu, fwd_h(g, h, s, mu));
                const Quat<R> c = load_q<false>(f, 1 - parity, mu, fwd_h(g, h, s, nu));
                const Quat<R> d = load_q<false>(f, parity, nu, h);
                // Re tr[a b c^dag d^dag] = 2 (a b o (d c)^dag)_0, in float64
                const Quat<double> A{(double)a.b0, (double)a.b1, (double)a.b2, (double)a.b3};
                const Quat<double> B{(double)b.b0, (double)b.b1, (double)b.b2, (double)b.b3};
                const Quat<double> C{(double)c.b0, (double)c.b1, (double)c.b2, (double)c.b3};
                const Quat<double> D{(double)d.b0, (double)d.b1, (double)d.b2, (double)d.b3};
                acc += 2.0 * qmul(qmul(A, B), qdag(qmul(D, C))).b0;
            }
    }
    block_sum2<RB>(acc, 0.0, partial + 2 * (size_t)(blockIdx.y * gridDim.x + blockIdx.x));
}

template <typename R>
__global__ void __launch_bounds__(RB) k_su2_reunitarize(Su2Field<R> f, uint32_t vh)
{
    const uint32_t h = blockIdx.x * RB + threadIdx.x;
    if (h >= vh) return;
    const int parity = blockIdx.y >> 2, mu = blockIdx.y & 3;
    Quat<R> q = load_q<false>(f, parity, mu, h);
    const R inv = R(1) / sqrt(fmad(q.b0, q.b0, fmad(q.b1, q.b1, fmad(q.b2, q.b2, q.b3 * q.b3))));
    q = Quat<R>{q.b0 * inv, q.b1 * inv, q.b2 * inv, q.b3 * inv};
    store_q<false>(f, parity, mu, h, q);
}

__device__ __forceinline__ void lex_half(const Geom& g, uint32_t s, int* parity, uint32_t* h)
{
    uint32_t x = s % (uint32_t)g.n[0];
    uint32_t r = s / (uint32_t)g.n[0];
    uint32_t y = r % (uint32_t)g.n[1];
    r /= (uint32_t)g.n[1];
    uint32_t z = r % (uint32_t)g.n[2];
    uint32_t t = r / (uint32_t)g.n[2];
    *parity = (int)((x + y + z + t) & 1u);
    *h = s >> 1;
}

// canonical [site][mu][2][2][re,im] -> quaternion: the element's coefficients in
// the real span of SU(2) (for an SU(2) matrix, its own quaternion)
template <typename R>
__global__ void __launch_bounds__(RB) k_su2_pack(const double* canon, Su2Field<R> f, Geom g)
{
    const uint64_t gid = (uint64_t)blockIdx.x * RB + threadIdx.x;
    if (gid >= (uint64_t)g.vh * 8) return;
    const uint32_t s = (uint32_t)(gid / 4);
    const int mu = (int)(gid % 4);
    int parity;
    uint32_t h;
    lex_half(g, s, &parity, &h);
    const double* u = canon + gid * 8;  // u00 (0,1) u01 (2,3) u10 (4,5) u11 (6,7)
    const double q0 = 0.5 * (u[0] + u[6]);
    const double q3 = 0.5 * (u[1] - u[7]);
    const double q2 = 0.5 * (u[2] - u[4]);
    const double q1 = 0.5 * (u[3] + u[5]);
    store_q<false>(f, parity, mu, h, Quat<R>{(R)q0, (R)q1, (R)q2, (R)q3});
}

template <typename R>
__global__ void __launch_bounds__(RB) k_su2_unpack(Su2Field<R> f, Geom g, double* canon)
{
    const uint64_t gid = (uint64_t)blockIdx.x * RB + threadIdx.x;
    if (gid >= (uint64_t)g.vh * 8) return;
    const uint32_t s = (uint32_t)(gid / 4);
    const int mu = (int)(gid % 4);
    int parity;
    uint32_t h;
    lex_half(g, s, &parity, &h);
    const Quat<R> q = load_q<false>(f, parity, mu, h);
    double* u = canon + gid * 8;
    u[0] = (double)q.b0;
    u[1] = (double)q.b3;
    u[2] = (double)q.b2;
    u[3] = (double)q.b1;
    u[4] = -(double)q.b2;
    u[5] = (double)q.b1;
    u[6] = (double)q.b0;
    u[7] = -(double)q.b3;
}

template <typename R, int MODE, int NDIR>
hipError_t launch_block(const Su2Field<R>& f, const Geom& g, int parity, const Rule<R>& rule, const SweepConfig& c,
                        hipStream_t st, double* est)
{
    const uint32_t grid = (g.vh + (uint32_t)c.block - 1) / (uint32_t)c.block;
#define GF_SU2(B, CPV) \
    hipLaunchKernelGGL((k_su2_half_sweep<R, MODE, B, CPV, NDIR>), dim3(grid), dim3(B), 0, st, f, g, parity, rule, est)
#define GF_SU2_BLOCKS(CPV)                    \
    switch (c.block) {                        \
        case 64: GF_SU2(64, CPV); break;      \
        case 128: GF_SU2(128, CPV); break;    \
        case 256: GF_SU2(256, CPV); break;    \
        default: GF_SU2(512, CPV); break;     \
    }
    switch (c.nt) {
        case 1: GF_SU2_BLOCKS(1) break;
        case 2: GF_SU2_BLOCKS(2) break;
        default: GF_SU2_BLOCKS(0) break;
    }
#undef GF_SU2_BLOCKS
#undef GF_SU2
    return hipGetLastError();
}

template <typename R, int MODE>
hipError_t launch_gauge(const Su2Field<R>& f, const Geom& g, int parity, const Rule<R>& rule, const SweepConfig& c,
                        hipStream_t st, int gauge, double* est)
{
    return gauge == GAUGE_COULOMB ? launch_block<R, MODE, NDIR_COULOMB>(f, g, parity, rule, c, st, est)
                                  : launch_block<R, MODE, NDIR_LANDAU>(f, g, parity, rule, c, st, est);
}

template <typename R>
hipError_t or_impl(const Su2Field<R>& f, const Geom& g, int parity, R omega, int mode, const SweepConfig& c,
                   hipStream_t st, int gauge, double* est)
{
    const Rule<R> rule{omega, R(1), 0u, 0u, 0u};
    return mode == OR_EXACT ? launch_gauge<R, 0>(f, g, parity, rule, c, st, gauge, est)
                            : launch_gauge<R, 1>(f, g, parity, rule, c, st, gauge, est);
}

template <typename R>
hipError_t hb_impl(const Su2Field<R>& f, const Geom& g, int parity, R T, uint64_t seed, uint32_t sweep,
                   const SweepConfig& c, hipStream_t st, int gauge)
{
    const Rule<R> rule{R(1), T, (uint32_t)seed, (uint32_t)(seed >> 32), sweep};
    return launch_gauge<R, HEATBATH>(f, g, parity, rule, c, st, gauge, nullptr);
}

uint32_t su2_blocks(const Geom& g)
{
    return (g.vh + RB - 1) / RB;
}

template <typename R>
hipError_t measure_impl(const Su2Field<R>& f, const Geom& g, int gauge, double* partial, double* out, hipStream_t st)
{
    if (gauge == GAUGE_COULOMB) {
        const uint32_t nb = 2 * ((g.hs3 + RB - 1) / RB);
        hipLaunchKernelGGL((k_su2_measure<R, NDIR_COULOMB>), dim3(nb, (uint32_t)g.n[3]), dim3(RB), 0, st, f, g,
                           partial);
        const double V3 = 2.0 * (double)g.hs3;
        hipLaunchKernelGGL(k_su2_finalize, dim3((uint32_t)g.n[3]), dim3(RB), 0, st, partial, nb, 1.0 / (2.0 * V3),
                           1.0 / (6.0 * V3), out);
    } else {
        const uint32_t nb = 2 * su2_blocks(g);
        hipLaunchKernelGGL((k_su2_measure<R, NDIR_LANDAU>), dim3(nb, 1), dim3(RB), 0, st, f, g, partial);
        const double V = 2.0 * (double)g.vh;
        hipLaunchKernelGGL(k_su2_finalize, dim3(1), dim3(RB), 0, st, partial, nb, 1.0 / (2.0 * V), 1.0 / (8.0 * V),
                           out);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t plaquette_impl(const Su2Field<R>& f, const Geom& g, double* partial, double* out, hipStream_t st)
{
    const uint32_t nb = su2_blocks(g);
    hipLaunchKernelGGL((k_su2_plaquette<R>), dim3(nb, 2), dim3(RB), 0, st, f, g, partial);
    const double V = 2.0 * (double)g.vh;
    hipLaunchKernelGGL(k_su2_finalize, dim3(1), dim3(RB), 0, st, partial, 2 * nb, 1.0 / (12.0 * V), 0.0, out);
    return hipGetLastError();
}

}  // namespace

uint32_t su2_partials(const Geom& g)
{
    const uint32_t landau = 2 * su2_blocks(g);
    const uint32_t coulomb = 2 * ((g.hs3 + RB - 1) / RB) * (uint32_t)g.n[3];
    return landau > coulomb ? landau : coulomb;
}

bool su2_config_valid(const SweepConfig& c)
{
    return c.tps == 1 && (c.block == 64 || c.block == 128 || c.block == 256 || c.block == 512) &&
           (c.nt == 0 || c.nt == 1 || c.nt == 2) && c.minw == 0;
}

uint32_t su2_sweep_blocks(const Geom& g, const SweepConfig& c)
{
    return (g.vh + (uint32_t)c.block - 1) / (uint32_t)c.block;
}

hipError_t launch_su2_or(const Su2Field<double>& f, const Geom& g, int parity, double omega, int mode,
                         const SweepConfig& c, hipStream_t st, int gauge, double* est)
{
    return or_impl(f, g, parity, omega, mode, c, st, gauge, est);
}
hipError_t launch_su2_or(const Su2Field<float>& f, const Geom& g, int parity, float omega, int mode,
                         const SweepConfig& c, hipStream_t st, int gauge, double* est)
{
    return or_impl(f, g, parity, omega, mode, c, st, gauge, est);
}
hipError_t launch_su2_hb(const Su2Field<double>& f, const Geom& g, int parity, double T, uint64_t seed,
                         uint32_t sweep, const SweepConfig& c, hipStream_t st, int gauge)
{
    return hb_impl(f, g, parity, T, seed, sweep, c, st, gauge);
}
hipError_t launch_su2_hb(const Su2Field<float>& f, const Geom& g, int parity, float T, uint64_t seed,
                         uint32_t sweep, const SweepConfig& c, hipStream_t st, int gauge)
{
    return hb_impl(f, g, parity, T, seed, sweep, c, st, gauge);
}
hipError_t launch_su2_measure(const Su2Field<double>& f, const Geom& g, int gauge, double* p, double* o,
                              hipStream_t st)
{
    return measure_impl(f, g, gauge, p, o, st);
}
hipError_t launch_su2_measure(const Su2Field<float>& f, const Geom& g, int gauge, double* p, double* o,
                              hipStream_t st)
{
    return measure_impl(f, g, gauge, p, o, st);
}
hipError_t launch_su2_plaquette(const Su2Field<double>& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return plaquette_impl(f, g, p, o, st);
}
hipError_t launch_su2_plaquette(const Su2Field<float>& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return plaquette_impl(f, g, p, o, st);
}
hipError_t launch_su2_reunitarize(const Su2Field<double>& f, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_su2_reunitarize<double>), dim3(su2_blocks(g), 8), dim3(RB), 0, st, f, g.vh);
    return hipGetLastError();
}
hipError_t launch_su2_reunitarize(const Su2Field<float>& f, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_su2_reunitarize<float>), dim3(su2_blocks(g), 8), dim3(RB), 0, st, f, g.vh);
    return hipGetLastError();
}
hipError_t launch_su2_pack(const double* canon, const Su2Field<double>& f, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_su2_pack<double>), dim3((uint32_t)(((uint64_t)g.vh * 8 + RB - 1) / RB)), dim3(RB), 0, st,
                       canon, f, g);
    return hipGetLastError();
}
hipError_t launch_su2_pack(const double* canon, const Su2Field<float>& f, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_su2_pack<float>), dim3((uint32_t)(((uint64_t)g.vh * 8 + RB - 1) / RB)), dim3(RB), 0, st,
                       canon, f, g);
    return hipGetLastError();
}
hipError_t launch_su2_unpack(const Su2Field<double>& f, const Geom& g, double* canon, hipStream_t st)
{
    hipLaunchKernelGGL((k_su2_unpack<double>), dim3((uint32_t)(((uint64_t)g.vh * 8 + RB - 1) / RB)), dim3(RB), 0,
                       st, f, g, canon);
    return hipGetLastError();
}
hipError_t launch_su2_unpack(const Su2Field<float>& f, const Geom& g, double* canon, hipStream_t st)
{
    hipLaunchKernelGGL((k_su2_unpack<float>), dim3((uint32_t)(((uint64_t)g.vh * 8 + RB - 1) / RB)), dim3(RB), 0,
                       st, f, g, canon);
    return hipGetLastError();
}

}  // namespace gf
