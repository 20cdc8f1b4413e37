// gf_measure.hip -- lattice reductions (gauge condition theta, functional F,
// plaquette), reunitarisation and layout conversion for libgf on gfx950.
//
// theta / F (Sec. 2 of arXiv:1412.3655): with K(x) as in Eq. (localfunctional),
//   Delta(x) = sum_mu (A_mu(x) - A_mu(x-mu^)) = [(K(x) - K(x)^dag)/(2i)]_traceless
// (A_mu of Sec. 2 with a g = 1; the two forms are equal term by term), and
//   theta = (1/(3V)) sum_x tr[Delta Delta^dag],
//   F     = (1/(12V)) sum_x sum_mu Re tr U_mu(x)     (Eq. landaufunctional, g = 1);
// for Coulomb gauge the same per timeslice with mu over x, y, z only
// (k_measure_slices).
// One thread per site (both colours), float64 arithmetic and sums whatever the
// link precision; wavefront sums by xor-shuffles, block sums through LDS, one
// partial per block, then one block adds the partials in index order.  The
// reduction order depends only on the lattice shape, so results are bitwise
// reproducible.  Traffic: every link is read twice (once from each end),
// 768 B per site in FP64.
#include "gf_kernels.h"
#include "gf_site.h"

namespace gf {

namespace {

constexpr int RBLOCK = 256;

// Blocks alternate colours tile by tile (block 2b + p: colour p, tile b), so
// the second read of a link (from its other end, a few planes away) follows
// the first while the Infinity Cache still holds it, instead of half a lattice
// later.  Partial (p, b) holds the same sites whatever the dispatch order.
template <typename Field>
__global__ void __launch_bounds__(RBLOCK) k_measure(Field f, Geom g, double* partial)
{
    const int parity = (int)(blockIdx.x & 1u);
    const uint32_t tile = blockIdx.x >> 1;
    const uint32_t tiles = gridDim.x >> 1;
    const uint32_t h = tile * RBLOCK + threadIdx.x;
    double th = 0.0, fr = 0.0;
    if (h < g.vh) measure_site(f, g, parity, h, th, fr);
    block_sum2<RBLOCK>(th, fr, partial + 2 * (size_t)(parity * tiles + tile));
}

// Coulomb gauge: the sites of timeslice t are the half indices
// t*hs3 .. (t+1)*hs3 - 1 of each colour (hs3 = V3/2), so block (b, t) covers
// tile b >> 1 of colour b & 1 of timeslice t, alternating colours as k_measure
// does; partial (t, b) holds the same sites whatever the dispatch order.
template <typename Field>
__global__ void __launch_bounds__(RBLOCK) k_measure_slices(Field f, Geom g, double* partial)
{
    const int parity = (int)(blockIdx.x & 1u);
    const uint32_t k = (blockIdx.x >> 1) * RBLOCK + threadIdx.x;
    double th = 0.0, fr = 0.0;
    if (k < g.hs3) measure_site<NDIR_COULOMB>(f, g, parity, blockIdx.y * g.hs3 + k, th, fr);
    block_sum2<RBLOCK>(th, fr, partial + 2 * ((size_t)blockIdx.y * gridDim.x + blockIdx.x));
}

// Block t adds timeslice t's n partial pairs in index order.
__global__ void __launch_bounds__(RBLOCK) k_finalize_slices(const double* partial, uint32_t n, double s0, double s1,
                                                            double* out)
{
    finalize_pairs<RBLOCK>(partial + 2 * (size_t)blockIdx.x * n, n, s0, s1, out + 2 * (size_t)blockIdx.x);
}

// Re tr[U_mu(x) U_nu(x+mu^) U_mu(x+nu^)^dag U_nu(x)^dag] summed over mu < nu.
template <typename Field>
__global__ void __launch_bounds__(RBLOCK) k_plaquette(Field f, Geom g, double* partial)
{
    const int parity = blockIdx.y;
    const uint32_t h = blockIdx.x * RBLOCK + threadIdx.x;
    double acc = 0.0;
    if (h < g.vh) {
        const Site s = decode_site(g, parity, h);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int nu = mu + 1; nu < 4; ++nu) {
                M3<double> a, b, c, d;
                load_full_f64(f, parity, mu, h, a);
                load_full_f64(f, 1 - parity, nu, fwd_h(g, h, s, mu), b);
                load_full_f64(f, 1 - parity, mu, fwd_h(g, h, s, nu), c);
                load_full_f64(f, parity, nu, h, d);
                // P = a b, Q = d c; tr[P Q^dag] = sum_ij P_ij conj(Q_ij)
                double re = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            pr += a.re[i][k] * b.re[k][j] - a.im[i][k] * b.im[k][j];
                            pi += a.re[i][k] * b.im[k][j] + a.im[i][k] * b.re[k][j];
                            qr += d.re[i][k] * c.re[k][j] - d.im[i][k] * c.im[k][j];
                            qi += d.re[i][k] * c.im[k][j] + d.im[i][k] * c.re[k][j];
                        }
                        re += pr * qr + pi * qi;
                    }
                acc += re;
            }
    }
    block_sum2<RBLOCK>(acc, 0.0, partial + 2 * (size_t)(blockIdx.y * gridDim.x + blockIdx.x));
}

// The nine independent real components of Delta = [(K - K^dag)/(2i)]_traceless:
// d[0..2] the traceless diagonal (Im K_ii minus the mean), d[3..8] the real and
// imaginary parts of the off-diagonal entries (i, j), i < j, which count twice
// in tr[Delta Delta^dag].
template <typename T>
__device__ __forceinline__ void delta_components(const M3<T>& K, T d[9])
{
    const T tr3 = (K.im[0][0] + K.im[1][1] + K.im[2][2]) / T(3);
    d[0] = K.im[0][0] - tr3;
    d[1] = K.im[1][1] - tr3;
    d[2] = K.im[2][2] - tr3;
    int c = 3;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            d[c++] = T(0.5) * (K.im[i][j] + K.im[j][i]);
            d[c++] = T(0.5) * (K.re[i][j] - K.re[j][i]);
        }
}

// K(x) of the site from the float64 links, in float64 (K64) and, with every
// stored real rounded to float32 and row 2 rebuilt in float32, in float32
// (K32): what a float32 sweep sees of the same configuration.
// M8: the float32 links are the 8-real float32 storage of the float64 ones
// (encoded in float64, the values rounded, decoded in float32), as the 8-real
// float32 sweep sees them; otherwise rows 0, 1 rounded to float32.
template <bool M8>
__device__ __forceinline__ void site_K_both(const LinkField<double>& f, const Geom& g, int parity, uint32_t h,
                                            M3<double>& K64, M3<float>& K32)
{
    const Site s = decode_site(g, parity, h);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            K64.re[i][j] = 0.0;
            K64.im[i][j] = 0.0;
            K32.re[i][j] = 0.f;
            K32.im[i][j] = 0.f;
        }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            M3<double> u;
            M3<float> v;
            const int p = b ? 1 - parity : parity;
            load_rows01(f, p, mu, b ? back_h(g, h, s, mu) : h, u);
            if constexpr (M8) {
                float4 q[kMin8Chunks32];
                encode_min8(u, q);
                decode_min8(q, v);
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        v.re[i][j] = (float)u.re[i][j];
                        v.im[i][j] = (float)u.im[i][j];
                    }
                rebuild_row2(v);
            }
            rebuild_row2(u);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    K64.re[i][j] += b ? u.re[j][i] : u.re[i][j];
                    K64.im[i][j] += b ? -u.im[j][i] : u.im[i][j];
                    K32.re[i][j] += b ? v.re[j][i] : v.re[i][j];
                    K32.im[i][j] += b ? -v.im[j][i] : v.im[i][j];
                }
        }
}

// Per site: tr[E E^dag] with E = Delta(K32) - Delta(K64), the float32 rounding
// error of the local gauge condition.
template <bool M8>
__global__ void __launch_bounds__(RBLOCK) k_fp32_floor(LinkField<double> f, Geom g, double* partial)
{
    const int parity = blockIdx.y;
    const uint32_t h = blockIdx.x * RBLOCK + threadIdx.x;
    double acc = 0.0;
    if (h < g.vh) {
        M3<double> K64;
        M3<float> K32;
        site_K_both<M8>(f, g, parity, h, K64, K32);
        double d64[9];
        float d32[9];
        delta_components(K64, d64);
        delta_components(K32, d32);
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const double e = (double)d32[c] - d64[c];
            acc += (c < 3 ? 1.0 : 2.0) * e * e;
        }
    }
    block_sum2<RBLOCK>(acc, 0.0, partial + 2 * (size_t)(blockIdx.y * gridDim.x + blockIdx.x));
}

// out[k] = scale[k] * sum_i partial[2 i + k], summed in a fixed order.
__global__ void __launch_bounds__(RBLOCK) k_finalize(const double* partial, uint32_t n, double s0, double s1, double* out)
{
    finalize_pairs<RBLOCK>(partial, n, s0, s1, out);
}

// Gram-Schmidt on rows 0, 1 (row 2 stays implicit).
template <typename R>
__global__ void __launch_bounds__(RBLOCK) k_reunitarize(LinkField<R> f, uint32_t vh)
{
    const uint32_t h = blockIdx.x * RBLOCK + threadIdx.x;
    if (h >= vh) return;
    const int parity = blockIdx.y >> 2, mu = blockIdx.y & 3;
    M3<R> u;
    load_rows01(f, parity, mu, h, u);
    gram_schmidt_rows01(u);
    store_rows01(f, parity, mu, h, u);
}

__global__ void __launch_bounds__(RBLOCK) k_g_identity(GField gacc, uint32_t vh)
{
    const uint32_t h = blockIdx.x * RBLOCK + threadIdx.x;
    if (h >= vh) return;
    const int parity = blockIdx.y;
    gacc.base[g_index(gacc, parity, 0, h)] = make_float4(1.f, 0.f, 0.f, 0.f);  // g00, g01
    gacc.base[g_index(gacc, parity, 1, h)] = make_float4(0.f, 0.f, 0.f, 0.f);  // g02, g10
    gacc.base[g_index(gacc, parity, 2, h)] = make_float4(1.f, 0.f, 0.f, 0.f);  // g11, g12
}

__global__ void __launch_bounds__(RBLOCK) k_g_reunitarize(GField gacc, uint32_t vh)
{
    const uint32_t h = blockIdx.x * RBLOCK + threadIdx.x;
    if (h >= vh) return;
    const int parity = blockIdx.y;
    M3<float> u;
    load_g(gacc, parity, h, u);
    gram_schmidt_rows01(u);
#pragma unroll
    for (int c = 0; c < 3; ++c) store_g_chunk(gacc, parity, h, c, u);
}

// g(x) as a float64 SU(3) matrix: rows 0, 1 orthonormalised in float64, row 2 rebuilt.
__device__ __forceinline__ void load_g_f64(const GField& gacc, int parity, uint32_t h, M3<double>& g)
{
    M3<float> t;
    load_g(gacc, parity, h, t);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            g.re[i][j] = (double)t.re[i][j];
            g.im[i][j] = (double)t.im[i][j];
        }
    gram_schmidt_rows01(g);
    rebuild_row2(g);
}

// U_mu(x) <- g(x) U0_mu(x) g(x+mu^)^dag (the gauge transformation of Sec. 2 with
// the accumulated g), in place over the float64 field that holds U0.
__global__ void __launch_bounds__(RBLOCK) k_rebuild_from_g(LinkField<double> u0, GField gacc, Geom g)
{
    const uint32_t h = blockIdx.x * RBLOCK + threadIdx.x;
    if (h >= g.vh) return;
    const int parity = blockIdx.y >> 2, mu = blockIdx.y & 3;
    const Site s = decode_site(g, parity, h);
    M3<double> gx, gy, u;
    load_g_f64(gacc, parity, h, gx);
    load_g_f64(gacc, 1 - parity, fwd_h(g, h, s, mu), gy);
    load_rows01(u0, parity, mu, h, u);
    rebuild_row2(u);
    left_mul_rows01(gx, u);
    right_mul_dag_rows01(gy, u);
    store_rows01(u0, parity, mu, h, u);
}

// canonical lex site s, direction mu -> (colour, half index)
__device__ __forceinline__ void lex_to_half(const Geom& g, uint32_t s, int* parity, uint32_t* h)
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

// R: the field's real type; Field: 12-real LinkField<R> or 8-real Link8Field
// (rows 0 and 1 of the canonical link are encoded).  Links first .. first+n-1
// (canonical order, 4 per site), read from canon[0 .. 18 n).
template <typename R, typename Field>
__global__ void __launch_bounds__(RBLOCK) k_pack(const double* canon, Field f, Geom g, uint64_t first, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * RBLOCK + threadIdx.x;
    if (i >= n) return;
    const uint64_t gid = first + i;
    const uint32_t s = (uint32_t)(gid >> 2);
    const int mu = (int)(gid & 3);
    int parity;
    uint32_t h;
    lex_to_half(g, s, &parity, &h);
    const double* src = canon + i * 18;
    M3<R> u;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            u.re[i][j] = (R)src[(i * 3 + j) * 2];
            u.im[i][j] = (R)src[(i * 3 + j) * 2 + 1];
        }
    store_link(f, parity, mu, h, u);
}

// Links first .. first+n-1 written to canon[0 .. 18 n).
template <typename Field>
__global__ void __launch_bounds__(RBLOCK) k_unpack(Field f, Geom g, double* canon, uint64_t first, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * RBLOCK + threadIdx.x;
    if (i >= n) return;
    const uint64_t gid = first + i;
    const uint32_t s = (uint32_t)(gid >> 2);
    const int mu = (int)(gid & 3);
    int parity;
    uint32_t h;
    lex_to_half(g, s, &parity, &h);
    M3<double> u;
    load_full_f64(f, parity, mu, h, u);
    double* dst = canon + i * 18;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            dst[(i * 3 + j) * 2] = u.re[i][j];
            dst[(i * 3 + j) * 2 + 1] = u.im[i][j];
        }
}

// Every link of one field written into another of the other storage (12-real
// rows 0, 1 with row 2 rebuilt <-> 8-real codec).
template <typename From, typename To>
__global__ void __launch_bounds__(RBLOCK) k_convert(From from, To to, uint32_t vh)
{
    const uint32_t h = blockIdx.x * RBLOCK + threadIdx.x;
    if (h >= vh) return;
    const int parity = blockIdx.y >> 2, mu = blockIdx.y & 3;
    M3<double> u;
    load_full_f64(from, parity, mu, h, u);
    store_link(to, parity, mu, h, u);
}

uint32_t site_blocks(const Geom& g)
{
    return (g.vh + RBLOCK - 1) / RBLOCK;
}

template <typename Field>
hipError_t measure_impl(const Field& f, const Geom& g, double* partial, double* out, hipStream_t st)
{
    const uint32_t nb = site_blocks(g);
    hipLaunchKernelGGL((k_measure<Field>), dim3(2 * nb), dim3(RBLOCK), 0, st, f, g, partial);
    const double V = 2.0 * (double)g.vh;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RBLOCK), 0, st, partial, 2 * nb, 1.0 / (3.0 * V), 1.0 / (12.0 * V),
                       out);
    return hipGetLastError();
}

// Blocks per timeslice of k_measure_slices (both colours).
uint32_t slice_blocks(const Geom& g)
{
    return 2 * ((g.hs3 + RBLOCK - 1) / RBLOCK);
}

template <typename Field>
hipError_t measure_slices_impl(const Field& f, const Geom& g, double* partial, double* out, hipStream_t st)
{
    const uint32_t nb = slice_blocks(g);
    hipLaunchKernelGGL((k_measure_slices<Field>), dim3(nb, (uint32_t)g.n[3]), dim3(RBLOCK), 0, st, f, g, partial);
    const double V3 = 2.0 * (double)g.hs3;
    hipLaunchKernelGGL(k_finalize_slices, dim3((uint32_t)g.n[3]), dim3(RBLOCK), 0, st, partial, nb,
                       1.0 / (3.0 * V3), 1.0 / (9.0 * V3), out);
    return hipGetLastError();
}

template <typename Field>
hipError_t plaquette_impl(const Field& f, const Geom& g, double* partial, double* out, hipStream_t st)
{
    const uint32_t nb = site_blocks(g);
    hipLaunchKernelGGL((k_plaquette<Field>), dim3(nb, 2), dim3(RBLOCK), 0, st, f, g, partial);
    const double V = 2.0 * (double)g.vh;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RBLOCK), 0, st, partial, 2 * nb, 1.0 / (18.0 * V), 0.0, out);
    return hipGetLastError();
}

template <typename R>
hipError_t reunit_impl(const LinkField<R>& f, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_reunitarize<R>), dim3(site_blocks(g), 8), dim3(RBLOCK), 0, st, f, g.vh);
    return hipGetLastError();
}

// n = 0 stands for every link of the lattice; a range must lie inside it.
template <typename R, typename Field>
hipError_t pack_impl(const double* canon, const Field& f, const Geom& g, hipStream_t st, uint64_t first = 0,
                     uint64_t n = 0)
{
    const uint64_t nlinks = (uint64_t)g.vh * 8;
    if (n == 0 && first == 0) n = nlinks;
    if (first > nlinks || n > nlinks - first) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_pack<R, Field>), dim3((uint32_t)((n + RBLOCK - 1) / RBLOCK)), dim3(RBLOCK), 0, st, canon, f,
                       g, first, n);
    return hipGetLastError();
}

template <typename Field>
hipError_t unpack_impl(const Field& f, const Geom& g, double* canon, hipStream_t st, uint64_t first = 0,
                       uint64_t n = 0)
{
    const uint64_t nlinks = (uint64_t)g.vh * 8;
    if (n == 0 && first == 0) n = nlinks;
    if (first > nlinks || n > nlinks - first) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_unpack<Field>), dim3((uint32_t)((n + RBLOCK - 1) / RBLOCK)), dim3(RBLOCK), 0, st, f, g,
                       canon, first, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_g_identity(const GField& gacc, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL(k_g_identity, dim3(site_blocks(g), 2), dim3(RBLOCK), 0, st, gacc, g.vh);
    return hipGetLastError();
}

hipError_t launch_g_reunitarize(const GField& gacc, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL(k_g_reunitarize, dim3(site_blocks(g), 2), dim3(RBLOCK), 0, st, gacc, g.vh);
    return hipGetLastError();
}

hipError_t launch_rebuild_from_g(const LinkField<double>& u0, const GField& gacc, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL(k_rebuild_from_g, dim3(site_blocks(g), 8), dim3(RBLOCK), 0, st, u0, gacc, g);
    return hipGetLastError();
}

uint32_t measure_blocks(const Geom& g)
{
    return 2 * site_blocks(g);
}

hipError_t launch_finalize(const double* partial, uint32_t n, double s0, double s1, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RBLOCK), 0, st, partial, n, s0, s1, out);
    return hipGetLastError();
}

uint32_t slice_partials(const Geom& g)
{
    return slice_blocks(g) * (uint32_t)g.n[3];
}

hipError_t launch_measure_slices(const LinkField<double>& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_slices_impl(f, g, p, o, st);
}
hipError_t launch_measure_slices(const LinkField<float>& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_slices_impl(f, g, p, o, st);
}

hipError_t launch_fp32_floor(const LinkField<double>& f, const Geom& g, double* partial, double* out, hipStream_t st,
                             bool min8)
{
    const uint32_t nb = site_blocks(g);
    if (min8)
        hipLaunchKernelGGL(k_fp32_floor<true>, dim3(nb, 2), dim3(RBLOCK), 0, st, f, g, partial);
    else
        hipLaunchKernelGGL(k_fp32_floor<false>, dim3(nb, 2), dim3(RBLOCK), 0, st, f, g, partial);
    const double V = 2.0 * (double)g.vh;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RBLOCK), 0, st, partial, 2 * nb, 1.0 / (3.0 * V), 0.0, out);
    return hipGetLastError();
}

hipError_t launch_measure(const LinkField<double>& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_impl(f, g, p, o, st);
}
hipError_t launch_measure(const LinkField<float>& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_impl(f, g, p, o, st);
}
hipError_t launch_measure_canonical(const double* canon, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_impl(CanonField{canon, g}, g, p, o, st);
}
hipError_t launch_plaquette(const LinkField<double>& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return plaquette_impl(f, g, p, o, st);
}
hipError_t launch_plaquette(const LinkField<float>& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return plaquette_impl(f, g, p, o, st);
}
hipError_t launch_reunitarize(const LinkField<double>& f, const Geom& g, hipStream_t st)
{
    return reunit_impl(f, g, st);
}
hipError_t launch_reunitarize(const LinkField<float>& f, const Geom& g, hipStream_t st)
{
    return reunit_impl(f, g, st);
}
hipError_t launch_pack(const double* c, const LinkField<double>& f, const Geom& g, hipStream_t st)
{
    return pack_impl<double>(c, f, g, st);
}
hipError_t launch_pack(const double* c, const LinkField<float>& f, const Geom& g, hipStream_t st)
{
    return pack_impl<float>(c, f, g, st);
}
hipError_t launch_unpack(const LinkField<double>& f, const Geom& g, double* c, hipStream_t st)
{
    return unpack_impl(f, g, c, st);
}
hipError_t launch_unpack(const LinkField<float>& f, const Geom& g, double* c, hipStream_t st)
{
    return unpack_impl(f, g, c, st);
}
hipError_t launch_pack_range(const double* c, const LinkField<double>& f, const Geom& g, uint64_t first, uint64_t n,
                             hipStream_t st)
{
    return n ? pack_impl<double>(c, f, g, st, first, n) : hipSuccess;
}
hipError_t launch_pack_range(const double* c, const LinkField<float>& f, const Geom& g, uint64_t first, uint64_t n,
                             hipStream_t st)
{
    return n ? pack_impl<float>(c, f, g, st, first, n) : hipSuccess;
}
hipError_t launch_unpack_range(const LinkField<double>& f, const Geom& g, double* c, uint64_t first, uint64_t n,
                               hipStream_t st)
{
    return n ? unpack_impl(f, g, c, st, first, n) : hipSuccess;
}
hipError_t launch_unpack_range(const LinkField<float>& f, const Geom& g, double* c, uint64_t first, uint64_t n,
                               hipStream_t st)
{
    return n ? unpack_impl(f, g, c, st, first, n) : hipSuccess;
}

hipError_t launch_measure(const Link8Field& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_impl(f, g, p, o, st);
}
hipError_t launch_measure_slices(const Link8Field& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_slices_impl(f, g, p, o, st);
}
hipError_t launch_plaquette(const Link8Field& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return plaquette_impl(f, g, p, o, st);
}
hipError_t launch_pack(const double* c, const Link8Field& f, const Geom& g, hipStream_t st)
{
    return pack_impl<double>(c, f, g, st);
}
hipError_t launch_unpack(const Link8Field& f, const Geom& g, double* c, hipStream_t st)
{
    return unpack_impl(f, g, c, st);
}

hipError_t launch_convert(const LinkField<double>& from, const Link8Field& to, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_convert<LinkField<double>, Link8Field>), dim3(site_blocks(g), 8), dim3(RBLOCK), 0, st, from,
                       to, g.vh);
    return hipGetLastError();
}
hipError_t launch_convert(const Link8Field& from, const LinkField<double>& to, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_convert<Link8Field, LinkField<double>>), dim3(site_blocks(g), 8), dim3(RBLOCK), 0, st, from,
                       to, g.vh);
    return hipGetLastError();
}

hipError_t launch_measure(const Link8Field32& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_impl(f, g, p, o, st);
}
hipError_t launch_measure_slices(const Link8Field32& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return measure_slices_impl(f, g, p, o, st);
}
hipError_t launch_plaquette(const Link8Field32& f, const Geom& g, double* p, double* o, hipStream_t st)
{
    return plaquette_impl(f, g, p, o, st);
}
hipError_t launch_pack(const double* c, const Link8Field32& f, const Geom& g, hipStream_t st)
{
    return pack_impl<double>(c, f, g, st);
}
hipError_t launch_unpack(const Link8Field32& f, const Geom& g, double* c, hipStream_t st)
{
    return unpack_impl(f, g, c, st);
}
hipError_t launch_pack_range(const double* c, const Link8Field32& f, const Geom& g, uint64_t first, uint64_t n,
                             hipStream_t st)
{
    return n ? pack_impl<double>(c, f, g, st, first, n) : hipSuccess;
}
hipError_t launch_unpack_range(const Link8Field32& f, const Geom& g, double* c, uint64_t first, uint64_t n,
                               hipStream_t st)
{
    return n ? unpack_impl(f, g, c, st, first, n) : hipSuccess;
}
hipError_t launch_convert(const LinkField<float>& from, const Link8Field32& to, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_convert<LinkField<float>, Link8Field32>), dim3(site_blocks(g), 8), dim3(RBLOCK), 0, st, from,
                       to, g.vh);
    return hipGetLastError();
}
hipError_t launch_convert(const Link8Field32& from, const LinkField<float>& to, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_convert<Link8Field32, LinkField<float>>), dim3(site_blocks(g), 8), dim3(RBLOCK), 0, st, from,
                       to, g.vh);
    return hipGetLastError();
}

}  // namespace gf
