// gf_device.h -- device-side lattice layout, 12-real link codec and SU(3)
// register arithmetic for the gfx950 kernels of libgf.
//
// Layout (Sec. 3.1 of arXiv:1412.3655: checkerboard-split sublattices, site
// index fastest; two-row 12-real SU(3) representation):
//   The V sites split into two colours, black (x+y+z+t even) and white.  A
//   site of colour p has the half index h = lex >> 1, lex = x + Nx*(y + ...),
//   so both colours number their sites 0..V/2-1 and the half index of
//   (x, y, z, t) is (x>>1) + Nx/2*(y + Ny*(z + Nz*t)).
//   Links are stored as 16-byte chunks in tiles of T = 64 sites: chunk c of
//   the link U_mu of the site (p, h) at
//     base[(((p*4 + mu)*(ld/T) + h/T)*NC + c)*T + h%T],
//   ld = V/2 rounded up to 64.  A tile holds the NC chunk runs of 64
//   consecutive sites of one colour and direction back to back (6 KiB in
//   FP64), so a wavefront's loads of one link fall in one contiguous region
//   instead of NC regions ld apart.
//   FP64: NC = 6 chunks of double2 = (re, im) of u00 u01 u02 u10 u11 u12.
//   FP32: NC = 3 chunks of float4  = (u00 u01), (u02 u10), (u11 u12).
//   Consecutive sites of one colour are consecutive 16-byte words within a
//   chunk run, so a wavefront reads each chunk of its forward links as one
//   contiguous run.
//   Row 2 is never stored; it is rebuilt as conj(row0 x row1).
//   A backward link U_mu(x - mu^) lives in the other colour at half index
//   h - stride_mu/2 for mu = y, z, t (wrapping), and at h or h-1 for mu = x:
//   those gathers are also contiguous runs.
//
// Arithmetic: every multiply-add below is an explicit fma and automatic FP
// contraction is off, so each expression rounds the same way wherever it is
// inlined; this keeps the links bitwise identical across launch shapes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace gf {

__device__ __forceinline__ double fmad(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}

__device__ __forceinline__ float fmad(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}

// ---------------------------------------------------------------- geometry --

// Division by a runtime constant d >= 1 for 0 <= n < 2^31:
// q = (n * m) >> (32 + l), l = ceil(log2 d), m = floor(2^(32+l) / d) + 1.
// The host checks exactness over every n the kernels use.
struct FastDiv {
    uint64_t m;
    uint32_t shift;
    uint32_t d;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    return (uint32_t)(((uint64_t)n * f.m) >> f.shift);
}

struct Geom {
    int32_t n[4];     // Nx, Ny, Nz, Nt
    int32_t hx;       // Nx / 2
    uint32_t vh;      // V / 2 sites per colour
    uint32_t ld;      // chunk row length (vh rounded up to 64)
    uint32_t hs1, hs2, hs3;  // half-index strides of y, z, t
    FastDiv div_hx, div_ny, div_nz;
};

struct Site {
    int32_t x, y, z, t;
};

// Coordinates of the site (parity, h).
__device__ __forceinline__ Site decode_site(const Geom& g, int parity, uint32_t h)
{
    uint32_t r1 = fdiv(h, g.div_hx);
    int32_t xh = (int32_t)(h - r1 * (uint32_t)g.hx);
    uint32_t r2 = fdiv(r1, g.div_ny);
    int32_t y = (int32_t)(r1 - r2 * (uint32_t)g.n[1]);
    uint32_t t = fdiv(r2, g.div_nz);
    int32_t z = (int32_t)(r2 - t * (uint32_t)g.n[2]);
    Site s;
    s.y = y;
    s.z = z;
    s.t = (int32_t)t;
    s.x = 2 * xh + ((parity + y + z + (int32_t)t) & 1);
    return s;
}

// Half index of x - mu^ (lives in the other colour).
__device__ __forceinline__ uint32_t back_h(const Geom& g, uint32_t h, const Site& s, int mu)
{
    if (mu == 0) {
        int32_t xb = s.x == 0 ? g.n[0] - 1 : s.x - 1;
        return h - (uint32_t)(s.x >> 1) + (uint32_t)(xb >> 1);
    }
    if (mu == 1) return s.y == 0 ? h + g.hs1 * (uint32_t)(g.n[1] - 1) : h - g.hs1;
    if (mu == 2) return s.z == 0 ? h + g.hs2 * (uint32_t)(g.n[2] - 1) : h - g.hs2;
    return s.t == 0 ? h + g.hs3 * (uint32_t)(g.n[3] - 1) : h - g.hs3;
}

// Half index of x + mu^ (other colour).
__device__ __forceinline__ uint32_t fwd_h(const Geom& g, uint32_t h, const Site& s, int mu)
{
    if (mu == 0) {
        int32_t xf = s.x == g.n[0] - 1 ? 0 : s.x + 1;
        return h - (uint32_t)(s.x >> 1) + (uint32_t)(xf >> 1);
    }
    if (mu == 1) return s.y == g.n[1] - 1 ? h - g.hs1 * (uint32_t)(g.n[1] - 1) : h + g.hs1;
    if (mu == 2) return s.z == g.n[2] - 1 ? h - g.hs2 * (uint32_t)(g.n[2] - 1) : h + g.hs2;
    return s.t == g.n[3] - 1 ? h - g.hs3 * (uint32_t)(g.n[3] - 1) : h + g.hs3;
}

// ------------------------------------------------------------ link fields --

template <typename R>
struct ChunkOf;
template <>
struct ChunkOf<double> {
    using T = double2;
    static constexpr int N = 6;
};
template <>
struct ChunkOf<float> {
    using T = float4;
    static constexpr int N = 3;
};

template <typename R>
struct LinkField {
    typename ChunkOf<R>::T* base;
    uint32_t ld;
};

// 3x3 complex matrix held in registers; all indices must be compile-time.
template <typename R>
struct M3 {
    R re[3][3];
    R im[3][3];
};

constexpr uint32_t kLinkTile = 64;  // sites per tile of the link layout; ld is a multiple of it

template <typename R>
__device__ __forceinline__ size_t chunk_index(const LinkField<R>& f, int parity, int mu, int c, uint32_t h)
{
    const size_t tile = (size_t)(parity * 4 + mu) * (f.ld / kLinkTile) + h / kLinkTile;
    return (tile * ChunkOf<R>::N + c) * kLinkTile + h % kLinkTile;
}

// 16-byte chunk access; NT = non-temporal (streaming) access.
//
// Cache policy of a sweep's link accesses, the autotuner's cache axis:
// 0 = plain loads and stores, 1 = non-temporal loads and stores,
// 2 = plain loads and non-temporal stores.
constexpr bool nt_loads(int cp)
{
    return cp == 1;
}
constexpr bool nt_stores(int cp)
{
    return cp == 1 || cp == 2;
}
typedef double nt_v2d __attribute__((ext_vector_type(2)));
typedef float nt_v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ double2 ld16(const double2* p)
{
    if constexpr (NT) {
        const nt_v2d v = __builtin_nontemporal_load((const nt_v2d*)p);
        return make_double2(v.x, v.y);
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ float4 ld16(const float4* p)
{
    if constexpr (NT) {
        const nt_v4f v = __builtin_nontemporal_load((const nt_v4f*)p);
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ void st16(double2* p, double2 v)
{
    if constexpr (NT) {
        nt_v2d w;
        w.x = v.x;
        w.y = v.y;
        __builtin_nontemporal_store(w, (nt_v2d*)p);
    } else {
        *p = v;
    }
}

template <bool NT>
__device__ __forceinline__ void st16(float4* p, float4 v)
{
    if constexpr (NT) {
        nt_v4f w;
        w.x = v.x;
        w.y = v.y;
        w.z = v.z;
        w.w = v.w;
        __builtin_nontemporal_store(w, (nt_v4f*)p);
    } else {
        *p = v;
    }
}

// Rows 0 and 1 of U_mu at (parity, h).
template <bool NT = false>
__device__ __forceinline__ void load_rows01(const LinkField<double>& f, int parity, int mu, uint32_t h, M3<double>& u)
{
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double2 v = ld16<NT>(f.base + chunk_index(f, parity, mu, c, h));
        u.re[c / 3][c % 3] = v.x;
        u.im[c / 3][c % 3] = v.y;
    }
}

template <bool NT = false>
__device__ __forceinline__ void load_rows01(const LinkField<float>& f, int parity, int mu, uint32_t h, M3<float>& u)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float4 v = ld16<NT>(f.base + chunk_index(f, parity, mu, c, h));
        const int e0 = 2 * c, e1 = 2 * c + 1;
        u.re[e0 / 3][e0 % 3] = v.x;
        u.im[e0 / 3][e0 % 3] = v.y;
        u.re[e1 / 3][e1 % 3] = v.z;
        u.im[e1 / 3][e1 % 3] = v.w;
    }
}

template <bool NT = false>
__device__ __forceinline__ void store_rows01(const LinkField<double>& f, int parity, int mu, uint32_t h,
                                             const M3<double>& u)
{
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double2 v;
        v.x = u.re[c / 3][c % 3];
        v.y = u.im[c / 3][c % 3];
        st16<NT>(f.base + chunk_index(f, parity, mu, c, h), v);
    }
}

template <bool NT = false>
__device__ __forceinline__ void store_rows01(const LinkField<float>& f, int parity, int mu, uint32_t h,
                                             const M3<float>& u)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int e0 = 2 * c, e1 = 2 * c + 1;
        float4 v;
        v.x = u.re[e0 / 3][e0 % 3];
        v.y = u.im[e0 / 3][e0 % 3];
        v.z = u.re[e1 / 3][e1 % 3];
        v.w = u.im[e1 / 3][e1 % 3];
        st16<NT>(f.base + chunk_index(f, parity, mu, c, h), v);
    }
}

// row2 = conj(row0 x row1): the unit-determinant completion of two orthonormal rows.
template <typename R>
__device__ __forceinline__ void rebuild_row2(M3<R>& u)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int a = (j + 1) % 3, b = (j + 2) % 3;
        // c = r0_a r1_b - r0_b r1_a, row2_j = conj(c)
        R cre = u.im[0][b] * u.im[1][a];
        cre = fmad(-u.re[0][b], u.re[1][a], cre);
        cre = fmad(-u.im[0][a], u.im[1][b], cre);
        cre = fmad(u.re[0][a], u.re[1][b], cre);
        R cim = -(u.im[0][b] * u.re[1][a]);
        cim = fmad(-u.re[0][b], u.im[1][a], cim);
        cim = fmad(u.im[0][a], u.re[1][b], cim);
        cim = fmad(u.re[0][a], u.im[1][b], cim);
        u.re[2][j] = cre;
        u.im[2][j] = -cim;
    }
}

// Gram-Schmidt of rows 0 and 1 (row 2 stays implicit):
// r0 <- r0/|r0|, r1 <- r1 - <r0, r1> r0, r1 <- r1/|r1|, <a, b> = sum conj(a_j) b_j.
template <typename R>
__device__ __forceinline__ void gram_schmidt_rows01(M3<R>& u)
{
    R n0 = u.re[0][0] * u.re[0][0];
    n0 = fmad(u.im[0][0], u.im[0][0], n0);
#pragma unroll
    for (int j = 1; j < 3; ++j) {
        n0 = fmad(u.re[0][j], u.re[0][j], n0);
        n0 = fmad(u.im[0][j], u.im[0][j], n0);
    }
    const R i0 = R(1) / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        u.re[0][j] *= i0;
        u.im[0][j] *= i0;
    }
    R pr = u.re[0][0] * u.re[1][0];
    R pi = u.re[0][0] * u.im[1][0];
    pr = fmad(u.im[0][0], u.im[1][0], pr);
    pi = fmad(-u.im[0][0], u.re[1][0], pi);
#pragma unroll
    for (int j = 1; j < 3; ++j) {
        pr = fmad(u.re[0][j], u.re[1][j], pr);
        pr = fmad(u.im[0][j], u.im[1][j], pr);
        pi = fmad(u.re[0][j], u.im[1][j], pi);
        pi = fmad(-u.im[0][j], u.re[1][j], pi);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        u.re[1][j] = fmad(-pr, u.re[0][j], fmad(pi, u.im[0][j], u.re[1][j]));
        u.im[1][j] = fmad(-pr, u.im[0][j], fmad(-pi, u.re[0][j], u.im[1][j]));
    }
    R n1 = u.re[1][0] * u.re[1][0];
    n1 = fmad(u.im[1][0], u.im[1][0], n1);
#pragma unroll
    for (int j = 1; j < 3; ++j) {
        n1 = fmad(u.re[1][j], u.re[1][j], n1);
        n1 = fmad(u.im[1][j], u.im[1][j], n1);
    }
    const R i1 = R(1) / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        u.re[1][j] *= i1;
        u.im[1][j] *= i1;
    }
}

// --------------------------------------------------------- gauge-field g(x) --
//
// The float32 gauge transformation accumulated by mixed-precision sweeps:
// rows 0, 1 of g(x) as 3 float4 chunks per site, chunk c of the site (p, h)
// at base[(p*3 + c)*ld + h] (same chunk contents as a float32 link).
struct GField {
    float4* base;
    uint32_t ld;
};

__device__ __forceinline__ size_t g_index(const GField& f, int parity, int c, uint32_t h)
{
    return ((size_t)(parity * 3 + c)) * f.ld + h;
}

__device__ __forceinline__ void load_g(const GField& f, int parity, uint32_t h, M3<float>& g)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float4 v = f.base[g_index(f, parity, c, h)];
        const int e0 = 2 * c, e1 = 2 * c + 1;
        g.re[e0 / 3][e0 % 3] = v.x;
        g.im[e0 / 3][e0 % 3] = v.y;
        g.re[e1 / 3][e1 % 3] = v.z;
        g.im[e1 / 3][e1 % 3] = v.w;
    }
}

__device__ __forceinline__ void store_g_chunk(const GField& f, int parity, uint32_t h, int c, const M3<float>& g)
{
    const int e0 = 2 * c, e1 = 2 * c + 1;
    float4 v;
    v.x = g.re[e0 / 3][e0 % 3];
    v.y = g.im[e0 / 3][e0 % 3];
    v.z = g.re[e1 / 3][e1 % 3];
    v.w = g.im[e1 / 3][e1 % 3];
    f.base[g_index(f, parity, c, h)] = v;
}

// ---------------------------------------------------------- cross-lane sums --

// DPP controls: quad_perm [1,0,3,2] (lane ^ 1), quad_perm [2,3,0,1] (lane ^ 2),
// row_half_mirror (lane i <-> 7 - i inside each group of 8).
constexpr int DPP_XOR1 = 0xB1;
constexpr int DPP_XOR2 = 0x4E;
constexpr int DPP_HALF_MIRROR = 0x141;

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    int w = __builtin_bit_cast(int, v);
    w = __builtin_amdgcn_update_dpp(w, w, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(float, w);
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    int2 w = __builtin_bit_cast(int2, v);
    w.x = __builtin_amdgcn_update_dpp(w.x, w.x, CTRL, 0xF, 0xF, false);
    w.y = __builtin_amdgcn_update_dpp(w.y, w.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, w);
}

// a += partner's a, where the partner lane is picked by CTRL.  Floating-point
// addition is commutative, so both lanes of a pair end with identical bits.
template <int CTRL, typename R>
__device__ __forceinline__ void dpp_accumulate(M3<R>& a)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            a.re[i][j] = a.re[i][j] + dpp_mov<CTRL>(a.re[i][j]);
            a.im[i][j] = a.im[i][j] + dpp_mov<CTRL>(a.im[i][j]);
        }
}

// --------------------------------------------------------- small matrix ops --

template <typename R>
__device__ __forceinline__ void m_add(M3<R>& a, const M3<R>& b)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            a.re[i][j] += b.re[i][j];
            a.im[i][j] += b.im[i][j];
        }
}

// a = u (forward leaf of K) or a = u^dagger (backward leaf)
template <typename R>
__device__ __forceinline__ void m_leaf(M3<R>& a, const M3<R>& u, bool dagger)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            a.re[i][j] = dagger ? u.re[j][i] : u.re[i][j];
            a.im[i][j] = dagger ? -u.im[j][i] : u.im[i][j];
        }
}

// rows 0, 1 of G u  (u needs all three rows)
template <typename R>
__device__ __forceinline__ void left_mul_rows01(const M3<R>& G, M3<R>& u)
{
    R ore[2][3], oim[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            R sr = G.re[i][0] * u.re[0][j];
            R si = G.re[i][0] * u.im[0][j];
            sr = fmad(-G.im[i][0], u.im[0][j], sr);
            si = fmad(G.im[i][0], u.re[0][j], si);
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                sr = fmad(G.re[i][k], u.re[k][j], sr);
                sr = fmad(-G.im[i][k], u.im[k][j], sr);
                si = fmad(G.re[i][k], u.im[k][j], si);
                si = fmad(G.im[i][k], u.re[k][j], si);
            }
            ore[i][j] = sr;
            oim[i][j] = si;
        }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            u.re[i][j] = ore[i][j];
            u.im[i][j] = oim[i][j];
        }
}

// rows 0, 1 of u G^dagger  (only rows 0, 1 of u are read)
template <typename R>
__device__ __forceinline__ void right_mul_dag_rows01(const M3<R>& G, M3<R>& u)
{
    R ore[2][3], oim[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // sum_k u_ik conj(G_jk)
            R sr = u.re[i][0] * G.re[j][0];
            R si = u.im[i][0] * G.re[j][0];
            sr = fmad(u.im[i][0], G.im[j][0], sr);
            si = fmad(-u.re[i][0], G.im[j][0], si);
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                sr = fmad(u.re[i][k], G.re[j][k], sr);
                sr = fmad(u.im[i][k], G.im[j][k], sr);
                si = fmad(u.im[i][k], G.re[j][k], si);
                si = fmad(-u.re[i][k], G.im[j][k], si);
            }
            ore[i][j] = sr;
            oim[i][j] = si;
        }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            u.re[i][j] = ore[i][j];
            u.im[i][j] = oim[i][j];
        }
}

// ----------------------------------------------- SU(2) subgroup arithmetic --

__device__ __forceinline__ void sin_cos(double x, double* s, double* c)
{
    sincos(x, s, c);
}

__device__ __forceinline__ void sin_cos(float x, float* s, float* c)
{
    sincosf(x, s, c);
}

// An SU(2) element as the quaternion b, i.e. the 2x2 block
// [[b0 + i b3, b2 + i b1], [-b2 + i b1, b0 - i b3]].
template <typename R>
struct Quat {
    R b0, b1, b2, b3;
};

// Rows I and J of M <- S M, S the embedding of b in the (I, J) subgroup.
template <int I, int J, typename R>
__device__ __forceinline__ void rotate_rows(const Quat<R>& s, M3<R>& m)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R xr = m.re[I][c], xi = m.im[I][c], yr = m.re[J][c], yi = m.im[J][c];
        // row I: (b0 + i b3) x + (b2 + i b1) y
        R ir = s.b0 * xr;
        ir = fmad(-s.b3, xi, ir);
        ir = fmad(s.b2, yr, ir);
        ir = fmad(-s.b1, yi, ir);
        R ii = s.b0 * xi;
        ii = fmad(s.b3, xr, ii);
        ii = fmad(s.b2, yi, ii);
        ii = fmad(s.b1, yr, ii);
        // row J: (-b2 + i b1) x + (b0 - i b3) y
        R jr = s.b0 * yr;
        jr = fmad(s.b3, yi, jr);
        jr = fmad(-s.b2, xr, jr);
        jr = fmad(-s.b1, xi, jr);
        R ji = s.b0 * yi;
        ji = fmad(-s.b3, yr, ji);
        ji = fmad(-s.b2, xi, ji);
        ji = fmad(s.b1, xr, ji);
        m.re[I][c] = ir;
        m.im[I][c] = ii;
        m.re[J][c] = jr;
        m.im[J][c] = ji;
    }
}

// G = embedding of b in the (I, J) subgroup (G was the identity).
template <int I, int J, typename R>
__device__ __forceinline__ void set_embedding(const Quat<R>& s, M3<R>& G)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            G.re[i][j] = (i == j) ? R(1) : R(0);
            G.im[i][j] = R(0);
        }
    G.re[I][I] = s.b0;
    G.im[I][I] = s.b3;
    G.re[I][J] = s.b2;
    G.im[I][J] = s.b1;
    G.re[J][I] = -s.b2;
    G.im[J][I] = s.b1;
    G.re[J][J] = s.b0;
    G.im[J][J] = -s.b3;
}

// Twice the coefficients of the SU(2)-span projection q of the (I, J) block
// of K: q = a0 + i(a1 s1 + a2 s2 + a3 s3) (up to the common factor 1/2).
template <int I, int J, typename R>
__device__ __forceinline__ Quat<R> block_quaternion(const M3<R>& K)
{
    Quat<R> a;
    a.b0 = K.re[I][I] + K.re[J][J];
    a.b1 = K.im[I][J] + K.im[J][I];
    a.b2 = K.re[I][J] - K.re[J][I];
    a.b3 = K.im[I][I] - K.im[J][J];
    return a;
}

}  // namespace gf
