// gf_min8.h -- float64 SU(3) links stored in 8 reals (the minimal 8-parameter
// representation that Sec. 4.1 of arXiv:1412.3655 names among those cuLGT2
// does not provide; the paper gives no formulae).
//
// Representation (a row-pivoted form of the 8-real reconstruction of Clark et
// al., Comput. Phys. Commun. 181 (2010) 1517, in which every square root is
// taken of a quantity >= 1/3 and every phase is a half-angle tangent, so the
// decode needs no trigonometric function):
//   k = the column of the largest |U_0c|, i = k+1, j = k+2 (mod 3); columns are
//   taken in the cyclic order (k, i, j), which keeps cross products oriented.
//   p0 + i p1 = U_0i, p2 + i p3 = U_0j, p4 = tan(arg U_0k / 2),
//   |U_0k| = sqrt(1 - |U_0i|^2 - |U_0j|^2).
//   With n = sqrt(1 - |U_0j|^2), e1 = (-conj U_0i, conj U_0k, 0)/n and
//   e2 = (-U_0k conj U_0j / n, -U_0i conj U_0j / n, n) (over k, i, j) are an
//   orthonormal basis of the complement of row 0, and row 1 = alpha e1 + beta e2.
//   q = 1 if |beta| > |alpha|: p5 + i p6 = the smaller of alpha, beta and
//   p7 = tan(arg of the larger / 2), its modulus sqrt(1 - |smaller|^2).
//   k (2 bits) and q ride in the lowest mantissa bits of p0, p1 and p5.
//   A phase with tangent t is ((1 - t^2) + 2t i)/(1 + t^2); t is formed as
//   Im/(|z| + Re) for Re >= 0, (|z| - Re)/Im otherwise, held to |t| <= 1e150.
//   Row 2 is conj(row 0 x row 1), as for the 12-real layout.
// Decoding always yields SU(3) to rounding, so a link stored this way is
// re-projected onto the group at every store: no separate reunitarisation.
//
// Layout: the tiled layout of the 12-real field with 4 chunks of double2 per
// link, (p0, p1) (p2, p3) (p4, p5) (p6, p7): 64 B per link, a float64 site
// update moves 1024 B instead of 1536 B.  Float32 links (Link8Field32, the
// float32 sweeps of GF_FP32 and GF_MIXED lattices) hold the same 8 values in
// 2 chunks of float4, 32 B per link: 512 B per site update instead of 768 B.
// The sweeps decode and encode in the field's precision; measurement, unpack
// and storage conversion decode the stored values in float64 (the float32
// values define an SU(3) matrix exactly), and packing encodes in float64 and
// rounds the 8 values to float32.
#pragma once

#include <type_traits>

#include "gf_device.h"

namespace gf {

struct Link8Field {
    double2* base;
    uint32_t ld;
};

struct Link8Field32 {
    float4* base;
    uint32_t ld;
};

constexpr int kMin8Chunks = 4;    // double2 chunks per float64 link
constexpr int kMin8Chunks32 = 2;  // float4 chunks per float32 link

// R: real type of the stored values; C, N: chunk type and chunks per link.
template <typename F>
struct Min8Of {
    static constexpr bool value = false;
};
template <>
struct Min8Of<Link8Field> {
    static constexpr bool value = true;
    using R = double;
    using C = double2;
    static constexpr int N = kMin8Chunks;
};
template <>
struct Min8Of<Link8Field32> {
    static constexpr bool value = true;
    using R = float;
    using C = float4;
    static constexpr int N = kMin8Chunks32;
};

template <typename F>
__device__ __forceinline__ size_t chunk_index8(const F& f, int parity, int mu, int c, uint32_t h)
{
    const size_t tile = (size_t)(parity * 4 + mu) * (f.ld / kLinkTile) + h / kLinkTile;
    return (tile * Min8Of<F>::N + c) * kLinkTile + h % kLinkTile;
}

__device__ __forceinline__ uint32_t low_bit(double v)
{
    return (uint32_t)__double2loint(v) & 1u;
}

__device__ __forceinline__ double with_low_bit(double v, uint32_t bit)
{
    return __hiloint2double(__double2hiint(v), (int)(((uint32_t)__double2loint(v) & ~1u) | bit));
}

__device__ __forceinline__ uint32_t low_bit(float v)
{
    return __float_as_uint(v) & 1u;
}

// Float32: a value whose lowest bit differs from the flag moves one unit in the
// last place up or down in magnitude, chosen by its next bit, so that a flag
// adds no bias.  (Clearing or setting the bit would shrink or grow the
// flagged values by half a unit on average at every store, a drift that
// sweeps compound: a float32 unit is 2^29 times a float64 one.)
__device__ __forceinline__ float with_low_bit(float v, uint32_t bit)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 1u) != bit) u = (u & 2u) ? u - 1u : u + 1u;
    return __uint_as_float(u);
}

// Largest stored half-angle tangent: t^2 + 1 stays finite in the type (the
// phase pi is then represented to 2/t).
template <typename R>
__device__ __forceinline__ constexpr R tan_clamp()
{
    return sizeof(R) == 8 ? (R)1e150 : (R)1e18;
}

// The codec's square roots and quotients take operands in fixed ranges (every
// square root of a value in [1/3, 1], every divisor of magnitude <= 2 or a
// finite 1 + t^2), so they skip the general routines' range scaling and
// special-value handling: a hardware reciprocal or reciprocal square root
// seed refined by Newton's (reciprocal) and Goldschmidt's (square root)
// iterations, two steps each (a seed good to 2^-14 ends within 1-2 units in
// the last place), then one residual correction.

// 1/d for 1 <= |d| < 2^1000
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fmad(-d, r, 1.0);
    r = fmad(r, e, r);
    e = fmad(-d, r, 1.0);
    return fmad(r, e, r);
}

// n / d for |n| <= 2 and 0 < |d| <= 2 (d = +-0 or subnormal gives an infinite
// or NaN quotient, which the caller clamps)
__device__ __forceinline__ double quotient(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fmad(-d, r, 1.0);
    r = fmad(r, e, r);
    e = fmad(-d, r, 1.0);
    r = fmad(r, e, r);
    const double q = n * r;
    return fmad(r, fmad(-d, q, n), q);
}

// sqrt(x) and 1/sqrt(x) for 1/4 <= x <= 2
__device__ __forceinline__ void sqrt_rsqrt(double x, double& sq, double& rs)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fmad(-g, h, 0.5);
    g = fmad(g, r, g);
    h = fmad(h, r, h);
    r = fmad(-g, h, 0.5);
    g = fmad(g, r, g);
    h = fmad(h, r, h);
    g = fmad(fmad(-g, g, x), h, g);
    double i = 2.0 * h;
    i = fmad(i, fmad(-g, i, 1.0), i);
    sq = g;
    rs = i;
}

__device__ __forceinline__ double sqrt_of(double x)
{
    double sq, rs;
    sqrt_rsqrt(x, sq, rs);
    return sq;
}

// Float32: the hardware seeds are good to about 1 unit in the last place, so
// one refinement step and the residual correction suffice.
__device__ __forceinline__ float recip(float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    return fmad(r, fmad(-d, r, 1.0f), r);
}

__device__ __forceinline__ float quotient(float n, float d)
{
    const float r = recip(d);
    const float q = n * r;
    return fmad(r, fmad(-d, q, n), q);
}

__device__ __forceinline__ void sqrt_rsqrt(float x, float& sq, float& rs)
{
    const float y = __builtin_amdgcn_rsqf(x);
    float g = x * y, h = 0.5f * y;
    const float r = fmad(-g, h, 0.5f);
    g = fmad(g, r, g);
    h = fmad(h, r, h);
    g = fmad(fmad(-g, g, x), h, g);
    float i = 2.0f * h;
    i = fmad(i, fmad(-g, i, 1.0f), i);
    sq = g;
    rs = i;
}

__device__ __forceinline__ float sqrt_of(float x)
{
    float sq, rs;
    sqrt_rsqrt(x, sq, rs);
    return sq;
}

// (cos, sin) of the phase whose half-angle tangent is t
template <typename R>
__device__ __forceinline__ void phase_of_tan_half(R t, R& c, R& s)
{
    const R d = recip(fmad(t, t, (R)1));
    c = fmad(-t, t, (R)1) * d;
    s = ((R)2 * t) * d;
}

// half-angle tangent of the phase of z = re + i im, |z|^2 = a2 >= 1/3, held
// to |t| <= clamp
template <typename R>
__device__ __forceinline__ R tan_half_of(R re, R im, R a2, R clamp)
{
    const R a = sqrt_of(a2);
    const bool right = re >= (R)0;
    R t = quotient(right ? im : a - re, right ? a + re : im);
    if (!(fabs(t) <= clamp)) t = copysign(clamp, im);
    return t;
}

// v[c] for c = (k + f) mod 3, i.e. the entry of frame index f of a row whose
// pivot column is k (k in 0..2)
template <typename R>
__device__ __forceinline__ R frame_pick(uint32_t k, int f, R v0, R v1, R v2)
{
    const uint32_t c = (k + (uint32_t)f) % 3u;
    return c == 0 ? v0 : (c == 1 ? v1 : v2);
}

// natural column c of a row held in frame order (x0, x1, x2) = columns (k, k+1, k+2)
template <typename R>
__device__ __forceinline__ R natural_pick(uint32_t k, int c, R x0, R x1, R x2)
{
    const uint32_t f = ((uint32_t)c + 3u - k) % 3u;
    return f == 0 ? x0 : (f == 1 ? x1 : x2);
}

// The 8 stored values (flag bits k, q already taken out of their low bits,
// which stay in the values: one unit in the last place) -> the link's 3x3
// matrix, computed in R.
template <typename R>
__device__ __forceinline__ void decode_min8_vals(const R (&v)[8], uint32_t k, bool q, M3<R>& u)
{
    const R air = v[0], aii = v[1], ajr = v[2], aji = v[3];
    const R t0 = v[4], sr = v[5], si = v[6], t1 = v[7];
    const R ai2 = fmad(air, air, aii * aii);
    const R aj2 = fmad(ajr, ajr, aji * aji);
    const R rho = sqrt_of(fmax((R)1 / (R)3, ((R)1 - ai2) - aj2));
    R c, s;
    phase_of_tan_half(t0, c, s);
    const R akr = rho * c, aki = rho * s;
    R n, in;
    sqrt_rsqrt((R)1 - aj2, n, in);
    const R bm = sqrt_of(fmax((R)0.5, (R)1 - fmad(sr, sr, si * si)));
    phase_of_tan_half(t1, c, s);
    const R br = bm * c, bi = bm * s;
    const R alr = q ? sr : br, ali = q ? si : bi;
    const R ber = q ? br : sr, bei = q ? bi : si;
    // row 1 in frame order: r1_k = (-alpha conj(ai) - beta ak conj(aj)) / n,
    // r1_i = (alpha conj(ak) - beta ai conj(aj)) / n, r1_j = beta n
    const R xr = fmad(akr, ajr, aki * aji), xi = fmad(aki, ajr, -akr * aji);  // ak conj(aj)
    const R yr = fmad(air, ajr, aii * aji), yi = fmad(aii, ajr, -air * aji);  // ai conj(aj)
    R r1kr = fmad(-alr, air, -ali * aii);
    R r1ki = fmad(alr, aii, -ali * air);
    r1kr = fmad(-ber, xr, fmad(bei, xi, r1kr));
    r1ki = fmad(-ber, xi, fmad(-bei, xr, r1ki));
    R r1ir = fmad(alr, akr, ali * aki);
    R r1ii = fmad(ali, akr, -alr * aki);
    r1ir = fmad(-ber, yr, fmad(bei, yi, r1ir));
    r1ii = fmad(-ber, yi, fmad(-bei, yr, r1ii));
    r1kr *= in;
    r1ki *= in;
    r1ir *= in;
    r1ii *= in;
    const R r1jr = ber * n, r1ji = bei * n;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        u.re[0][cc] = natural_pick(k, cc, akr, air, ajr);
        u.im[0][cc] = natural_pick(k, cc, aki, aii, aji);
        u.re[1][cc] = natural_pick(k, cc, r1kr, r1ir, r1jr);
        u.im[1][cc] = natural_pick(k, cc, r1ki, r1ii, r1ji);
    }
    rebuild_row2(u);
}

// Rows 0 and 1 of a link (orthonormal to rounding) -> the 8 values (without
// flag bits), the pivot k and q, computed in R; tangents held to clamp.
template <typename R>
__device__ __forceinline__ void encode_min8_vals(const M3<R>& u, R clamp, R (&v)[8], uint32_t& kk, bool& qq)
{
    const R m0 = fmad(u.re[0][0], u.re[0][0], u.im[0][0] * u.im[0][0]);
    const R m1 = fmad(u.re[0][1], u.re[0][1], u.im[0][1] * u.im[0][1]);
    const R m2 = fmad(u.re[0][2], u.re[0][2], u.im[0][2] * u.im[0][2]);
    uint32_t k = m1 > m0 ? 1u : 0u;
    const R mk = fmax(m0, m1);
    if (m2 > mk) k = 2u;
    const R ak2 = fmax(mk, m2);
    const R akr = frame_pick(k, 0, u.re[0][0], u.re[0][1], u.re[0][2]);
    const R aki = frame_pick(k, 0, u.im[0][0], u.im[0][1], u.im[0][2]);
    const R air = frame_pick(k, 1, u.re[0][0], u.re[0][1], u.re[0][2]);
    const R aii = frame_pick(k, 1, u.im[0][0], u.im[0][1], u.im[0][2]);
    const R ajr = frame_pick(k, 2, u.re[0][0], u.re[0][1], u.re[0][2]);
    const R aji = frame_pick(k, 2, u.im[0][0], u.im[0][1], u.im[0][2]);
    const R r1kr = frame_pick(k, 0, u.re[1][0], u.re[1][1], u.re[1][2]);
    const R r1ki = frame_pick(k, 0, u.im[1][0], u.im[1][1], u.im[1][2]);
    const R r1ir = frame_pick(k, 1, u.re[1][0], u.re[1][1], u.re[1][2]);
    const R r1ii = frame_pick(k, 1, u.im[1][0], u.im[1][1], u.im[1][2]);
    const R r1jr = frame_pick(k, 2, u.re[1][0], u.re[1][1], u.re[1][2]);
    const R r1ji = frame_pick(k, 2, u.im[1][0], u.im[1][1], u.im[1][2]);
    const R aj2 = fmad(ajr, ajr, aji * aji);
    R n, in;
    sqrt_rsqrt((R)1 - aj2, n, in);
    // alpha = <e1, r1> = (-ai r1_k + ak r1_i) / n
    R alr = fmad(-air, r1kr, aii * r1ki);
    R ali = fmad(-air, r1ki, -aii * r1kr);
    alr = fmad(akr, r1ir, fmad(-aki, r1ii, alr));
    ali = fmad(akr, r1ii, fmad(aki, r1ir, ali));
    alr *= in;
    ali *= in;
    // beta: e1 has no j component and e2_j = n, so r1_j = beta n
    const R ber = r1jr * in, bei = r1ji * in;
    const R al2 = fmad(alr, alr, ali * ali), be2 = fmad(ber, ber, bei * bei);
    const bool q = be2 > al2;
    v[0] = air;
    v[1] = aii;
    v[2] = ajr;
    v[3] = aji;
    v[4] = tan_half_of(akr, aki, ak2, clamp);
    v[5] = q ? alr : ber;
    v[6] = q ? ali : bei;
    v[7] = tan_half_of(q ? ber : alr, q ? bei : ali, fmax((R)0.5, fmax(al2, be2)), clamp);
    kk = k;
    qq = q;
}

// The stored chunks of a link -> its 3x3 matrix in the field's precision.
__device__ __forceinline__ void decode_min8(const double2 (&p)[kMin8Chunks], M3<double>& u)
{
    const double v[8] = {p[0].x, p[0].y, p[1].x, p[1].y, p[2].x, p[2].y, p[3].x, p[3].y};
    decode_min8_vals(v, low_bit(v[0]) | (low_bit(v[1]) << 1), low_bit(v[5]) != 0u, u);
}

__device__ __forceinline__ void decode_min8(const float4 (&p)[kMin8Chunks32], M3<float>& u)
{
    const float v[8] = {p[0].x, p[0].y, p[0].z, p[0].w, p[1].x, p[1].y, p[1].z, p[1].w};
    decode_min8_vals(v, low_bit(v[0]) | (low_bit(v[1]) << 1), low_bit(v[5]) != 0u, u);
}

// Float32 stored values decoded in float64.
__device__ __forceinline__ void decode_min8(const float4 (&p)[kMin8Chunks32], M3<double>& u)
{
    const double v[8] = {p[0].x, p[0].y, p[0].z, p[0].w, p[1].x, p[1].y, p[1].z, p[1].w};
    decode_min8_vals(v, low_bit(p[0].x) | (low_bit(p[0].y) << 1), low_bit(p[1].y) != 0u, u);
}

// Rows 0 and 1 of a link (orthonormal to rounding) -> its stored chunks.
__device__ __forceinline__ void encode_min8(const M3<double>& u, double2 (&p)[kMin8Chunks])
{
    double v[8];
    uint32_t k;
    bool q;
    encode_min8_vals(u, tan_clamp<double>(), v, k, q);
    p[0] = make_double2(with_low_bit(v[0], k & 1u), with_low_bit(v[1], k >> 1));
    p[1] = make_double2(v[2], v[3]);
    p[2] = make_double2(v[4], with_low_bit(v[5], q ? 1u : 0u));
    p[3] = make_double2(v[6], v[7]);
}

template <typename R>
__device__ __forceinline__ void encode_min8(const M3<R>& u, float4 (&p)[kMin8Chunks32])
{
    R v[8];
    uint32_t k;
    bool q;
    encode_min8_vals(u, (R)tan_clamp<float>(), v, k, q);
    p[0] = make_float4(with_low_bit((float)v[0], k & 1u), with_low_bit((float)v[1], k >> 1), (float)v[2],
                       (float)v[3]);
    p[1] = make_float4((float)v[4], with_low_bit((float)v[5], q ? 1u : 0u), (float)v[6], (float)v[7]);
}

template <bool NT = false, typename F>
__device__ __forceinline__ void load_min8_raw(const F& f, int parity, int mu, uint32_t h,
                                              typename Min8Of<F>::C (&p)[Min8Of<F>::N])
{
#pragma unroll
    for (int c = 0; c < Min8Of<F>::N; ++c) p[c] = ld16<NT>(f.base + chunk_index8(f, parity, mu, c, h));
}

template <bool NT = false>
__device__ __forceinline__ void store_link(const Link8Field& f, int parity, int mu, uint32_t h, const M3<double>& u)
{
    double2 p[kMin8Chunks];
    encode_min8(u, p);
#pragma unroll
    for (int c = 0; c < kMin8Chunks; ++c) st16<NT>(f.base + chunk_index8(f, parity, mu, c, h), p[c]);
}

// R = float: the sweep's encode; R = double: packing and conversion (encoded
// in float64, the values rounded to float32).
template <bool NT = false, typename R>
__device__ __forceinline__ void store_link(const Link8Field32& f, int parity, int mu, uint32_t h, const M3<R>& u)
{
    float4 p[kMin8Chunks32];
    encode_min8(u, p);
#pragma unroll
    for (int c = 0; c < kMin8Chunks32; ++c) st16<NT>(f.base + chunk_index8(f, parity, mu, c, h), p[c]);
}

template <bool NT = false, typename R>
__device__ __forceinline__ void store_link(const LinkField<R>& f, int parity, int mu, uint32_t h, const M3<R>& u)
{
    store_rows01<NT>(f, parity, mu, h, u);
}

// A float64 matrix into float32 12-real storage (conversion from 8 reals).
template <bool NT = false>
__device__ __forceinline__ void store_link(const LinkField<float>& f, int parity, int mu, uint32_t h,
                                           const M3<double>& u)
{
    M3<float> t;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            t.re[i][j] = (float)u.re[i][j];
            t.im[i][j] = (float)u.im[i][j];
        }
    store_rows01<NT>(f, parity, mu, h, t);
}

// Whole float64 matrix of a stored link (the measurement kernels' view).
template <typename F, typename std::enable_if<Min8Of<F>::value, int>::type = 0>
__device__ __forceinline__ void load_full_f64(const F& f, int parity, int mu, uint32_t h, M3<double>& u)
{
    typename Min8Of<F>::C p[Min8Of<F>::N];
    load_min8_raw(f, parity, mu, h, p);
    decode_min8(p, u);
}

}  // namespace gf
