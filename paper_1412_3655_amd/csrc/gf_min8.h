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
// update moves 1024 B instead of 1536 B.
#pragma once

#include "gf_device.h"

namespace gf {

struct Link8Field {
    double2* base;
    uint32_t ld;
};

constexpr int kMin8Chunks = 4;

__device__ __forceinline__ size_t chunk_index8(const Link8Field& f, int parity, int mu, int c, uint32_t h)
{
    const size_t tile = (size_t)(parity * 4 + mu) * (f.ld / kLinkTile) + h / kLinkTile;
    return (tile * kMin8Chunks + c) * kLinkTile + h % kLinkTile;
}

__device__ __forceinline__ uint32_t low_bit(double v)
{
    return (uint32_t)__double2loint(v) & 1u;
}

__device__ __forceinline__ double with_low_bit(double v, uint32_t bit)
{
    return __hiloint2double(__double2hiint(v), (int)(((uint32_t)__double2loint(v) & ~1u) | bit));
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

// (cos, sin) of the phase whose half-angle tangent is t
__device__ __forceinline__ void phase_of_tan_half(double t, double& c, double& s)
{
    const double d = recip(fmad(t, t, 1.0));
    c = fmad(-t, t, 1.0) * d;
    s = (2.0 * t) * d;
}

// half-angle tangent of the phase of z = re + i im, |z|^2 = a2 >= 1/3
__device__ __forceinline__ double tan_half_of(double re, double im, double a2)
{
    const double a = sqrt_of(a2);
    const bool right = re >= 0.0;
    double t = quotient(right ? im : a - re, right ? a + re : im);
    if (!(fabs(t) <= 1e150)) t = copysign(1e150, im);
    return t;
}

// v[c] for c = (k + f) mod 3, i.e. the entry of frame index f of a row whose
// pivot column is k (k in 0..2)
__device__ __forceinline__ double frame_pick(uint32_t k, int f, double v0, double v1, double v2)
{
    const uint32_t c = (k + (uint32_t)f) % 3u;
    return c == 0 ? v0 : (c == 1 ? v1 : v2);
}

// natural column c of a row held in frame order (x0, x1, x2) = columns (k, k+1, k+2)
__device__ __forceinline__ double natural_pick(uint32_t k, int c, double x0, double x1, double x2)
{
    const uint32_t f = ((uint32_t)c + 3u - k) % 3u;
    return f == 0 ? x0 : (f == 1 ? x1 : x2);
}

// The 4 stored chunks of a link -> its 3x3 matrix.
__device__ __forceinline__ void decode_min8(const double2 (&p)[kMin8Chunks], M3<double>& u)
{
    const double air = p[0].x, aii = p[0].y, ajr = p[1].x, aji = p[1].y;
    const double t0 = p[2].x, sr = p[2].y, si = p[3].x, t1 = p[3].y;
    const uint32_t k = low_bit(air) | (low_bit(aii) << 1);
    const bool q = low_bit(sr) != 0u;
    const double ai2 = fmad(air, air, aii * aii);
    const double aj2 = fmad(ajr, ajr, aji * aji);
    const double rho = sqrt_of(fmax(1.0 / 3.0, (1.0 - ai2) - aj2));
    double c, s;
    phase_of_tan_half(t0, c, s);
    const double akr = rho * c, aki = rho * s;
    double n, in;
    sqrt_rsqrt(1.0 - aj2, n, in);
    const double bm = sqrt_of(fmax(0.5, 1.0 - fmad(sr, sr, si * si)));
    phase_of_tan_half(t1, c, s);
    const double br = bm * c, bi = bm * s;
    const double alr = q ? sr : br, ali = q ? si : bi;
    const double ber = q ? br : sr, bei = q ? bi : si;
    // row 1 in frame order: r1_k = (-alpha conj(ai) - beta ak conj(aj)) / n,
    // r1_i = (alpha conj(ak) - beta ai conj(aj)) / n, r1_j = beta n
    const double xr = fmad(akr, ajr, aki * aji), xi = fmad(aki, ajr, -akr * aji);  // ak conj(aj)
    const double yr = fmad(air, ajr, aii * aji), yi = fmad(aii, ajr, -air * aji);  // ai conj(aj)
    double r1kr = fmad(-alr, air, -ali * aii);
    double r1ki = fmad(alr, aii, -ali * air);
    r1kr = fmad(-ber, xr, fmad(bei, xi, r1kr));
    r1ki = fmad(-ber, xi, fmad(-bei, xr, r1ki));
    double r1ir = fmad(alr, akr, ali * aki);
    double r1ii = fmad(ali, akr, -alr * aki);
    r1ir = fmad(-ber, yr, fmad(bei, yi, r1ir));
    r1ii = fmad(-ber, yi, fmad(-bei, yr, r1ii));
    r1kr *= in;
    r1ki *= in;
    r1ir *= in;
    r1ii *= in;
    const double r1jr = ber * n, r1ji = bei * n;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        u.re[0][cc] = natural_pick(k, cc, akr, air, ajr);
        u.im[0][cc] = natural_pick(k, cc, aki, aii, aji);
        u.re[1][cc] = natural_pick(k, cc, r1kr, r1ir, r1jr);
        u.im[1][cc] = natural_pick(k, cc, r1ki, r1ii, r1ji);
    }
    rebuild_row2(u);
}

// Rows 0 and 1 of a link (orthonormal to rounding) -> its 4 stored chunks.
__device__ __forceinline__ void encode_min8(const M3<double>& u, double2 (&p)[kMin8Chunks])
{
    const double m0 = fmad(u.re[0][0], u.re[0][0], u.im[0][0] * u.im[0][0]);
    const double m1 = fmad(u.re[0][1], u.re[0][1], u.im[0][1] * u.im[0][1]);
    const double m2 = fmad(u.re[0][2], u.re[0][2], u.im[0][2] * u.im[0][2]);
    uint32_t k = m1 > m0 ? 1u : 0u;
    const double mk = fmax(m0, m1);
    if (m2 > mk) k = 2u;
    const double ak2 = fmax(mk, m2);
    const double akr = frame_pick(k, 0, u.re[0][0], u.re[0][1], u.re[0][2]);
    const double aki = frame_pick(k, 0, u.im[0][0], u.im[0][1], u.im[0][2]);
    const double air = frame_pick(k, 1, u.re[0][0], u.re[0][1], u.re[0][2]);
    const double aii = frame_pick(k, 1, u.im[0][0], u.im[0][1], u.im[0][2]);
    const double ajr = frame_pick(k, 2, u.re[0][0], u.re[0][1], u.re[0][2]);
    const double aji = frame_pick(k, 2, u.im[0][0], u.im[0][1], u.im[0][2]);
    const double r1kr = frame_pick(k, 0, u.re[1][0], u.re[1][1], u.re[1][2]);
    const double r1ki = frame_pick(k, 0, u.im[1][0], u.im[1][1], u.im[1][2]);
    const double r1ir = frame_pick(k, 1, u.re[1][0], u.re[1][1], u.re[1][2]);
    const double r1ii = frame_pick(k, 1, u.im[1][0], u.im[1][1], u.im[1][2]);
    const double r1jr = frame_pick(k, 2, u.re[1][0], u.re[1][1], u.re[1][2]);
    const double r1ji = frame_pick(k, 2, u.im[1][0], u.im[1][1], u.im[1][2]);
    const double aj2 = fmad(ajr, ajr, aji * aji);
    double n, in;
    sqrt_rsqrt(1.0 - aj2, n, in);
    // alpha = <e1, r1> = (-ai r1_k + ak r1_i) / n
    double alr = fmad(-air, r1kr, aii * r1ki);
    double ali = fmad(-air, r1ki, -aii * r1kr);
    alr = fmad(akr, r1ir, fmad(-aki, r1ii, alr));
    ali = fmad(akr, r1ii, fmad(aki, r1ir, ali));
    alr *= in;
    ali *= in;
    // beta: e1 has no j component and e2_j = n, so r1_j = beta n
    const double ber = r1jr * in, bei = r1ji * in;
    const double al2 = fmad(alr, alr, ali * ali), be2 = fmad(ber, ber, bei * bei);
    const bool q = be2 > al2;
    const double smr = q ? alr : ber, smi = q ? ali : bei;
    const double bgr = q ? ber : alr, bgi = q ? bei : ali;
    p[0] = make_double2(with_low_bit(air, k & 1u), with_low_bit(aii, k >> 1));
    p[1] = make_double2(ajr, aji);
    p[2] = make_double2(tan_half_of(akr, aki, ak2), with_low_bit(smr, q ? 1u : 0u));
    p[3] = make_double2(smi, tan_half_of(bgr, bgi, fmax(0.5, fmax(al2, be2))));
}

template <bool NT = false>
__device__ __forceinline__ void load_min8_raw(const Link8Field& f, int parity, int mu, uint32_t h,
                                              double2 (&p)[kMin8Chunks])
{
#pragma unroll
    for (int c = 0; c < kMin8Chunks; ++c) p[c] = ld16<NT>(f.base + chunk_index8(f, parity, mu, c, h));
}

template <bool NT = false>
__device__ __forceinline__ void store_link(const Link8Field& f, int parity, int mu, uint32_t h, const M3<double>& u)
{
    double2 p[kMin8Chunks];
    encode_min8(u, p);
#pragma unroll
    for (int c = 0; c < kMin8Chunks; ++c) st16<NT>(f.base + chunk_index8(f, parity, mu, c, h), p[c]);
}

template <bool NT = false, typename R>
__device__ __forceinline__ void store_link(const LinkField<R>& f, int parity, int mu, uint32_t h, const M3<R>& u)
{
    store_rows01<NT>(f, parity, mu, h, u);
}

// Whole float64 matrix of a stored link (the measurement kernels' view).
__device__ __forceinline__ void load_full_f64(const Link8Field& f, int parity, int mu, uint32_t h, M3<double>& u)
{
    double2 p[kMin8Chunks];
    load_min8_raw(f, parity, mu, h, p);
    decode_min8(p, u);
}

}  // namespace gf
