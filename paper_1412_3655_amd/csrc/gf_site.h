// gf_site.h -- the per-site bodies shared by the single-lattice and the
// batched kernels of libgf: the overrelaxation / heat-bath site update and the
// per-site gauge-condition terms.
//
// One site update (Sec. 2 of arXiv:1412.3655): K(x) = sum_mu [U_mu(x) +
// U_mu(x-mu^)^dag] (Eq. localfunctional); for the SU(2) subgroups (0,1),
// (0,2), (1,2) the maximiser of the SU(2)-span projection of the 2x2 block of
// K is raised to the power omega (or, for the annealing prelude, a heat-bath
// element is drawn) and rotates K and the accumulated G; finally U_mu(x) <-
// G U_mu(x) and U_mu(x-mu^) <- U_mu(x-mu^) G^dag (the gauge transformation of
// Sec. 2 with g(x) = G and g = 1 elsewhere).  Rotating K by the subgroup
// element equals recomputing it from the rotated links (forward links become
// S U, backward links U S^dag, so K -> S K).
//
// Work split (Sec. 3.2 and 4.2 of the paper use 8 or 4 threads per site):
// TPS lanes of one wavefront share a site, lane r owning the 8/TPS links with
// leaf index r*(8/TPS) .. (r+1)*(8/TPS)-1 in the leaf order U_0(x),
// U_0(x-0^)^dag, U_1(x), U_1(x-1^)^dag, ...  Each lane sums its leaves in the
// fixed pairwise tree ((L0+L1)+(L2+L3))+((L4+L5)+(L6+L7)) and the lanes finish
// the same tree with DPP butterflies (no LDS), so K is bitwise the same for
// every TPS.  The subgroup algebra then runs redundantly in every lane of the
// group, and each lane applies G to the links it loaded and stores them.
#pragma once

#include <type_traits>

#include "gf_device.h"
#include "gf_min8.h"

namespace gf {

constexpr int OR_EXACT = 0;
constexpr int HEATBATH = 2;

// Parameters of the subgroup rule: omega for overrelaxation; temperature T,
// Philox key and sweep counter for the heat bath.
template <typename R>
struct Rule {
    R omega;
    R T;
    uint32_t key0, key1, sweep;
};

// The SU(2) element applied for the projected block quaternion a (unnormalised,
// a0 + i(a1 s1 + a2 s2 + a3 s3)): the maximiser b = (a0, -a1, -a2, -a3)/|a|
// raised to the power omega.  EXACT: with phi = atan2(|a_vec|, a0), b^omega =
// (cos(omega phi), -sin(omega phi) a_vec/|a_vec|).  BINOMIAL1: normalise
// (1 - omega) + omega b.  |a| = 0 leaves the subgroup alone.
template <int MODE, typename R>
__device__ __forceinline__ Quat<R> or_element(const Quat<R>& a, const R omega)
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


// ------------------------------------------------------------- heat bath --
//
// Simulated-annealing prelude (named in the abstract of arXiv:1412.3655; the
// paper gives no algorithm).  Each subgroup element is drawn from
// exp(Re tr[g k]/T) dHaar(g).  With q = n qhat the SU(2)-span projection of
// the block (n = |a|/2 for the quaternion a of block_quaternion) the new
// element is g = w qhat^dag where w = (r0, sqrt(1-r0^2) e), e uniform on S^2
// and r0 has density sqrt(1-r0^2) exp(kappa r0), kappa = 2n/T: Creutz's
// exponential proposal below kappa = 2, Kennedy-Pendleton from 2 on, at most
// 128 attempts (then r0 = 1).  Random numbers: Philox4x32-10 (Salmon et al.,
// SC'11) keyed by the seed, counter (lexicographic site, sweep,
// subgroup<<16 | call, 0x48420000); float64 uniforms take 27+26 bits of two
// words, float32 ones 24 bits of one word.

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

constexpr uint32_t HB_STREAM_TAG = 0x48420000u;
constexpr int HB_MAX_ATTEMPTS = 128;

__device__ __forceinline__ void uniform_pair(const uint32_t w[4], double* a, double* b)
{
    *a = ((double)(w[0] >> 5) * 67108864.0 + (double)(w[1] >> 6) + 0.5) * (1.0 / 9007199254740992.0);
    *b = ((double)(w[2] >> 5) * 67108864.0 + (double)(w[3] >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void uniform_pair(const uint32_t w[4], float* a, float* b)
{
    *a = ((float)(w[0] >> 8) + 0.5f) * (1.0f / 16777216.0f);
    *b = ((float)(w[2] >> 8) + 0.5f) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ double hb_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float hb_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double hb_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float hb_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double hb_log(double x) { return log(x); }
__device__ __forceinline__ float hb_log(float x) { return logf(x); }
__device__ __forceinline__ double hb_cos(double x) { return cos(x); }
__device__ __forceinline__ float hb_cos(float x) { return cosf(x); }
__device__ __forceinline__ double hb_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float hb_sqrt(float x) { return sqrtf(x); }

template <typename R>
struct HBStream {
    uint32_t key0, key1, site, sweep, subgroup, call;

    __device__ __forceinline__ void draw2(R* a, R* b)
    {
        uint32_t w[4];
        philox4x32_10(site, sweep, (subgroup << 16) | call, HB_STREAM_TAG, key0, key1, w);
        ++call;
        uniform_pair(w, a, b);
    }
};

template <typename R>
__device__ __forceinline__ R hb_sample_r0(HBStream<R>& st, R kappa)
{
    const R two_pi = R(6.283185307179586476925286766559);
    for (int attempt = 0; attempt < HB_MAX_ATTEMPTS; ++attempt) {
        if (kappa < R(2)) {
            R u1, u2;
            st.draw2(&u1, &u2);
            const R r0 = kappa == R(0) ? R(2) * u1 - R(1)
                                       : R(1) + hb_log1p((R(1) - u1) * hb_expm1(R(-2) * kappa)) / kappa;
            if (u2 * u2 <= R(1) - r0 * r0) return r0;
        } else {
            R u1, u2, u3, u4;
            st.draw2(&u1, &u2);
            st.draw2(&u3, &u4);
            const R c = hb_cos(two_pi * u2);
            const R lam2 = -(hb_log(u1) + c * c * hb_log(u3)) / (R(2) * kappa);
            if (u4 * u4 <= R(1) - lam2) return R(1) - R(2) * lam2;
        }
    }
    return R(1);
}

template <typename R>
__device__ __forceinline__ Quat<R> hb_element(const Quat<R>& a, const Rule<R>& rule, uint32_t lex, uint32_t sg)
{
    const R two_pi = R(6.283185307179586476925286766559);
    HBStream<R> st{rule.key0, rule.key1, lex, rule.sweep, sg, 0u};
    const R n2 = fmad(a.b0, a.b0, fmad(a.b1, a.b1, fmad(a.b2, a.b2, a.b3 * a.b3)));
    const R n = hb_sqrt(n2);
    const R kappa = n2 > R(0) ? n / rule.T : R(0);
    const R r0 = hb_sample_r0(st, kappa);
    R u5, u6;
    st.draw2(&u5, &u6);
    const R ct = R(2) * u5 - R(1);
    const R stt = hb_sqrt(fmax(R(0), R(1) - ct * ct));
    R sp, cp;
    sin_cos(two_pi * u6, &sp, &cp);
    const R rr = hb_sqrt(fmax(R(0), R(1) - r0 * r0));
    Quat<R> w;
    w.b0 = r0;
    w.b1 = rr * stt * cp;
    w.b2 = rr * stt * sp;
    w.b3 = rr * ct;
    if (!(n2 > R(0))) return w;
    // w o qhat^dag, qhat^dag = (a0, -a1, -a2, -a3)/|a|; (p o q) = (p0 q0 - p.q, p0 q + q0 p - p x q)
    const R inv = R(1) / n;
    const R g0 = a.b0 * inv, g1 = -a.b1 * inv, g2 = -a.b2 * inv, g3 = -a.b3 * inv;
    Quat<R> b;
    b.b0 = fmad(w.b0, g0, -fmad(w.b1, g1, fmad(w.b2, g2, w.b3 * g3)));
    b.b1 = fmad(w.b0, g1, fmad(g0, w.b1, -fmad(w.b2, g3, -(w.b3 * g2))));
    b.b2 = fmad(w.b0, g2, fmad(g0, w.b2, -fmad(w.b3, g1, -(w.b1 * g3))));
    b.b3 = fmad(w.b0, g3, fmad(g0, w.b3, -fmad(w.b1, g2, -(w.b2 * g1))));
    return b;
}

template <int MODE, typename R>
__device__ __forceinline__ Quat<R> subgroup_element(const Quat<R>& a, const Rule<R>& rule, uint32_t lex, uint32_t sg)
{
    if constexpr (MODE == HEATBATH)
        return hb_element(a, rule, lex, sg);
    else
        return or_element<MODE>(a, rule.omega);
}

// Directions summed into K(x): 4 for Landau gauge, 3 (x, y, z) for Coulomb
// gauge, whose functional is that of Sec. 2 restricted to the spatial links,
// one independent problem per timeslice.  The gauge transformation of a
// Coulomb site update still acts on all 8 links at the site.
constexpr int NDIR_LANDAU = 4;
constexpr int NDIR_COULOMB = 3;

// Leaf k of this lane: U (forward, bwd = false) or U^dagger (backward), or
// zero for a direction outside the first NDIR.  Sum of NL consecutive leaves
// in the fixed pairwise tree; the zero leaves keep the tree, and so K, the
// same bitwise for every number of lanes per site.
template <int NL, int NDIR, typename R>
__device__ __forceinline__ void leaf_tree(const M3<R>* U, const bool* bwd, const int* mu, M3<R>& out)
{
    if constexpr (NL == 1) {
        m_leaf(out, U[0], bwd[0]);
        if constexpr (NDIR < 4) {
            if (mu[0] >= NDIR) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        out.re[i][j] = R(0);
                        out.im[i][j] = R(0);
                    }
            }
        }
    } else {
        M3<R> right;
        leaf_tree<NL / 2, NDIR>(U, bwd, mu, out);
        leaf_tree<NL / 2, NDIR>(U + NL / 2, bwd + NL / 2, mu + NL / 2, right);
        m_add(out, right);
    }
}

// tr[Delta Delta^dag] for Delta = [(K - K^dag)/(2i)]_traceless, in float64
// from K of either precision: M = (K - K^dag)/(2i) has diagonal Im K_ii and
// off-diagonal ((Im K_ij + Im K_ji) - i (Re K_ij - Re K_ji)) / 2, and
// Delta = M - tr(M)/3 (equal to Eq. (landaugauge) with A_mu of Sec. 2, a g = 1).
template <typename T>
__device__ __forceinline__ double delta_norm2(const M3<T>& K)
{
    const double d0 = (double)K.im[0][0], d1 = (double)K.im[1][1], d2 = (double)K.im[2][2];
    const double tr3 = (d0 + d1 + d2) / 3.0;
    const double e0 = d0 - tr3, e1 = d1 - tr3, e2 = d2 - tr3;
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            const double mr = 0.5 * ((double)K.im[i][j] + (double)K.im[j][i]);
            const double mi = 0.5 * ((double)K.re[i][j] - (double)K.re[j][i]);
            off += mr * mr + mi * mi;
        }
    return e0 * e0 + e1 * e1 + e2 * e2 + 2.0 * off;
}

// One site update of the site (parity, h) by lane r of its TPS-lane group.
// TRACKG (float32 mixed-precision bulk): also g(x) <- G g(x) for the float32
// gauge transformation accumulated since the original links; lane r of the
// group stores the chunks c with c % TPS == r.  NDIR: directions in K (Landau
// 4, Coulomb 3); all 8 links are transformed either way.  With est, lane 0 of
// the group returns tr[Delta Delta^dag] of the site's K before the update (the
// gauge-condition term of the configuration the site sees), every other lane
// and every call without est 0.  F: the link field, 12 reals per link
// (LinkField<R>) or 8 reals (Link8Field for float64, Link8Field32 for
// float32; decoded on load and encoded on store, in R).
template <typename R, int TPS, int MODE, bool TRACKG, int CP = 0, int NDIR = NDIR_LANDAU, typename F = LinkField<R>>
__device__ __forceinline__ double site_update(const F& f, const Geom& g, int parity, uint32_t h, int r,
                                              const Rule<R>& rule, const GField& gacc, bool est = false)
{
    constexpr bool kMin8 = Min8Of<F>::value;
    constexpr int NL = 8 / TPS;
    const Site s = decode_site(g, parity, h);
    const uint32_t lex = 2 * h + (uint32_t)(s.x & 1);

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
    if constexpr (kMin8) {
        static_assert(std::is_same<R, typename Min8Of<F>::R>::value, "decoded in the field's precision");
        // every load first, then the decodes (each yields SU(3) to rounding)
        typename Min8Of<F>::C raw[NL][Min8Of<F>::N];
#pragma unroll
        for (int k = 0; k < NL; ++k)
            load_min8_raw<nt_loads(CP)>(f, bwd[k] ? 1 - parity : parity, mu_of[k], at[k], raw[k]);
#pragma unroll
        for (int k = 0; k < NL; ++k) decode_min8(raw[k], U[k]);
    } else {
#pragma unroll
        for (int k = 0; k < NL; ++k)
            load_rows01<nt_loads(CP)>(f, bwd[k] ? 1 - parity : parity, mu_of[k], at[k], U[k]);
        // Row 2 is rebuilt from the two stored rows, so a departure d from unitarity
        // of those rows becomes up to ~2d after an update that mixes the rows.  Every
        // heat-bath update mixes them strongly (d would grow ~1.35x per sweep), so the
        // heat bath re-orthonormalises the two rows on load.  Overrelaxation mixes
        // them little (its subgroup elements approach 1; d grows ~1.004x per sweep on
        // rough inputs) and relies on the periodic reunitarisation of the fix-until
        // loop, which keeps its register footprint (and occupancy) unchanged.
        if constexpr (MODE == HEATBATH) {
#pragma unroll
            for (int k = 0; k < NL; ++k) gram_schmidt_rows01(U[k]);
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) rebuild_row2(U[k]);
    }

    M3<R> K;
    leaf_tree<NL, NDIR>(U, bwd, mu_of, K);
    if constexpr (TPS >= 2) dpp_accumulate<DPP_XOR1>(K);
    if constexpr (TPS >= 4) dpp_accumulate<DPP_XOR2>(K);
    if constexpr (TPS >= 8) dpp_accumulate<DPP_HALF_MIRROR>(K);
    const double th = (est && r == 0) ? delta_norm2(K) : 0.0;

    M3<R> G;
    {
        const Quat<R> b = subgroup_element<MODE>(block_quaternion<0, 1>(K), rule, lex, 0u);
        set_embedding<0, 1>(b, G);
        rotate_rows<0, 1>(b, K);
    }
    {
        const Quat<R> b = subgroup_element<MODE>(block_quaternion<0, 2>(K), rule, lex, 1u);
        rotate_rows<0, 2>(b, G);
        rotate_rows<0, 2>(b, K);
    }
    {
        const Quat<R> b = subgroup_element<MODE>(block_quaternion<1, 2>(K), rule, lex, 2u);
        rotate_rows<1, 2>(b, G);
    }

#pragma unroll
    for (int k = 0; k < NL; ++k) {
        if (bwd[k])
            right_mul_dag_rows01(G, U[k]);
        else
            left_mul_rows01(G, U[k]);
        store_link<nt_stores(CP)>(f, bwd[k] ? 1 - parity : parity, mu_of[k], at[k], U[k]);
    }

    if constexpr (TRACKG) {
        M3<R> gx;
        load_g(gacc, parity, h, gx);
        gram_schmidt_rows01(gx);  // g is only ever multiplied: keep it in SU(3) (see above)
        rebuild_row2(gx);
        left_mul_rows01(G, gx);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (c % TPS == r) store_g_chunk(gacc, parity, h, c, gx);
    }
    return th;
}

// ------------------------------------------------------------- reductions --

template <typename R>
__device__ __forceinline__ void load_full_f64(const LinkField<R>& f, int parity, int mu, uint32_t h, M3<double>& u)
{
    M3<R> t;
    load_rows01(f, parity, mu, h, t);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            u.re[i][j] = (double)t.re[i][j];
            u.im[i][j] = (double)t.im[i][j];
        }
    rebuild_row2(u);
}

// Links read in place from the ABI's canonical float64 array
// [site][mu][row][col][re,im], lexicographic site x + Nx(y + Ny(z + Nz t)).
// The half index h of (parity, h) is lex >> 1 (Nx is even), so
// lex = 2h + (x & 1).  Rows 0 and 1 are read and row 2 is rebuilt from them,
// exactly as from the 12-real device layout, so every measurement over a
// CanonField equals the one over the packed float64 field of the same links.
struct CanonField {
    const double* base;
    Geom g;
};

__device__ __forceinline__ void load_full_f64(const CanonField& f, int parity, int mu, uint32_t h, M3<double>& u)
{
    const Site s = decode_site(f.g, parity, h);
    const size_t lex = 2 * (size_t)h + (size_t)(s.x & 1);
    const double2* p = (const double2*)(f.base + (lex * 4 + (size_t)mu) * 18);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double2 v = p[c];
        u.re[c / 3][c % 3] = v.x;
        u.im[c / 3][c % 3] = v.y;
    }
    rebuild_row2(u);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum two values over the block; thread 0 writes them to out[0..1].
template <int NT>
__device__ __forceinline__ void block_sum2(double a, double b, double* out)
{
    __shared__ double lds[2][NT / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        lds[0][w] = a;
        lds[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int i = 0; i < NT / 64; ++i) {
            sa += lds[0][i];
            sb += lds[1][i];
        }
        out[0] = sa;
        out[1] = sb;
    }
}

// out[k] = scale[k] * sum_i partial[2 i + k] over n pairs, summed in a fixed
// order by one block of NT threads (the caller synchronises before reading out).
template <int NT>
__device__ __forceinline__ void finalize_pairs(const double* partial, uint32_t n, double s0, double s1, double* out)
{
    double a = 0.0, b = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += NT) {
        a += partial[2 * (size_t)i];
        b += partial[2 * (size_t)i + 1];
    }
    __shared__ double res[2];
    block_sum2<NT>(a, b, res);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = res[0] * s0;
        out[1] = res[1] * s1;
    }
}

// Gauge-condition and functional terms of the site (parity, h), float64:
// th = tr[Delta Delta^dag] with Delta = [(K - K^dag)/(2i)]_traceless (equal to
// Eq. (landaugauge) with A_mu of Sec. 2, a g = 1), fr = sum_mu Re tr U_mu(x),
// mu over the first NDIR directions (Landau 4; Coulomb 3, the spatial Delta_C
// and functional of one timeslice).
template <int NDIR = NDIR_LANDAU, typename Field>
__device__ __forceinline__ void measure_site(const Field& f, const Geom& g, int parity, uint32_t h, double& th,
                                             double& fr)
{
    const Site s = decode_site(g, parity, h);
    M3<double> K;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            K.re[i][j] = 0.0;
            K.im[i][j] = 0.0;
        }
#pragma unroll
    for (int mu = 0; mu < NDIR; ++mu) {
        M3<double> u;
        load_full_f64(f, parity, mu, h, u);
        fr += u.re[0][0] + u.re[1][1] + u.re[2][2];
        m_add(K, u);
        load_full_f64(f, 1 - parity, mu, back_h(g, h, s, mu), u);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                K.re[i][j] += u.re[j][i];
                K.im[i][j] -= u.im[j][i];
            }
    }
    th = delta_norm2(K);
}

}  // namespace gf
