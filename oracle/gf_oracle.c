/*
 * gf_oracle.c -- plain FP64 CPU oracle for SU(3) lattice Landau gauge fixing
 * by checkerboard overrelaxation, written from H. Vogt and M. Schroeck,
 * "cuLGT: Lattice Gauge Fixing on GPUs" (arXiv:1412.3655), Sec. 2.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this library.  The HIP product library
 * shares no code with it (no headers, no helpers, no tables) and never calls
 * it.
 *
 * Conventions
 *   - IEEE double everywhere, C99 complex, built without fast-math and with
 *     FP contraction off.
 *   - Full 3x3 links (18 reals) in the canonical layout
 *     U[site][mu][row][col][re,im], site = x + Nx*(y + Ny*(z + Nz*t)),
 *     mu = 0..3 for x, y, z, t; U[site][mu] is U_mu(x).
 *   - Periodic boundaries, all extents even (the checkerboard needs a
 *     bipartite periodic lattice).
 *
 * What each part follows
 *   transform_site ......... the gauge transformation of a link, Sec. 2
 *                            (first displayed equation) with g = 1 away from x.
 *   local_K ................ K(x) of Eq. (localfunctional).
 *   oracle_su2_maximiser ... the SU(2) maximiser g = K^dag / sqrt(det K^dag)
 *                            (Sec. 2), applied to the SU(2)-span projection of
 *                            a 2x2 subgroup block of K.
 *   or_site_update ......... iteration over the SU(2) subgroups for N_c > 2
 *                            and the overrelaxation g -> g^omega (Sec. 2).
 *   oracle_half_sweep /
 *   oracle_sweep ........... black-then-white checkerboard sweep (Sec. 2).
 *   gauge_potential ........ A_mu of Sec. 2 with a*g = 1.
 *   oracle_measure ......... Delta(x) of Eq. (landaugauge), its norm theta,
 *                            and F of Eq. (landaufunctional) with g = 1 (the
 *                            links already carry the accumulated transform).
 *   oracle_fix_until ....... "iterated until the gauge condition holds to a
 *                            given precision" (Sec. 2, last paragraph).
 *   oracle_anneal .......... simulated-annealing prelude named in the
 *                            abstract; the paper gives no algorithm, so it is
 *                            the standard SU(2)-subgroup heat bath (Creutz
 *                            sampler for small kappa, Kennedy-Pendleton above)
 *                            driven by Philox4x32-10 (Salmon et al., SC'11).
 *   oracle_coulomb_* ....... Coulomb gauge (abstract, Sec. 1): the same
 *                            iteration with K, Delta and F over the spatial
 *                            directions only, per timeslice; the heat-bath
 *                            prelude of the Coulomb functional likewise.
 *   oracle_su2lat_* ........ the same method for gauge group SU(2) (abstract;
 *                            Sec. 2's maximiser applies to K directly, Sec.
 *                            4.1 swaps the group by the parameterisation).
 *   oracle_reunitarize ..... Gram-Schmidt of rows 0 and 1, row 2 rebuilt as
 *                            the conjugated cross product (the two-row
 *                            representation of Sec. 3.1 keeps row 2 implicit).
 *   oracle_plaquette ....... the gauge-invariant average plaquette, used to
 *                            check that sweeps stay on the gauge orbit.
 *   oracle_min8_* .......... the minimal 8-parameter SU(3) representation
 *                            that Sec. 4.1 names (the paper gives no
 *                            formulae; see the definition at the functions).
 *
 * Readings taken where the paper is silent (each also listed in the design
 * notes of the repository):
 *   - subgroups (0,1), (0,2), (1,2), in that order, one pass per site update;
 *     K is recomputed from the current links before every subgroup step;
 *   - a 2x2 block k of K is replaced by its projection q = (k + s2 k* s2)/2
 *     onto the real span of SU(2) before the maximiser (Re tr[g k] =
 *     Re tr[g q] for every g in SU(2)); det q = 0 skips the subgroup;
 *   - g^omega: EXACT is the principal SU(2) power cos(w phi) 1 +
 *     (sin(w phi)/sin(phi)) (g - cos(phi) 1); BINOMIAL1 is
 *     (1 - w) 1 + w g renormalised onto SU(2);
 *   - black = even (x+y+z+t), swept first;
 *   - theta = (1/(N_c V)) sum_x tr[Delta(x) Delta(x)^dag].
 */

#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cx;

enum { OR_EXACT = 0, OR_BINOMIAL1 = 1 };

/* Lattices smaller than this are processed by one thread (thread start-up
 * would dominate); the results do not depend on the thread count. */
#define OMP_MIN_SITES 32768

/* ------------------------------------------------------------------ */
/* lattice geometry                                                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int n[4];
    long V;
} geom;

static geom mkgeom(const int32_t* dims)
{
    geom g;
    g.V = 1;
    for (int m = 0; m < 4; ++m) {
        g.n[m] = dims[m];
        g.V *= dims[m];
    }
    return g;
}

static void coords_of(const geom* g, long s, int x[4])
{
    for (int m = 0; m < 4; ++m) {
        x[m] = (int)(s % g->n[m]);
        s /= g->n[m];
    }
}

static long site_of(const geom* g, const int x[4])
{
    return x[0] + (long)g->n[0] * (x[1] + (long)g->n[1] * (x[2] + (long)g->n[2] * x[3]));
}

/* neighbour s + step * mu^ (step = +1 or -1), periodic */
static long hop(const geom* g, long s, int mu, int step)
{
    int x[4];
    coords_of(g, s, x);
    x[mu] = (x[mu] + step + g->n[mu]) % g->n[mu];
    return site_of(g, x);
}

static int colour_of(const geom* g, long s)
{
    int x[4];
    coords_of(g, s, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

static cx* link_at(double* U, long s, int mu)
{
    return (cx*)(U + ((size_t)s * 4 + (size_t)mu) * 18);
}

static const cx* clink_at(const double* U, long s, int mu)
{
    return (const cx*)(U + ((size_t)s * 4 + (size_t)mu) * 18);
}

/* ------------------------------------------------------------------ */
/* 3x3 complex matrices, row-major cx[9]                               */
/* ------------------------------------------------------------------ */

static void m_zero(cx* a)
{
    for (int i = 0; i < 9; ++i) a[i] = 0.0;
}

static void m_unit(cx* a)
{
    m_zero(a);
    a[0] = a[4] = a[8] = 1.0;
}

static void m_copy(cx* d, const cx* s)
{
    memcpy(d, s, 9 * sizeof(cx));
}

static void m_dag(cx* d, const cx* s)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) d[3 * i + j] = conj(s[3 * j + i]);
}

/* c = a b; c must not alias a or b */
static void m_mul(cx* c, const cx* a, const cx* b)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cx acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = acc;
        }
}

static double m_retr(const cx* a)
{
    return creal(a[0]) + creal(a[4]) + creal(a[8]);
}

/* ------------------------------------------------------------------ */
/* the local problem at one site                                       */
/* ------------------------------------------------------------------ */

/* K(x) = sum_mu [ U_mu(x) + U_mu(x - mu^)^dagger ]   (Eq. localfunctional),
 * mu over the first ndir directions: 4 for Landau gauge, 3 (x, y, z) for
 * Coulomb gauge. */
static void local_K(const double* U, const geom* g, long s, int ndir, cx* K)
{
    m_zero(K);
    for (int mu = 0; mu < ndir; ++mu) {
        const cx* f = clink_at(U, s, mu);
        const cx* b = clink_at(U, hop(g, s, mu, -1), mu);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) K[3 * i + j] += f[3 * i + j] + conj(b[3 * j + i]);
    }
}

/* Gauge transformation with g(x) = S at site s and g = 1 everywhere else:
 * U_mu(s) <- S U_mu(s) and U_mu(s - mu^) <- U_mu(s - mu^) S^dagger. */
static void transform_site(double* U, const geom* g, long s, const cx* S)
{
    cx Sd[9], T[9];
    m_dag(Sd, S);
    for (int mu = 0; mu < 4; ++mu) {
        cx* f = link_at(U, s, mu);
        m_mul(T, S, f);
        m_copy(f, T);
        cx* b = link_at(U, hop(g, s, mu, -1), mu);
        m_mul(T, b, Sd);
        m_copy(b, T);
    }
}

/* 2x2 complex matrices are cx[4] = {m00, m01, m10, m11}. */

/* Projection onto the real span of SU(2): q = (k + s2 conj(k) s2) / 2. */
void oracle_su2_project(const double* k_in, double* q_out)
{
    const cx* k = (const cx*)k_in;
    cx q[4];
    q[0] = 0.5 * (k[0] + conj(k[3]));
    q[1] = 0.5 * (k[1] - conj(k[2]));
    q[2] = 0.5 * (k[2] - conj(k[1]));
    q[3] = 0.5 * (k[3] + conj(k[0]));
    memcpy(q_out, q, sizeof q);
}

/* Maximiser of Re tr[g k] over g in SU(2): g = q^dag / sqrt(det q^dag) with q
 * the projection of k.  Returns 0 (and g = 1) when det q = 0. */
int oracle_su2_maximiser(const double* k_in, double* g_out)
{
    cx q[4];
    oracle_su2_project(k_in, (double*)q);
    cx qd[4] = {conj(q[0]), conj(q[2]), conj(q[1]), conj(q[3])};
    cx det = qd[0] * qd[3] - qd[1] * qd[2];
    cx* g = (cx*)g_out;
    if (cabs(det) == 0.0) {
        g[0] = 1.0;
        g[1] = 0.0;
        g[2] = 0.0;
        g[3] = 1.0;
        return 0;
    }
    cx root = csqrt(det);
    for (int i = 0; i < 4; ++i) g[i] = qd[i] / root;
    return 1;
}

/* Overrelaxation of an SU(2) element, g -> g^omega.
 * EXACT: with cos(phi) = tr(g)/2 and sin(phi) = sqrt(det(g - cos(phi) 1)),
 *   g^omega = cos(omega phi) 1 + sin(omega phi)/sin(phi) (g - cos(phi) 1),
 *   phi in [0, pi] (principal power along the one-parameter subgroup).
 * BINOMIAL1: (1 - omega) 1 + omega g, renormalised onto SU(2). */
void oracle_su2_overrelax(const double* g_in, double omega, int mode, double* out)
{
    const cx* g = (const cx*)g_in;
    cx h[4];
    if (mode == OR_EXACT) {
        double c0 = 0.5 * creal(g[0] + g[3]);
        cx a[4] = {g[0] - c0, g[1], g[2], g[3] - c0};
        double s2 = creal(a[0] * a[3] - a[1] * a[2]);
        double sphi = s2 > 0.0 ? sqrt(s2) : 0.0;
        if (sphi == 0.0) {
            memcpy(h, g, sizeof h);
        } else {
            double phi = atan2(sphi, c0);
            double cw = cos(omega * phi);
            double sw = sin(omega * phi) / sphi;
            h[0] = cw + sw * a[0];
            h[1] = sw * a[1];
            h[2] = sw * a[2];
            h[3] = cw + sw * a[3];
        }
    } else {
        h[0] = (1.0 - omega) + omega * g[0];
        h[1] = omega * g[1];
        h[2] = omega * g[2];
        h[3] = (1.0 - omega) + omega * g[3];
        cx det = h[0] * h[3] - h[1] * h[2];
        cx root = csqrt(det);
        for (int i = 0; i < 4; ++i) h[i] /= root;
    }
    memcpy(out, h, sizeof h);
}

static const int SUBGROUP[3][2] = {{0, 1}, {0, 2}, {1, 2}};

static void block_of(const cx* K, int i, int j, cx* k)
{
    k[0] = K[3 * i + i];
    k[1] = K[3 * i + j];
    k[2] = K[3 * j + i];
    k[3] = K[3 * j + j];
}

static void embed(const cx* g2, int i, int j, cx* S)
{
    m_unit(S);
    S[3 * i + i] = g2[0];
    S[3 * i + j] = g2[1];
    S[3 * j + i] = g2[2];
    S[3 * j + j] = g2[3];
}

/* One overrelaxation update of site s; returns the change of Re tr K(x).  K
 * sums the first ndir directions; the transformation acts on all 8 links at
 * s (a gauge transformation, Sec. 2). */
static double or_site_update(double* U, const geom* g, long s, double omega, int mode, int ndir)
{
    double gain = 0.0;
    for (int sg = 0; sg < 3; ++sg) {
        int i = SUBGROUP[sg][0], j = SUBGROUP[sg][1];
        cx K[9], k[4], g2[4], S[9], SK[9];
        local_K(U, g, s, ndir, K);
        block_of(K, i, j, k);
        if (!oracle_su2_maximiser((const double*)k, (double*)g2)) continue;
        oracle_su2_overrelax((const double*)g2, omega, mode, (double*)g2);
        embed(g2, i, j, S);
        m_mul(SK, S, K);
        gain += m_retr(SK) - m_retr(K);
        transform_site(U, g, s, S);
    }
    return gain;
}

double oracle_site_update(double* U, const int32_t* dims, int64_t site, double omega, int mode)
{
    geom g = mkgeom(dims);
    return or_site_update(U, &g, (long)site, omega, mode, 4);
}

/* Update every site of one colour (0 = black = even x+y+z+t).  Sites of one
 * colour share no link, so the order inside the colour does not matter. */
void oracle_half_sweep(double* U, const int32_t* dims, int colour, double omega, int mode)
{
    geom g = mkgeom(dims);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s)
        if (colour_of(&g, s) == colour) or_site_update(U, &g, s, omega, mode, 4);
}

/* Sequential updates in a caller-given order (for the order-independence check). */
void oracle_update_sites_in_order(double* U, const int32_t* dims, const int64_t* sites, int64_t n,
                                  double omega, int mode)
{
    geom g = mkgeom(dims);
    for (int64_t i = 0; i < n; ++i) or_site_update(U, &g, (long)sites[i], omega, mode, 4);
}

void oracle_sweep(double* U, const int32_t* dims, int32_t nsweeps, double omega, int mode)
{
    for (int32_t k = 0; k < nsweeps; ++k) {
        oracle_half_sweep(U, dims, 0, omega, mode);
        oracle_half_sweep(U, dims, 1, omega, mode);
    }
}

/* ------------------------------------------------------------------ */
/* measurements                                                        */
/* ------------------------------------------------------------------ */

/* A_mu = [(U - U^dag) / (2i)]_traceless   (a g = 1) */
static void gauge_potential(const cx* u, cx* A)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[3 * i + j] = (u[3 * i + j] - conj(u[3 * j + i])) / (2.0 * I);
    cx tr = (A[0] + A[4] + A[8]) / 3.0;
    A[0] -= tr;
    A[4] -= tr;
    A[8] -= tr;
}

/* tr[Delta(x) Delta(x)^dag] with Delta(x) = sum_mu (A_mu(x) - A_mu(x - mu^)),
 * mu over the first ndir directions (4: Landau, 3: Coulomb). */
static double theta_site(const double* U, const geom* g, long s, int ndir)
{
    cx D[9], A[9], Dd[9], P[9];
    m_zero(D);
    for (int mu = 0; mu < ndir; ++mu) {
        gauge_potential(clink_at(U, s, mu), A);
        for (int i = 0; i < 9; ++i) D[i] += A[i];
        gauge_potential(clink_at(U, hop(g, s, mu, -1), mu), A);
        for (int i = 0; i < 9; ++i) D[i] -= A[i];
    }
    m_dag(Dd, D);
    m_mul(P, D, Dd);
    return m_retr(P);
}

void oracle_theta_density(const double* U, const int32_t* dims, double* out)
{
    geom g = mkgeom(dims);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s) out[s] = theta_site(U, &g, s, 4);
}

/* theta = (1/(N_c V)) sum_x tr[Delta Delta^dag],
 * F = (1/(N_d N_c V)) sum_x sum_mu Re tr U_mu(x).
 * Per-site terms are summed in site order, so the result does not depend on
 * the thread count. */
void oracle_measure(const double* U, const int32_t* dims, double* theta, double* F)
{
    geom g = mkgeom(dims);
    double* th = (double*)malloc(sizeof(double) * (size_t)g.V);
    double* fr = (double*)malloc(sizeof(double) * (size_t)g.V);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s) {
        th[s] = theta_site(U, &g, s, 4);
        double f = 0.0;
        for (int mu = 0; mu < 4; ++mu) f += m_retr(clink_at(U, s, mu));
        fr[s] = f;
    }
    double st = 0.0, sf = 0.0;
    for (long s = 0; s < g.V; ++s) {
        st += th[s];
        sf += fr[s];
    }
    free(th);
    free(fr);
    *theta = st / (3.0 * (double)g.V);
    *F = sf / (12.0 * (double)g.V);
}

/* P = (1/(18 V)) sum_x sum_{mu<nu} Re tr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag] */
double oracle_plaquette(const double* U, const int32_t* dims)
{
    geom g = mkgeom(dims);
    double* ps = (double*)malloc(sizeof(double) * (size_t)g.V);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s) {
        double acc = 0.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cx a[9], b[9], t1[9], t2[9], d[9];
                m_mul(t1, clink_at(U, s, mu), clink_at(U, hop(&g, s, mu, +1), nu));
                m_dag(a, clink_at(U, hop(&g, s, nu, +1), mu));
                m_mul(t2, t1, a);
                m_dag(b, clink_at(U, s, nu));
                m_mul(d, t2, b);
                acc += m_retr(d);
            }
        ps[s] = acc;
    }
    double sum = 0.0;
    for (long s = 0; s < g.V; ++s) sum += ps[s];
    free(ps);
    return sum / (18.0 * (double)g.V);
}

/* max over links of ||U^dag U - 1||_F and |det U - 1| */
void oracle_unitarity(const double* U, int64_t nlinks, double* max_unit, double* max_det)
{
    double mu = 0.0, md = 0.0;
    for (int64_t l = 0; l < nlinks; ++l) {
        const cx* u = (const cx*)(U + (size_t)l * 18);
        cx ud[9], p[9];
        m_dag(ud, u);
        m_mul(p, ud, u);
        double fro = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                cx e = p[3 * i + j] - (i == j ? 1.0 : 0.0);
                fro += creal(e * conj(e));
            }
        fro = sqrt(fro);
        cx det = u[0] * (u[4] * u[8] - u[5] * u[7]) - u[1] * (u[3] * u[8] - u[5] * u[6]) +
                 u[2] * (u[3] * u[7] - u[4] * u[6]);
        double dd = cabs(det - 1.0);
        if (fro > mu) mu = fro;
        if (dd > md) md = dd;
    }
    *max_unit = mu;
    *max_det = md;
}

/* ------------------------------------------------------------------ */
/* reunitarisation and gauge transformation                            */
/* ------------------------------------------------------------------ */

void oracle_reunitarize(double* U, int64_t nlinks)
{
#pragma omp parallel for schedule(static) if (nlinks >= 4 * OMP_MIN_SITES)
    for (int64_t l = 0; l < nlinks; ++l) {
        cx* u = (cx*)(U + (size_t)l * 18);
        cx* r0 = u;
        cx* r1 = u + 3;
        cx* r2 = u + 6;
        double n0 = 0.0;
        for (int i = 0; i < 3; ++i) n0 += creal(r0[i] * conj(r0[i]));
        n0 = sqrt(n0);
        for (int i = 0; i < 3; ++i) r0[i] /= n0;
        cx ip = 0.0;
        for (int i = 0; i < 3; ++i) ip += conj(r0[i]) * r1[i];
        for (int i = 0; i < 3; ++i) r1[i] -= ip * r0[i];
        double n1 = 0.0;
        for (int i = 0; i < 3; ++i) n1 += creal(r1[i] * conj(r1[i]));
        n1 = sqrt(n1);
        for (int i = 0; i < 3; ++i) r1[i] /= n1;
        r2[0] = conj(r0[1] * r1[2] - r0[2] * r1[1]);
        r2[1] = conj(r0[2] * r1[0] - r0[0] * r1[2]);
        r2[2] = conj(r0[0] * r1[1] - r0[1] * r1[0]);
    }
}

/* U_mu(x) <- G(x) U_mu(x) G(x + mu^)^dag for a full gauge field G[site][3][3][2] */
void oracle_gauge_transform(double* U, const int32_t* dims, const double* G)
{
    geom g = mkgeom(dims);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s) {
        const cx* gx = (const cx*)(G + (size_t)s * 18);
        for (int mu = 0; mu < 4; ++mu) {
            const cx* gy = (const cx*)(G + (size_t)hop(&g, s, mu, +1) * 18);
            cx gyd[9], t[9];
            m_dag(gyd, gy);
            cx* u = link_at(U, s, mu);
            m_mul(t, gx, u);
            m_mul(u, t, gyd);
        }
    }
}

/* ------------------------------------------------------------------ */
/* fix until the gauge condition holds                                 */
/* ------------------------------------------------------------------ */

/* Measure; then, while theta >= target and fewer than max_sweeps sweeps were
 * done, do min(check_every, remaining) sweeps (reunitarising after every sweep
 * whose count is a multiple of reunit_every, if reunit_every > 0) and measure
 * again.  theta_hist (optional) receives theta at every check, starting with
 * the initial one; its length is written to *n_checks.  Returns 1 when
 * converged (theta < target). */
int oracle_fix_until(double* U, const int32_t* dims, double omega, int mode, double theta_target,
                     int32_t max_sweeps, int32_t check_every, int32_t reunit_every, int32_t* sweeps_out,
                     double* theta_out, double* F_out, double* theta_hist, int32_t* n_checks)
{
    geom g = mkgeom(dims);
    double theta, F;
    int32_t sweeps = 0, checks = 0;
    oracle_measure(U, dims, &theta, &F);
    if (theta_hist) theta_hist[checks] = theta;
    ++checks;
    while (theta >= theta_target && sweeps < max_sweeps) {
        int32_t n = max_sweeps - sweeps < check_every ? max_sweeps - sweeps : check_every;
        for (int32_t k = 0; k < n; ++k) {
            oracle_sweep(U, dims, 1, omega, mode);
            ++sweeps;
            if (reunit_every > 0 && sweeps % reunit_every == 0) oracle_reunitarize(U, 4 * (int64_t)g.V);
        }
        oracle_measure(U, dims, &theta, &F);
        if (theta_hist) theta_hist[checks] = theta;
        ++checks;
    }
    *sweeps_out = sweeps;
    *theta_out = theta;
    *F_out = F;
    if (n_checks) *n_checks = checks;
    return theta < theta_target;
}

/* ------------------------------------------------------------------ */
/* Coulomb gauge                                                       */
/* ------------------------------------------------------------------ */

/* Coulomb gauge (abstract and Sec. 1 list it beside Landau gauge): the
 * condition and functional of Sec. 2 with mu restricted to the spatial
 * directions x, y, z.  The functional sum_x sum_i Re tr[g(x) U_i(x)
 * g(x+i^)^dag] decouples into one independent problem per timeslice, so the
 * site update maximises Re tr[g(x) K_C(x)] with K_C(x) = sum_i [U_i(x) +
 * U_i(x-i^)^dag]; g(x) is a gauge transformation and acts on all 8 links at x,
 * the temporal ones included, which keeps the configuration on its gauge
 * orbit.  Per timeslice t (V_3 = Nx Ny Nz sites):
 *   theta_C(t) = (1/(N_c V_3)) sum_{x in t} tr[Delta_C Delta_C^dag],
 *   Delta_C(x) = sum_i (A_i(x) - A_i(x - i^)),
 *   F_C(t)     = (1/((N_d - 1) N_c V_3)) sum_{x in t} sum_i Re tr U_i(x). */

void oracle_coulomb_half_sweep(double* U, const int32_t* dims, int colour, double omega, int mode)
{
    geom g = mkgeom(dims);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s)
        if (colour_of(&g, s) == colour) or_site_update(U, &g, s, omega, mode, 3);
}

void oracle_coulomb_sweep(double* U, const int32_t* dims, int32_t nsweeps, double omega, int mode)
{
    for (int32_t k = 0; k < nsweeps; ++k) {
        oracle_coulomb_half_sweep(U, dims, 0, omega, mode);
        oracle_coulomb_half_sweep(U, dims, 1, omega, mode);
    }
}

/* Sequential Coulomb updates in a caller-given order. */
void oracle_coulomb_update_sites_in_order(double* U, const int32_t* dims, const int64_t* sites, int64_t n,
                                          double omega, int mode)
{
    geom g = mkgeom(dims);
    for (int64_t i = 0; i < n; ++i) or_site_update(U, &g, (long)sites[i], omega, mode, 3);
}

/* theta_C(t) and F_C(t) for every timeslice t = 0 .. Nt-1 (arrays of Nt);
 * per-site terms summed in site order. */
void oracle_coulomb_measure(const double* U, const int32_t* dims, double* theta_t, double* F_t)
{
    geom g = mkgeom(dims);
    const long V3 = g.V / g.n[3];
    double* th = (double*)malloc(sizeof(double) * (size_t)g.V);
    double* fr = (double*)malloc(sizeof(double) * (size_t)g.V);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s) {
        th[s] = theta_site(U, &g, s, 3);
        double f = 0.0;
        for (int i = 0; i < 3; ++i) f += m_retr(clink_at(U, s, i));
        fr[s] = f;
    }
    for (int t = 0; t < g.n[3]; ++t) {
        double st = 0.0, sf = 0.0;
        for (long s = (long)t * V3; s < (long)(t + 1) * V3; ++s) {
            st += th[s];
            sf += fr[s];
        }
        theta_t[t] = st / (3.0 * (double)V3);
        F_t[t] = sf / (9.0 * (double)V3);
    }
    free(th);
    free(fr);
}

/* As oracle_fix_until for Coulomb gauge: the stop test is max_t theta_C(t) <
 * target (every timeslice satisfies the condition).  *theta_out = that
 * maximum, *F_out = the mean of F_C(t) over timeslices. */
int oracle_coulomb_fix_until(double* U, const int32_t* dims, double omega, int mode, double theta_target,
                             int32_t max_sweeps, int32_t check_every, int32_t reunit_every, int32_t* sweeps_out,
                             double* theta_out, double* F_out)
{
    geom g = mkgeom(dims);
    const int nt = g.n[3];
    double* th = (double*)malloc(sizeof(double) * (size_t)nt);
    double* fr = (double*)malloc(sizeof(double) * (size_t)nt);
    double theta = 0.0, F = 0.0;
    int32_t sweeps = 0;
    for (;;) {
        oracle_coulomb_measure(U, dims, th, fr);
        theta = 0.0;
        F = 0.0;
        for (int t = 0; t < nt; ++t) {
            if (th[t] > theta) theta = th[t];
            F += fr[t];
        }
        F /= (double)nt;
        if (!(theta >= theta_target) || sweeps >= max_sweeps) break;
        int32_t n = max_sweeps - sweeps < check_every ? max_sweeps - sweeps : check_every;
        for (int32_t k = 0; k < n; ++k) {
            oracle_coulomb_sweep(U, dims, 1, omega, mode);
            ++sweeps;
            if (reunit_every > 0 && sweeps % reunit_every == 0) oracle_reunitarize(U, 4 * (int64_t)g.V);
        }
    }
    free(th);
    free(fr);
    *sweeps_out = sweeps;
    *theta_out = theta;
    *F_out = F;
    return theta < theta_target;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 and the heat-bath prelude                             */
/* ------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds, as published by Salmon, Moraes, Dror and Shaw
 * (SC'11): multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments
 * 0x9E3779B9 / 0xBB67AE85. */
void oracle_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

#define HB_STREAM_TAG 0x48420000u

/* Random stream of one subgroup update: counter (site, sweep, subgroup<<16 | call, tag). */
typedef struct {
    uint32_t key[2];
    uint32_t site, sweep, subgroup, call;
} hb_stream;

/* uniform in (0,1) from 53 bits: 27 of a, 26 of b */
static double u01_53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

static void hb_draw2(hb_stream* st, double* ua, double* ub)
{
    uint32_t ctr[4] = {st->site, st->sweep, (st->subgroup << 16) | st->call, HB_STREAM_TAG};
    uint32_t o[4];
    st->call++;
    oracle_philox4x32_10(ctr, st->key, o);
    *ua = u01_53(o[0], o[1]);
    *ub = u01_53(o[2], o[3]);
}

#define HB_MAX_ATTEMPTS 128

/* r0 in [-1,1] with density proportional to sqrt(1 - r0^2) exp(kappa r0).
 * kappa < 2: exponential proposal by inverse CDF, accepted with probability
 * sqrt(1 - r0^2) (Creutz).  kappa >= 2: Kennedy-Pendleton.  After
 * HB_MAX_ATTEMPTS rejections r0 = 1 and *capped is incremented. */
static double hb_sample_r0(hb_stream* st, double kappa, int* capped)
{
    for (int attempt = 0; attempt < HB_MAX_ATTEMPTS; ++attempt) {
        if (kappa < 2.0) {
            double u1, u2;
            hb_draw2(st, &u1, &u2);
            double r0 = kappa == 0.0 ? 2.0 * u1 - 1.0 : 1.0 + log1p((1.0 - u1) * expm1(-2.0 * kappa)) / kappa;
            if (u2 * u2 <= 1.0 - r0 * r0) return r0;
        } else {
            double u1, u2, u3, u4;
            hb_draw2(st, &u1, &u2);
            hb_draw2(st, &u3, &u4);
            double c = cos(2.0 * M_PI * u2);
            double lam2 = -(log(u1) + c * c * log(u3)) / (2.0 * kappa);
            if (u4 * u4 <= 1.0 - lam2) return 1.0 - 2.0 * lam2;
        }
    }
    ++*capped;
    return 1.0;
}

/* SU(2) element r = (r0, sqrt(1-r0^2) n) with n uniform on the sphere, as the
 * 2x2 matrix [[r0 + i r3, r2 + i r1], [-r2 + i r1, r0 - i r3]]. */
static void hb_sample_su2(hb_stream* st, double kappa, int* capped, cx* w)
{
    double r0 = hb_sample_r0(st, kappa, capped);
    double u5, u6;
    hb_draw2(st, &u5, &u6);
    double ct = 2.0 * u5 - 1.0;
    double stt = sqrt(fmax(0.0, 1.0 - ct * ct));
    double ph = 2.0 * M_PI * u6;
    double rr = sqrt(fmax(0.0, 1.0 - r0 * r0));
    double r1 = rr * stt * cos(ph), r2 = rr * stt * sin(ph), r3 = rr * ct;
    w[0] = r0 + I * r3;
    w[1] = r2 + I * r1;
    w[2] = -r2 + I * r1;
    w[3] = r0 - I * r3;
}

/* One subgroup element drawn from exp(Re tr[g k] / T) dHaar(g) for the 2x2
 * block k of K.  With q = n * qhat the SU(2)-span projection of k (qhat in
 * SU(2)), Re tr[g k] = Re tr[g q] = 2 n w0 for g = w qhat^dag, so w has
 * density exp(2 n w0 / T) dHaar(w): kappa = 2n/T; qhat^dag is the SU(2)
 * maximiser.  n = 0 draws g Haar-uniformly (kappa = 0). */
static void hb_subgroup_element(const cx* k, double T, hb_stream* st, int* capped, cx* g2)
{
    cx q[4], gm[4], w[4];
    oracle_su2_project((const double*)k, (double*)q);
    double det = creal(q[0] * q[3] - q[1] * q[2]);
    double n = det > 0.0 ? sqrt(det) : 0.0;
    if (n == 0.0) {
        hb_sample_su2(st, 0.0, capped, g2);
        return;
    }
    hb_sample_su2(st, 2.0 * n / T, capped, w);
    oracle_su2_maximiser((const double*)k, (double*)gm);
    g2[0] = w[0] * gm[0] + w[1] * gm[2];
    g2[1] = w[0] * gm[1] + w[1] * gm[3];
    g2[2] = w[2] * gm[0] + w[3] * gm[2];
    g2[3] = w[2] * gm[1] + w[3] * gm[3];
}

/* Heat-bath update of site s at temperature T: for every subgroup the new
 * element is drawn by hb_subgroup_element from the current block of K, K
 * summed over the first ndir directions (4: Landau, 3: Coulomb). */
static void hb_site_update(double* U, const geom* g, long s, double T, const uint32_t* key, uint32_t sweep,
                           int* capped, int ndir)
{
    for (int sg = 0; sg < 3; ++sg) {
        int i = SUBGROUP[sg][0], j = SUBGROUP[sg][1];
        cx K[9], k[4], g2[4], S[9];
        local_K(U, g, s, ndir, K);
        block_of(K, i, j, k);
        hb_stream st = {{key[0], key[1]}, (uint32_t)s, sweep, (uint32_t)sg, 0u};
        hb_subgroup_element(k, T, &st, capped, g2);
        embed(g2, i, j, S);
        transform_site(U, g, s, S);
    }
}

/* Temperature of annealing sweep s of n: linear from T0 (s = 0) to T1
 * (s = n-1), both endpoints taken exactly (the interpolation formula alone can
 * miss T1 by an ulp). */
static double anneal_temperature(int32_t s, int32_t n, double T0, double T1)
{
    if (n <= 1 || s == 0) return T0;
    if (s == n - 1) return T1;
    return T0 + (T1 - T0) * (double)s / (double)(n - 1);
}

/* n heat-bath sweeps (black then white) with the linear schedule; the Philox
 * key is the 64-bit seed and the sweep counter starts at sweep_offset.
 * Returns the number of subgroup updates that hit the rejection cap. */
static int64_t anneal_ndir(double* U, const int32_t* dims, int32_t nsweeps, double T0, double T1, uint64_t seed,
                           int32_t sweep_offset, int ndir)
{
    geom g = mkgeom(dims);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int64_t capped_total = 0;
    for (int32_t sw = 0; sw < nsweeps; ++sw) {
        double T = anneal_temperature(sw, nsweeps, T0, T1);
        for (int c = 0; c < 2; ++c) {
            int capped = 0;
#pragma omp parallel for schedule(static) reduction(+ : capped) if (g.V >= OMP_MIN_SITES)
            for (long s = 0; s < g.V; ++s)
                if (colour_of(&g, s) == c)
                    hb_site_update(U, &g, s, T, key, (uint32_t)(sweep_offset + sw), &capped, ndir);
            capped_total += capped;
        }
    }
    return capped_total;
}

int64_t oracle_anneal(double* U, const int32_t* dims, int32_t nsweeps, double T0, double T1, uint64_t seed,
                      int32_t sweep_offset)
{
    return anneal_ndir(U, dims, nsweeps, T0, T1, seed, sweep_offset, 4);
}

/* Simulated annealing of the Coulomb functional: the heat bath above with the
 * weight exp(Re tr[g k_C]/T), k_C a block of the spatial K_C(x); g(x) still
 * transforms all 8 links at x. */
int64_t oracle_coulomb_anneal(double* U, const int32_t* dims, int32_t nsweeps, double T0, double T1, uint64_t seed,
                              int32_t sweep_offset)
{
    return anneal_ndir(U, dims, nsweeps, T0, T1, seed, sweep_offset, 3);
}

/* Sampler checks: n draws of r0 (or of the SU(2) element as 4 reals) at a
 * fixed kappa, stream i using counter site = i, sweep = 0, subgroup = 0. */
int64_t oracle_hb_sample_r0(double kappa, uint64_t seed, int64_t n, double* out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int capped = 0;
    for (int64_t i = 0; i < n; ++i) {
        hb_stream st = {{key[0], key[1]}, (uint32_t)i, 0u, 0u, 0u};
        out[i] = hb_sample_r0(&st, kappa, &capped);
    }
    return capped;
}

int64_t oracle_hb_sample_su2(double kappa, uint64_t seed, int64_t n, double* out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int capped = 0;
    for (int64_t i = 0; i < n; ++i) {
        hb_stream st = {{key[0], key[1]}, (uint32_t)i, 0u, 0u, 0u};
        cx w[4];
        hb_sample_su2(&st, kappa, &capped, w);
        out[4 * i + 0] = creal(w[0]);
        out[4 * i + 1] = cimag(w[1]);
        out[4 * i + 2] = creal(w[1]);
        out[4 * i + 3] = cimag(w[0]);
    }
    return capped;
}

/* Site-level heat-bath draws: n subgroup elements for one fixed 2x2 block k
 * (4 complex numbers, row-major, as 8 doubles) at temperature T, draw i on
 * counter site = i, sweep = 0, subgroup = 0; out holds n 2x2 complex
 * matrices (8 doubles each).  The same code path as the annealing sweep. */
int64_t oracle_hb_subgroup_draws(const double* k, double T, uint64_t seed, int64_t n, double* out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int capped = 0;
    for (int64_t i = 0; i < n; ++i) {
        hb_stream st = {{key[0], key[1]}, (uint32_t)i, 0u, 0u, 0u};
        hb_subgroup_element((const cx*)k, T, &st, &capped, (cx*)(out + 8 * i));
    }
    return capped;
}

/* ------------------------------------------------------------------ */
/* SU(2) gauge group                                                   */
/* ------------------------------------------------------------------ */

/* The paper's method for gauge group SU(2) (abstract; Sec. 2 states the SU(2)
 * maximiser, and Sec. 4.1 changes the group by the link parameterisation
 * alone): links are 2x2 complex matrices, canonical layout
 * U[site][mu][row][col][re,im] (8 doubles per link).  K(x) sums U_mu(x) +
 * U_mu(x-mu^)^dag over the first ndir directions (4: Landau, 3: Coulomb); the
 * site's element is the maximiser K^dag / sqrt(det K^dag) itself (no subgroup
 * iteration; a sum of SU(2) matrices lies in the real span of SU(2), so the
 * projection leaves it unchanged) raised to omega, and it transforms the 8
 * links at x.  Measurements with N_c = 2:
 *   theta = (1/(2V)) sum_x tr[Delta Delta^dag],  F = (1/(8V)) sum_x sum_mu Re tr U,
 *   plaquette = (1/(12V)) sum_x sum_{mu<nu} Re tr[U U U^dag U^dag]. */

static cx* link2_at(double* U, long s, int mu)
{
    return (cx*)(U + ((size_t)s * 4 + (size_t)mu) * 8);
}

static const cx* clink2_at(const double* U, long s, int mu)
{
    return (const cx*)(U + ((size_t)s * 4 + (size_t)mu) * 8);
}

static void m2_mul(cx* c, const cx* a, const cx* b)
{
    cx t[4];
    t[0] = a[0] * b[0] + a[1] * b[2];
    t[1] = a[0] * b[1] + a[1] * b[3];
    t[2] = a[2] * b[0] + a[3] * b[2];
    t[3] = a[2] * b[1] + a[3] * b[3];
    memcpy(c, t, sizeof t);
}

static void m2_dag(cx* d, const cx* a)
{
    cx t[4] = {conj(a[0]), conj(a[2]), conj(a[1]), conj(a[3])};
    memcpy(d, t, sizeof t);
}

static void local_K2(const double* U, const geom* g, long s, int ndir, cx* K)
{
    K[0] = K[1] = K[2] = K[3] = 0.0;
    for (int mu = 0; mu < ndir; ++mu) {
        const cx* f = clink2_at(U, s, mu);
        cx b[4];
        m2_dag(b, clink2_at(U, hop(g, s, mu, -1), mu));
        for (int i = 0; i < 4; ++i) K[i] += f[i] + b[i];
    }
}

/* U_mu(x) <- S U_mu(x), U_mu(x-mu^) <- U_mu(x-mu^) S^dag for all 4 mu. */
static void transform_site2(double* U, const geom* g, long s, const cx* S)
{
    cx Sd[4];
    m2_dag(Sd, S);
    for (int mu = 0; mu < 4; ++mu) {
        cx* f = link2_at(U, s, mu);
        m2_mul(f, S, f);
        cx* b = link2_at(U, hop(g, s, mu, -1), mu);
        m2_mul(b, b, Sd);
    }
}

/* Overrelaxation update of site s; returns the change of Re tr K(x). */
static double su2lat_site_update(double* U, const geom* g, long s, double omega, int mode, int ndir)
{
    cx K[4], g2[4], SK[4];
    local_K2(U, g, s, ndir, K);
    if (!oracle_su2_maximiser((const double*)K, (double*)g2)) return 0.0;
    oracle_su2_overrelax((const double*)g2, omega, mode, (double*)g2);
    m2_mul(SK, g2, K);
    transform_site2(U, g, s, g2);
    return creal(SK[0] + SK[3]) - creal(K[0] + K[3]);
}

double oracle_su2lat_site_update(double* U, const int32_t* dims, int64_t site, double omega, int mode, int ndir)
{
    geom g = mkgeom(dims);
    return su2lat_site_update(U, &g, (long)site, omega, mode, ndir);
}

void oracle_su2lat_half_sweep(double* U, const int32_t* dims, int colour, double omega, int mode, int ndir)
{
    geom g = mkgeom(dims);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s)
        if (colour_of(&g, s) == colour) su2lat_site_update(U, &g, s, omega, mode, ndir);
}

void oracle_su2lat_sweep(double* U, const int32_t* dims, int32_t nsweeps, double omega, int mode, int ndir)
{
    for (int32_t k = 0; k < nsweeps; ++k) {
        oracle_su2lat_half_sweep(U, dims, 0, omega, mode, ndir);
        oracle_su2lat_half_sweep(U, dims, 1, omega, mode, ndir);
    }
}

void oracle_su2lat_update_sites_in_order(double* U, const int32_t* dims, const int64_t* sites, int64_t n,
                                         double omega, int mode, int ndir)
{
    geom g = mkgeom(dims);
    for (int64_t i = 0; i < n; ++i) su2lat_site_update(U, &g, (long)sites[i], omega, mode, ndir);
}

/* A = [(U - U^dag)/(2i)]_traceless for a 2x2 link. */
static void gauge_potential2(const cx* u, cx* A)
{
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) A[2 * i + j] = (u[2 * i + j] - conj(u[2 * j + i])) / (2.0 * I);
    cx tr = (A[0] + A[3]) / 2.0;
    A[0] -= tr;
    A[3] -= tr;
}

static double theta_site2(const double* U, const geom* g, long s, int ndir)
{
    cx D[4] = {0.0, 0.0, 0.0, 0.0}, A[4], Dd[4], P[4];
    for (int mu = 0; mu < ndir; ++mu) {
        gauge_potential2(clink2_at(U, s, mu), A);
        for (int i = 0; i < 4; ++i) D[i] += A[i];
        gauge_potential2(clink2_at(U, hop(g, s, mu, -1), mu), A);
        for (int i = 0; i < 4; ++i) D[i] -= A[i];
    }
    m2_dag(Dd, D);
    m2_mul(P, D, Dd);
    return creal(P[0] + P[3]);
}

void oracle_su2lat_theta_density(const double* U, const int32_t* dims, int ndir, double* out)
{
    geom g = mkgeom(dims);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s) out[s] = theta_site2(U, &g, s, ndir);
}

/* Landau gauge (ndir 4): theta = (1/(2V)) sum tr[Delta Delta^dag], F = (1/(8V)) sum sum Re tr U. */
void oracle_su2lat_measure(const double* U, const int32_t* dims, double* theta, double* F)
{
    geom g = mkgeom(dims);
    double* th = (double*)malloc(sizeof(double) * (size_t)g.V);
    double* fr = (double*)malloc(sizeof(double) * (size_t)g.V);
#pragma omp parallel for schedule(static) if (g.V >= OMP_MIN_SITES)
    for (long s = 0; s < g.V; ++s) {
        th[s] = theta_site2(U, &g, s, 4);
        double f = 0.0;
        for (int mu = 0; mu < 4; ++mu) f += creal(clink2_at(U, s, mu)[0] + clink2_at(U, s, mu)[3]);
        fr[s] = f;
    }
    double st = 0.0, sf = 0.0;
    for (long s = 0; s < g.V; ++s) {
        st += th[s];
        sf += fr[s];
    }
    free(th);
    free(fr);
    *theta = st / (2.0 * (double)g.V);
    *F = sf / (8.0 * (double)g.V);
}

/* Coulomb gauge: theta_C(t) = (1/(2 V3)) sum_{x in t} tr[Delta_C Delta_C^dag],
 * F_C(t) = (1/(6 V3)) sum_{x in t} sum_i Re tr U_i(x). */
void oracle_su2lat_coulomb_measure(const double* U, const int32_t* dims, double* theta_t, double* F_t)
{
    geom g = mkgeom(dims);
    const long V3 = g.V / g.n[3];
    for (int t = 0; t < g.n[3]; ++t) {
        double st = 0.0, sf = 0.0;
        for (long s = (long)t * V3; s < (long)(t + 1) * V3; ++s) {
            st += theta_site2(U, &g, s, 3);
            for (int i = 0; i < 3; ++i) sf += creal(clink2_at(U, s, i)[0] + clink2_at(U, s, i)[3]);
        }
        theta_t[t] = st / (2.0 * (double)V3);
        F_t[t] = sf / (6.0 * (double)V3);
    }
}

double oracle_su2lat_plaquette(const double* U, const int32_t* dims)
{
    geom g = mkgeom(dims);
    double sum = 0.0;
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cx t1[4], a[4], b[4];
                m2_mul(t1, clink2_at(U, s, mu), clink2_at(U, hop(&g, s, mu, +1), nu));
                m2_dag(a, clink2_at(U, hop(&g, s, nu, +1), mu));
                m2_mul(t1, t1, a);
                m2_dag(b, clink2_at(U, s, nu));
                m2_mul(t1, t1, b);
                sum += creal(t1[0] + t1[3]);
            }
    return sum / (12.0 * (double)g.V);
}

/* max over links of ||U^dag U - 1||_F and |det U - 1| (2x2 links) */
void oracle_su2lat_unitarity(const double* U, int64_t nlinks, double* max_unit, double* max_det)
{
    double mu = 0.0, md = 0.0;
    for (int64_t l = 0; l < nlinks; ++l) {
        const cx* u = (const cx*)(U + (size_t)l * 8);
        cx ud[4], p[4];
        m2_dag(ud, u);
        m2_mul(p, ud, u);
        double fro = 0.0;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                cx e = p[2 * i + j] - (i == j ? 1.0 : 0.0);
                fro += creal(e * conj(e));
            }
        fro = sqrt(fro);
        double dd = cabs(u[0] * u[3] - u[1] * u[2] - 1.0);
        if (fro > mu) mu = fro;
        if (dd > md) md = dd;
    }
    *max_unit = mu;
    *max_det = md;
}

/* Back onto SU(2): the projection onto the real span of SU(2) (as for a
 * subgroup block), divided by the square root of its determinant. */
void oracle_su2lat_reunitarize(double* U, int64_t nlinks)
{
    for (int64_t l = 0; l < nlinks; ++l) {
        cx* u = (cx*)(U + (size_t)l * 8);
        cx q[4];
        oracle_su2_project((const double*)u, (double*)q);
        cx root = csqrt(q[0] * q[3] - q[1] * q[2]);
        for (int i = 0; i < 4; ++i) u[i] = q[i] / root;
    }
}

/* Fix-until for SU(2) (the loop of oracle_fix_until; Coulomb gauge: theta =
 * the largest theta_C(t), F = the mean F_C(t)). */
int oracle_su2lat_fix_until(double* U, const int32_t* dims, double omega, int mode, double theta_target,
                            int32_t max_sweeps, int32_t check_every, int32_t reunit_every, int ndir,
                            int32_t* sweeps_out, double* theta_out, double* F_out)
{
    geom g = mkgeom(dims);
    const int nt = g.n[3];
    double* th = (double*)malloc(sizeof(double) * (size_t)nt);
    double* fr = (double*)malloc(sizeof(double) * (size_t)nt);
    double theta = 0.0, F = 0.0;
    int32_t sweeps = 0;
    for (;;) {
        if (ndir == 4) {
            oracle_su2lat_measure(U, dims, &theta, &F);
        } else {
            oracle_su2lat_coulomb_measure(U, dims, th, fr);
            theta = 0.0;
            F = 0.0;
            for (int t = 0; t < nt; ++t) {
                if (th[t] > theta) theta = th[t];
                F += fr[t];
            }
            F /= (double)nt;
        }
        if (!(theta >= theta_target) || sweeps >= max_sweeps) break;
        int32_t n = max_sweeps - sweeps < check_every ? max_sweeps - sweeps : check_every;
        for (int32_t k = 0; k < n; ++k) {
            oracle_su2lat_sweep(U, dims, 1, omega, mode, ndir);
            ++sweeps;
            if (reunit_every > 0 && sweeps % reunit_every == 0) oracle_su2lat_reunitarize(U, 4 * (int64_t)g.V);
        }
    }
    free(th);
    free(fr);
    *sweeps_out = sweeps;
    *theta_out = theta;
    *F_out = F;
    return theta < theta_target;
}

/* Heat bath for SU(2): each site's element is drawn from exp(Re tr[g K]/T)
 * dHaar(g) with the sampler of the SU(3) subgroups (subgroup index 0 of the
 * Philox counter), K over the first ndir directions. */
int64_t oracle_su2lat_anneal(double* U, const int32_t* dims, int32_t nsweeps, double T0, double T1, uint64_t seed,
                             int32_t sweep_offset, int ndir)
{
    geom g = mkgeom(dims);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int64_t capped_total = 0;
    for (int32_t sw = 0; sw < nsweeps; ++sw) {
        double T = anneal_temperature(sw, nsweeps, T0, T1);
        for (int c = 0; c < 2; ++c) {
            int capped = 0;
#pragma omp parallel for schedule(static) reduction(+ : capped) if (g.V >= OMP_MIN_SITES)
            for (long s = 0; s < g.V; ++s) {
                if (colour_of(&g, s) != c) continue;
                cx K[4], g2[4];
                local_K2(U, &g, s, ndir, K);
                hb_stream st = {{key[0], key[1]}, (uint32_t)s, (uint32_t)(sweep_offset + sw), 0u, 0u};
                hb_subgroup_element(K, T, &st, &capped, g2);
                transform_site2(U, &g, s, g2);
            }
            capped_total += capped;
        }
    }
    return capped_total;
}

/* ------------------------------------------------------------------ */
/* 8-real storage of an SU(3) link                                     */
/* ------------------------------------------------------------------ */

/* Sec. 4.1 names the minimal 8-parameter representation of an SU(3) link
 * among the ones cuLGT2 does not provide; the paper gives no formulae.  The
 * parameterisation here is the row-pivoted variant of the 8-real
 * reconstruction of Clark et al. (Comput. Phys. Commun. 181 (2010) 1517),
 * chosen so that every square root is taken of a quantity >= 1/3 and every
 * phase is a half-angle tangent (no trigonometric function in the decode):
 *
 *   U in SU(3) with rows r0, r1 (r2 = conj(r0 x r1)).
 *   k = the column of the largest |U_0c| (first maximum), i = k+1, j = k+2
 *   (mod 3).  Columns are taken in the cyclic order (k, i, j) below.
 *   p0 + i p1 = U_0i,  p2 + i p3 = U_0j,  p4 = tan(arg(U_0k) / 2),
 *   so |U_0k| = sqrt(1 - |U_0i|^2 - |U_0j|^2) >= 1/sqrt(3).
 *   n = sqrt(1 - |U_0j|^2); over (k, i, j)
 *     e1 = (-conj(U_0i), conj(U_0k), 0) / n,
 *     e2 = (-U_0k conj(U_0j) / n, -U_0i conj(U_0j) / n, n)
 *   form an orthonormal basis of the complement of r0 (e2 = conj(r0 x e1)),
 *   and r1 = alpha e1 + beta e2 with |alpha|^2 + |beta|^2 = 1.
 *   q = 1 if |beta| > |alpha| (else 0); s = the smaller, b = the larger of the
 *   two: p5 + i p6 = s, p7 = tan(arg(b) / 2), |b| = sqrt(1 - |s|^2) >= 1/sqrt(2).
 *   The three bits k (2 bits) and q are the lowest mantissa bits of p0, p1
 *   (bit 0 and bit 1 of k) and p5 (q); writing them moves those values by at
 *   most one unit in the last place.
 *   A half-angle tangent t of the phase c + i s: c = (1 - t^2)/(1 + t^2),
 *   s = 2t/(1 + t^2); t is formed as Im/(|z| + Re) for Re >= 0 and as
 *   (|z| - Re)/Im otherwise (no cancellation either way), and held to
 *   |t| <= 1e150 (the phase pi).
 * A float64 site update then moves 8 links x 8 reals x 8 B x 2 = 1024 B. */

static double tan_half_arg(cx z)
{
    const double a = cabs(z), re = creal(z), im = cimag(z);
    double t = re >= 0.0 ? im / (a + re) : (a - re) / im;
    if (!(fabs(t) <= 1e150)) t = im < 0.0 || (im == 0.0 && signbit(im)) ? -1e150 : 1e150;
    return t;
}

static cx phase_of_tan_half(double t)
{
    const double d = 1.0 + t * t;
    return (1.0 - t * t) / d + I * (2.0 * t / d);
}

static double with_low_bit(double v, int bit)
{
    uint64_t w;
    memcpy(&w, &v, sizeof w);
    w = (w & ~(uint64_t)1) | (uint64_t)(bit & 1);
    memcpy(&v, &w, sizeof v);
    return v;
}

static int low_bit(double v)
{
    uint64_t w;
    memcpy(&w, &v, sizeof w);
    return (int)(w & 1u);
}

/* rows r0, r1 of an SU(3) matrix (columns in natural order) -> 8 reals */
static void min8_encode_link(const cx* u, double* p)
{
    const cx* r0 = u;
    const cx* r1 = u + 3;
    int k = 0;
    for (int c = 1; c < 3; ++c)
        if (cabs(r0[c]) > cabs(r0[k])) k = c;
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    const cx ak = r0[k], ai = r0[i], aj = r0[j];
    const double n = sqrt(1.0 - creal(aj * conj(aj)));
    /* e1, e2 as above, indexed by the natural column */
    cx e1[3], e2[3];
    e1[k] = -conj(ai) / n;
    e1[i] = conj(ak) / n;
    e1[j] = 0.0;
    e2[k] = -ak * conj(aj) / n;
    e2[i] = -ai * conj(aj) / n;
    e2[j] = n;
    cx alpha = 0.0, beta = 0.0;
    for (int c = 0; c < 3; ++c) {
        alpha += conj(e1[c]) * r1[c];
        beta += conj(e2[c]) * r1[c];
    }
    const int q = cabs(beta) > cabs(alpha);
    const cx sm = q ? alpha : beta, big = q ? beta : alpha;
    p[0] = with_low_bit(creal(ai), k & 1);
    p[1] = with_low_bit(cimag(ai), k >> 1);
    p[2] = creal(aj);
    p[3] = cimag(aj);
    p[4] = tan_half_arg(ak);
    p[5] = with_low_bit(creal(sm), q);
    p[6] = cimag(sm);
    p[7] = tan_half_arg(big);
}

/* 8 reals -> the full SU(3) matrix (3 rows) */
static void min8_decode_link(const double* p, cx* u)
{
    const int k = low_bit(p[0]) | (low_bit(p[1]) << 1);
    const int q = low_bit(p[5]);
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    const cx ai = p[0] + I * p[1];
    const cx aj = p[2] + I * p[3];
    const double rho = sqrt(fmax(0.0, 1.0 - creal(ai * conj(ai)) - creal(aj * conj(aj))));
    const cx ak = rho * phase_of_tan_half(p[4]);
    const double n = sqrt(1.0 - creal(aj * conj(aj)));
    const cx sm = p[5] + I * p[6];
    const cx big = sqrt(fmax(0.0, 1.0 - creal(sm * conj(sm)))) * phase_of_tan_half(p[7]);
    const cx alpha = q ? sm : big, beta = q ? big : sm;
    cx* r0 = u;
    cx* r1 = u + 3;
    cx* r2 = u + 6;
    r0[k] = ak;
    r0[i] = ai;
    r0[j] = aj;
    r1[k] = alpha * (-conj(ai) / n) + beta * (-ak * conj(aj) / n);
    r1[i] = alpha * (conj(ak) / n) + beta * (-ai * conj(aj) / n);
    r1[j] = beta * n;
    r2[0] = conj(r0[1] * r1[2] - r0[2] * r1[1]);
    r2[1] = conj(r0[2] * r1[0] - r0[0] * r1[2]);
    r2[2] = conj(r0[0] * r1[1] - r0[1] * r1[0]);
}

/* nlinks canonical links (18 reals each) -> 8 reals each */
void oracle_min8_encode(const double* U, int64_t nlinks, double* P)
{
    for (int64_t l = 0; l < nlinks; ++l) min8_encode_link((const cx*)(U + (size_t)l * 18), P + (size_t)l * 8);
}

/* nlinks x 8 reals -> canonical links */
void oracle_min8_decode(const double* P, int64_t nlinks, double* U)
{
    for (int64_t l = 0; l < nlinks; ++l) min8_decode_link(P + (size_t)l * 8, (cx*)(U + (size_t)l * 18));
}

/* The configuration a lattice stored in 8 reals per link holds after the
 * links U were written to it: decode(encode(U)) per link, in place. */
void oracle_min8_store(double* U, int64_t nlinks)
{
    for (int64_t l = 0; l < nlinks; ++l) {
        double p[8];
        cx* u = (cx*)(U + (size_t)l * 18);
        min8_encode_link(u, p);
        min8_decode_link(p, u);
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops from now on (n >= 1); timing control only. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
