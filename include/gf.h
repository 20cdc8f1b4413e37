/*
 * gf.h -- C ABI of libgf, SU(3) lattice Landau gauge fixing by checkerboard
 * overrelaxation on AMD Instinct MI355X (gfx950).
 *
 * Method: H. Vogt and M. Schroeck, "cuLGT: Lattice Gauge Fixing on GPUs",
 * arXiv:1412.3655, Sec. 2 (gauge transformation, Eq. (landaugauge),
 * Eq. (landaufunctional), Eq. (localfunctional), the SU(2) maximiser, the
 * SU(2)-subgroup iteration, overrelaxation g -> g^omega and the black/white
 * checkerboard), Sec. 3.1 (checkerboard-split, site-fastest storage and the
 * two-row 12-real SU(3) representation).
 *
 * Conventions shared by every entry point
 *   - Host link arrays are "canonical": float64, C order
 *     [site][mu][row][col][re,im] (18 doubles per link, 72 per site), with the
 *     lexicographic site index x + Nx*(y + Ny*(z + Nz*t)) and mu = 0..3 for
 *     x, y, z, t.  Element [site][mu] is U_mu(x), the link from x to x + mu^.
 *   - Extents dims[4] = {Nx, Ny, Nz, Nt}: each even and >= 2 (the checkerboard
 *     needs a bipartite periodic lattice); boundaries are periodic.
 *   - Ownership: the library owns every device buffer it allocates (hipMalloc);
 *     caller pointers are borrowed for the duration of the call only.
 *   - Streams: all device work of a lattice is ordered on the hip stream given
 *     at creation (NULL = the default stream).  Calls marked "async" only
 *     enqueue work; calls marked "syncs" wait for that stream.
 *   - Errors: every call returns a gf_status; no C++ exception crosses the ABI.
 *     Arguments are validated before any device work.  HIP failures return
 *     GF_E_HIP; gf_last_error() then returns a thread-local message.
 *   - Threads: one lattice must not be used by two threads at once.
 */
#ifndef GF_H
#define GF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_lattice_* gf_lattice; /* opaque, library-owned */

typedef enum {
    GF_OK = 0,
    GF_E_ARG = 1,     /* invalid argument (null pointer, odd extent, omega out of range, ...) */
    GF_E_NOMEM = 2,   /* device allocation failed */
    GF_E_HIP = 3,     /* a HIP runtime call failed; see gf_last_error() */
    GF_E_STATE = 4,   /* call not valid in the current state (e.g. no links set) */
    GF_E_NUMERIC = 5, /* theta or F is NaN or infinite */
    GF_E_FULL = 6,    /* no room (pool admission) */
    GF_E_CANCELLED = 7 /* the job was cancelled (gf_pool_cancel) */
} gf_status;

typedef enum {
    GF_FP64 = 0,  /* links stored and updated in float64 */
    GF_FP32 = 1,  /* links stored and updated in float32 (sums of theta/F in float64) */
    GF_MIXED = 2  /* float32 bulk sweeps, then float64 polish (see gf_fix_until) */
} gf_prec;

typedef enum {
    /* g^omega taken literally: the principal power of the SU(2) subgroup element,
     * (cos(w phi), sin(w phi) n) for g = (cos phi, sin phi n) (Sec. 2, overrelaxation). */
    GF_OR_EXACT = 0,
    /* normalise(1 + w (g - 1)): first-order form of the same power. */
    GF_OR_BINOMIAL1 = 1
} gf_or_mode;

typedef enum {
    /* Landau gauge (Sec. 2): functional and condition over all 4 directions. */
    GF_LANDAU = 0,
    /* Coulomb gauge (listed beside Landau gauge in the abstract and Sec. 1):
     * the functional and condition of Sec. 2 with mu over x, y, z only, one
     * independent problem per timeslice. */
    GF_COULOMB = 1
} gf_gauge;

typedef struct {
    double omega;         /* overrelaxation parameter, 1 <= omega < 2 */
    int32_t mode;         /* gf_or_mode */
    double theta_target;  /* stop at the first check with theta < theta_target */
    int32_t max_sweeps;   /* >= 0 */
    int32_t check_every;  /* >= 1: sweeps between measurements */
    int32_t reunit_every; /* reunitarise after every sweep whose count is a multiple of this; 0 = never */
    double theta_switch;  /* GF_MIXED only: leave float32 once theta < theta_switch;
                             < 0: the switch point gf_tune_switch picks for the lattice */
} gf_fix_params;

typedef struct {
    int32_t converged;   /* theta < theta_target at the last check */
    int32_t sweeps;      /* sweeps done by this call */
    int32_t sweeps_fp32; /* of which in float32 */
    int32_t sweeps_fp64; /* of which in float64 */
    double theta;        /* at the last check */
    double F;            /* at the last check */
} gf_fix_result;

/* Create a lattice of extents dims (see conventions) and precision prec.
 * hip_stream: a hipStream_t (NULL = default stream).  Allocates the link
 * fields in the checkerboard-split, site-fastest 12-real device layout
 * (Sec. 3.1): 4*V*12 reals, plus for GF_MIXED the float64 copy of the links
 * and a float32 gauge-transformation field.  Links start undefined. */
gf_status gf_create_lattice(const int32_t dims[4], gf_prec prec, void* hip_stream, gf_lattice* out);

/* The same method for gauge group SU(2) (the abstract lists SU(2) beside
 * SU(3); Sec. 2's maximiser K^dag / sqrt(det K^dag) is exact for SU(2), so a
 * site update has no subgroup iteration; Sec. 4.1 changes the group by the
 * link parameterisation).  prec GF_FP64 or GF_FP32 (GF_MIXED: GF_E_ARG).
 * Links are stored as quaternions (q0, q1, q2, q3) of
 * U = [[q0 + i q3, q2 + i q1], [-q2 + i q1, q0 - i q3]] in the same
 * checkerboard, site-fastest tiled layout (32 B per float64 link; a site
 * update moves 512 B).  Every entry point taking a lattice accepts an SU(2)
 * lattice, with these differences:
 *   - canonical arrays hold 2x2 links: [site][mu][row][col][re,im], 8 doubles
 *     per link, 32 per site (gf_set_links keeps the element's projection onto
 *     the real span of SU(2), i.e. the link itself for an SU(2) matrix);
 *   - theta = (1/(2V)) sum_x tr[Delta Delta^dag], F = (1/(8V)) sum_x sum_mu
 *     Re tr U, plaquette normalised by 12V (N_c = 2); Coulomb gauge:
 *     theta_C(t) and F_C(t) with 1/(2 V3) and 1/(6 V3);
 *   - the heat bath draws g from exp(Re tr[g K]/T) dHaar with the SU(3)
 *     subgroup sampler, Philox subgroup index 0;
 *   - sweep configurations: one lane per site (tps 1), block 64..512, cache
 *     policy 0..2; gf_autotune times those;
 *   - reunitarisation divides each quaternion by its norm;
 *   - gf_tune_switch and the pool are SU(3) only (GF_E_STATE / not offered). */
gf_status gf_create_lattice_su2(const int32_t dims[4], gf_prec prec, void* hip_stream, gf_lattice* out);

/* N_c of the lattice's gauge group: 3 (gf_create_lattice) or 2 (gf_create_lattice_su2). */
gf_status gf_lattice_group(gf_lattice lat, int32_t* nc);

/* An SU(3) float64 lattice whose links are stored in 8 reals: the minimal
 * 8-parameter representation that Sec. 4.1 names among those cuLGT2 does
 * not provide (the paper gives no formulae).  The parameterisation is a
 * row-pivoted form of the 8-real reconstruction of Clark et al. (Comput.
 * Phys. Commun. 181 (2010) 1517): with k the column of the largest |U_0c|
 * and i, j the next two columns cyclically, the stored reals are U_0i, U_0j,
 * tan(arg U_0k / 2), and row 1's coordinates (alpha, beta) in an orthonormal
 * basis of row 0's complement as the smaller of the two plus the half-angle
 * tangent of the larger's phase; k and which of alpha, beta is larger ride in
 * the lowest mantissa bits of three stored reals (each moved by at most one
 * unit in the last place).  Every square root in the decode is taken of a
 * quantity >= 1/3, so a stored link is SU(3) to float64 rounding.  Same
 * checkerboard, site-fastest tiled layout as the 12-real field with 4
 * chunks of 16 B per link: 64 B per link, a site update moves 1024 B instead
 * of 1536 B, at the cost of a decode per link load and an encode per store.
 * Every entry point taking a lattice accepts it, with these differences:
 *   - gf_set_links stores the projection of rows 0, 1 of each link onto
 *     SU(3) (the link itself for an SU(3) matrix, to rounding);
 *   - gf_reunitarize does nothing: every store re-projects onto SU(3);
 *   - sweep configurations as for GF_FP64 with min_waves 0 (gf_autotune
 *     times those; kernel GF_FP64);
 *   - gf_tune_switch: GF_E_STATE (no float32 phase).
 * Otherwise as gf_create_lattice(dims, GF_FP64, ...). */
gf_status gf_create_lattice_min8(const int32_t dims[4], void* hip_stream, gf_lattice* out);

/* Reals stored per link of the lattice's sweeping precision (the float64
 * links of GF_FP64, the float32 links of GF_FP32 and GF_MIXED): 12 (SU(3),
 * two rows), 8 (gf_create_lattice_min8, gf_set_storage) or 4 (SU(2)
 * quaternion). */
gf_status gf_lattice_storage(gf_lattice lat, int32_t* reals_per_link);

/* Switch an SU(3) lattice between 12-real and 8-real storage of the links
 * of its sweeping precision (reals_per_link 12 or 8; GF_E_ARG otherwise;
 * GF_E_STATE for SU(2) lattices): the float64 links of a GF_FP64 lattice,
 * the float32 links of a GF_FP32 or GF_MIXED one (a GF_MIXED lattice keeps
 * its float64 links, the original links and then the polish sweeps', in 12
 * reals).  The links are converted on the device: 12 -> 8 projects rows 0, 1
 * of each link onto SU(3) as gf_set_links on an 8-real lattice does (a
 * change at rounding level for SU(3) links), 8 -> 12 stores the decoded rows
 * (exactly for float64; float32 values are decoded in float64 and the rows
 * rounded).  Float32 links in 8 reals: 32 B per link, a float32 site update
 * moves 512 B instead of 768 B; the sweeps decode and encode in float32,
 * measurement decodes the stored values in float64, gf_set_links encodes in
 * float64 and rounds the 8 values to float32, and the float32 floor of
 * gf_tune_switch is that of links rounded through this storage.  The old
 * field is freed after the new one is written (both are held meanwhile);
 * captured sweep graphs are dropped and the register limit of the
 * configurations of the converted links reset to 0.  Syncs. */
gf_status gf_set_storage(gf_lattice lat, int32_t reals_per_link);

/* Storage as an autotuning axis (Sec. 4.1 and 5: the parameterisation and
 * the kernel configuration are both run-time choices in the paper's
 * design): tune the overrelaxation sweep of the sweeping precision of an
 * SU(3) lattice (as gf_autotune with kernel GF_FP64 for GF_FP64 lattices,
 * GF_FP32 for GF_FP32 and GF_MIXED ones, and no cache) in its current
 * storage, then on a scratch copy of its links converted to the other
 * storage, and switch the lattice to the faster storage with its fastest
 * configuration (gf_set_storage's conversion).  *reals_per_link (may be
 * NULL) receives the storage chosen, *us_12 and *us_8 (may be NULL) the best
 * time per sweep of each, in microseconds.  GF_E_STATE for SU(2) lattices.
 * Syncs. */
gf_status gf_autotune_storage(gf_lattice lat, int32_t n_sweeps, int32_t* reals_per_link, double* us_12,
                              double* us_8);

/* Free every device buffer of the lattice (waits for its stream).  NULL is accepted. */
gf_status gf_destroy_lattice(gf_lattice lat);

/* Number of sites V and bytes of device memory held by the lattice. */
gf_status gf_lattice_info(gf_lattice lat, int64_t* volume, int64_t* device_bytes);

/* Kernel configuration of the sweep in precision `kernel` (GF_FP64 or
 * GF_FP32; a GF_MIXED lattice uses both): tps lanes per site (1, 2, 4 or 8;
 * the paper's design uses 4 or 8 threads per site, Sec. 4.2), threads per
 * block (64, 128, 256 or 512; not 512 with tps 1), the cache policy of the
 * link accesses (0 = plain, 1 = non-temporal loads and stores, 2 = plain
 * loads and non-temporal stores; 1 and 2 only with tps <= 4 and block <= 256)
 * and the register limit (min_waves: 0 = the compiler's allocation, 2 = at
 * least 2 waves per SIMD, at most 256 registers per lane; 2 only with tps 1,
 * and it changes only float64 kernels, the paper's register-limit axis of
 * Sec. 5).  Every valid choice gives bitwise the same links.  Default
 * 4 / 256 / 0 / 0. */
gf_status gf_set_sweep_config(gf_lattice lat, gf_prec kernel, int32_t tps, int32_t block, int32_t nontemporal,
                              int32_t min_waves);

/* The same for the heat-bath sweeps of gf_anneal, which sample every
 * subgroup element in each lane of a site's group (so fewer lanes do less
 * arithmetic).  Default 1 / 256 / 0 for float32, 1 / 128 / 2 for float64. */
gf_status gf_set_anneal_config(gf_lattice lat, gf_prec kernel, int32_t tps, int32_t block, int32_t nontemporal,
                               int32_t min_waves);

/* GF_MIXED: leave the float32 phase now.  The float64 links become
 * g(x) U0_mu(x) g(x+mu^)^dag, U0 the links given to gf_set_links and g the
 * float32 transformation accumulated by the float32 sweeps (re-orthonormalised
 * in float64), so they stay on the gauge orbit of U0 to float64 precision.
 * No-op for other precisions or after promotion.  Async. */
gf_status gf_promote_fp64(gf_lattice lat);

typedef struct {
    int32_t tps;
    int32_t block;
    int32_t nontemporal;
    int32_t min_waves;   /* register limit: 0 = compiler's allocation, 2 = at least 2 waves per SIMD */
    double us_per_sweep; /* time of one sweep (both colours), microseconds: the faster of two rounds' means */
} gf_tune_entry;

/* Autotuner (the paper tunes threads per site, launch bounds and texture
 * loads at run time, Sec. 4 and 5): time every valid sweep configuration
 * (lanes per site, block size, cache policy, and for float64 the register
 * limit) of precision `kernel`
 * (GF_FP64 or GF_FP32) on a scratch copy of the lattice's links (two rounds
 * over all configurations, each with one warm-up sweep and then n_sweeps timed
 * sweeps per configuration; a configuration keeps its faster round), write up
 * to cap entries to table
 * (may be NULL), and make the fastest the lattice's configuration.  When
 * cache_path is not NULL, a result stored there for the same device
 * architecture, extents and kernel (float64; float32; float32 with the g(x)
 * update that a GF_MIXED lattice's float32 sweeps make) is applied without
 * timing (*n_out = 0),
 * and a newly timed result is appended to it (plain text, one line per key).
 * *chosen (may be NULL) receives the configuration applied.  The links are
 * not changed.  Syncs. */
gf_status gf_autotune(gf_lattice lat, gf_prec kernel, int32_t n_sweeps, const char* cache_path, gf_tune_entry* table,
                      int32_t cap, int32_t* n_out, gf_tune_entry* chosen);

/* As gf_autotune for the heat-bath sweep of gf_anneal (timed at T = 1 on the
 * scratch copy; cache lines keyed with an "-hb" suffix); sets the
 * configuration gf_set_anneal_config sets.  Syncs. */
gf_status gf_autotune_anneal(gf_lattice lat, gf_prec kernel, int32_t n_sweeps, const char* cache_path,
                             gf_tune_entry* table, int32_t cap, int32_t* n_out, gf_tune_entry* chosen);

/* Upload links from a host canonical array of 4*V*18 doubles; only rows 0
 * and 1 of each link are kept (row 2 is rebuilt as the conjugated cross
 * product whenever it is needed, Sec. 3.1).  Syncs. */
gf_status gf_set_links(gf_lattice lat, const double* host);

/* Same, from a device canonical array (hip device pointer).  Async. */
gf_status gf_set_links_device(gf_lattice lat, const double* dev);

/* Download links into a host canonical array (row 2 rebuilt).  Syncs. */
gf_status gf_get_links(gf_lattice lat, double* host);

/* Same, into a device canonical array.  Async. */
gf_status gf_get_links_device(gf_lattice lat, double* dev);

/* n_sweeps overrelaxation sweeps: each sweep updates every black site
 * ((x+y+z+t) even), then every white site.  A site update forms
 * K(x) = sum_mu [U_mu(x) + U_mu(x-mu^)^dag] (Eq. localfunctional), iterates
 * over the SU(2) subgroups (0,1), (0,2), (1,2) with the maximiser of the
 * SU(2)-span projection of each 2x2 block raised to the power omega, and
 * applies the accumulated g(x) to the 8 links at x (Sec. 2).
 * omega in [1, 2).  On a GF_MIXED lattice the sweep runs in the current
 * phase's precision.  Only two rows of each link are stored, so rounding
 * drift from SU(3) is not removed by the sweep itself: call gf_reunitarize
 * every ~100 sweeps (gf_fix_until does; measured drift without it on rough
 * inputs: <1e-12 after 2000 float64 sweeps, 2e-4 after 2000 float32 sweeps).
 * On a non-default stream, a call of n_sweeps >= 2 on a lattice of fewer
 * than 2^16 sites per colour is captured once as a hipGraph and replayed by
 * later calls with the same arguments and configuration; larger lattices
 * launch their kernels directly.  Async. */
gf_status gf_sweep_or(gf_lattice lat, int32_t n_sweeps, double omega, gf_or_mode mode);

/* One half-sweep over the sites of one colour (0 = black, 1 = white).  Async. */
gf_status gf_half_sweep_or(gf_lattice lat, int32_t colour, double omega, gf_or_mode mode);

/* n_sweeps heat-bath sweeps (simulated annealing prelude, abstract): every
 * subgroup element is drawn from exp(Re tr[g k]/T) dHaar(g), T falling
 * linearly from T_start (first sweep) to T_end (last sweep).  Random numbers:
 * Philox4x32-10 keyed by seed, counter (site, sweep, subgroup<<16 | call,
 * 0x48420000); the sweep counter continues across calls (reset by
 * gf_set_links).  T_start >= T_end > 0.  Async. */
gf_status gf_anneal(gf_lattice lat, int32_t n_sweeps, double T_start, double T_end, uint64_t seed);

/* Checkpoint / resume of annealing: the heat-bath sweep counter (sweeps run
 * by gf_anneal since gf_set_links).  Links saved with gf_get_links and the
 * counter, restored with gf_set_links and gf_set_anneal_counter, continue
 * bitwise as if never interrupted (counter-based random numbers).  GF_FP64
 * and GF_FP32 lattices; a GF_MIXED lattice also holds U0 and the float32
 * transformation, which gf_get_links does not return, so it cannot be
 * checkpointed this way (GF_E_STATE).  gf_set_anneal_counter comes after
 * gf_set_links (which resets the counter to 0; before any links: GF_E_STATE).
 * Neither call touches the device. */
gf_status gf_get_anneal_counter(gf_lattice lat, uint32_t* sweeps_done);
gf_status gf_set_anneal_counter(gf_lattice lat, uint32_t sweeps_done);

/* theta = (1/(3V)) sum_x tr[Delta(x) Delta(x)^dag] with
 * Delta(x) = [(K(x) - K(x)^dag)/(2i)]_traceless (equal to Eq. (landaugauge)
 * with A_mu of Sec. 2, a g = 1) and F = (1/(12V)) sum_x sum_mu Re tr U_mu(x)
 * (Eq. (landaufunctional) with the transformation already applied).  Sums in
 * float64 with a fixed reduction order.  Syncs.  GF_E_NUMERIC on NaN/Inf. */
gf_status gf_measure_theta_F(gf_lattice lat, double* theta, double* F);

/* Measure; then, while theta >= theta_target and sweeps < max_sweeps:
 * min(check_every, remaining) sweeps (reunitarising after every sweep whose
 * count is a multiple of reunit_every) and measure again (Sec. 2: iterate
 * until the gauge condition holds to a given precision).  GF_MIXED: float32
 * sweeps (with the transformation g(x) tracked) until theta < theta_switch,
 * until theta has reached no new minimum for 16 consecutive checks with a
 * best value below 1e-10 (a stall well above the float32 rounding floor is
 * the iteration's own slow convergence, not a precision limit), or until the
 * loop would end; then the float64 links are rebuilt as
 * g(x) U0_mu(x) g(x+mu^)^dag from the original links, theta is measured in
 * float64 and the loop continues in float64, so the result (links, theta, F,
 * converged) is always the float64 one.  Non-convergence is a result
 * (converged = 0), not an error.  Syncs. */
gf_status gf_fix_until(gf_lattice lat, const gf_fix_params* params, gf_fix_result* result);

/* How gf_fix_until checks the gauge condition (default: adaptive = 0, an
 * exact measurement after every check_every sweeps).  adaptive != 0: the
 * last sweep of every check_every also sums tr[Delta(x) Delta(x)^dag] of
 * each site's K(x), which the sweep forms anyway, just before the site's
 * update (see gf_sweep_estimate), and the exact measurement (a separate pass
 * reading every link twice) runs only where a decision can fall: when that
 * estimate is below margin x the smallest deciding threshold (theta_target;
 * in the float32 phase of GF_MIXED also theta_switch and the stall level
 * 1e-10), at every float32-phase check once theta has been below the stall
 * level, and at the last sweep.  The paper iterates until the condition holds
 * to a given precision (Sec. 2); where the estimate stays above margin x
 * every threshold no decision can be taken, so with a margin that covers the
 * ratio of estimate to theta (>= 1; default 100) the sweep count, links, theta
 * and F equal those of exact checks.  Does not touch the device. */
gf_status gf_set_check_policy(gf_lattice lat, int32_t adaptive, double margin);

/* One overrelaxation sweep (as gf_sweep_or with n_sweeps = 1) that also
 * returns *theta_est = (1/(3V)) sum_x tr[Delta(x) Delta(x)^dag] with each
 * site's Delta taken from its K(x) just before its update: the black sites'
 * terms before the black half-sweep, the white sites' after it (Coulomb gauge:
 * K_C and Delta_C, i.e. the mean over timeslices).  Per-block sums in float64
 * added in a fixed order.  GF_E_NUMERIC if NaN.  Syncs. */
gf_status gf_sweep_estimate(gf_lattice lat, double omega, gf_or_mode mode, double* theta_est);

/* Exact measurements (gf_measure_theta_F, and those of gf_fix_until) and
 * fused estimates taken on the lattice since its creation (may be NULL). */
gf_status gf_lattice_counters(gf_lattice lat, int64_t* measures, int64_t* estimates);

/* Switch point for the float32 -> float64 handover of GF_MIXED: *floor =
 * (1/(3V)) sum_x tr[E E^dag] with E = Delta(x) computed in float32 from the
 * float32-rounded float64 links minus Delta(x) in float64 (the float32
 * rounding floor of theta for this configuration), *theta_switch =
 * max(theta_target, 100 * floor).  Reads the float64 links (on GF_MIXED in
 * the float32 phase: the original links U0).  GF_E_STATE on a GF_FP32
 * lattice.  gf_fix_until calls it when theta_switch < 0.  Syncs. */
gf_status gf_tune_switch(gf_lattice lat, double theta_target, double* floor, double* theta_switch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): theta and F
 * exactly as gf_measure_theta_F computes them (same kernels, same reduction
 * order: bitwise equal to gf_measure_theta_F of a GF_FP64 lattice holding the
 * same links), over links the caller holds on the current device.
 *   dims       extents (even, >= 2), at most 2^24 sites (GF_E_ARG beyond:
 *              the reduction scratch is a fixed 1 MiB device array)
 *   dev_links  device canonical float64 array of 4*V*18 doubles (layout of
 *              the conventions above), read only; rows 0 and 1 of each link
 *              are read and row 2 is rebuilt from them
 *   dev_out    device array of 2 doubles: theta, then F
 *   hip_stream a hipStream_t of the current device (NULL = default stream)
 * Async: only enqueues kernels (no allocation, no memset, no copy, no
 * synchronisation), so it may be captured into a hipGraph; the caller checks
 * dev_out for NaN/Inf.  The scratch is one array per device, shared by every
 * call on that device: calls that overlap on one device race (serialise them
 * on one stream).  The first call on a device looks up that device's copy of
 * the array (hipGetSymbolAddress) and must not itself be under capture. */
gf_status gf_measure_theta_F_noalloc(const int32_t dims[4], const double* dev_links, double* dev_out,
                                     void* hip_stream);

/* Gauge fixed by the lattice's sweeps and measured by its measurements
 * (default GF_LANDAU).  With GF_COULOMB (abstract and Sec. 1 name Coulomb
 * gauge beside Landau gauge; its formulae are those of Sec. 2 restricted to the
 * spatial directions):
 *   - gf_sweep_or / gf_half_sweep_or / gf_anneal form
 *     K_C(x) = sum_{i=x,y,z} [U_i(x) + U_i(x-i^)^dag] in place of K(x), and the
 *     site's g(x) still transforms all 8 links at x, temporal ones included
 *     (so the configuration stays on its gauge orbit); the heat bath weighs
 *     each subgroup draw by exp(Re tr[g k_C]/T);
 *   - gf_measure_theta_F returns theta = max over timeslices t of
 *     theta_C(t) = (1/(3 V3)) sum_{x in t} tr[Delta_C Delta_C^dag],
 *     Delta_C = [(K_C - K_C^dag)/(2i)]_traceless, and F = the mean over t of
 *     F_C(t) = (1/(9 V3)) sum_{x in t} sum_i Re tr U_i(x), V3 = Nx Ny Nz;
 *   - gf_fix_until therefore stops once every timeslice satisfies the
 *     condition; with theta_switch < 0 a GF_MIXED lattice takes its switch
 *     point from gf_tune_switch, i.e. from the float32 floor of the Landau
 *     Delta (a performance heuristic: the result is float64 either way).
 * The pool (gf_pool_*) fixes Landau gauge only.  GF_E_ARG for an unknown
 * gauge, or GF_COULOMB with Nt > 65535.  Does not touch the device. */
gf_status gf_set_gauge(gf_lattice lat, gf_gauge gauge);
gf_status gf_get_gauge(gf_lattice lat, gf_gauge* gauge);

/* Coulomb gauge: theta_C(t) and F_C(t) (see gf_set_gauge) of every timeslice
 * t = 0..Nt-1 into two caller arrays of Nt doubles; float64 sums with a fixed
 * reduction order.  GF_E_STATE on a GF_LANDAU lattice; GF_E_NUMERIC if a value
 * is NaN/Inf.  Syncs. */
gf_status gf_measure_timeslices(gf_lattice lat, double* theta_t, double* F_t);

/* Reunitarise every link: Gram-Schmidt of rows 0 and 1 (row 2 is implicit).
 * The paper defines no reunitarisation; it is needed because only two rows
 * are stored (Sec. 3.1) and rounding drifts them off SU(3).  Rows are
 * r0 <- r0/|r0|, r1 <- (r1 - <r0,r1> r0)/|.|, row 2 their conjugated cross
 * product.  Async. */
gf_status gf_reunitarize(gf_lattice lat);

/* Average plaquette (1/(18V)) sum_x sum_{mu<nu} Re tr[U_mu(x) U_nu(x+mu^)
 * U_mu(x+nu^)^dag U_nu(x)^dag], float64 sums.  Not part of the paper's
 * method: a gauge-invariant observable (Sec. 2: gauge fixing moves along the
 * gauge orbit) used to check that sweeps leave it unchanged.  Syncs. */
gf_status gf_plaquette(gf_lattice lat, double* P);

/* ------------------------------------------------------------------------ */
/* Batched lattices and serving: a pool of resident lattices ("jobs") of any */
/* shapes swept together.                                                     */
/*                                                                            */
/* Every job runs exactly the fix-until iteration of gf_fix_until (optionally */
/* after gf_anneal) on its own lattice of the pool's precision, so its result */
/* equals the one it gets alone.  A pool step advances every active job by   */
/* up to check_every sweeps: per sweep one launch per kernel kind (heat      */
/* bath, float32 OR tracking g, float64 OR), one block per tile, covers the  */
/* sites of that colour of every job in that state, then reunitarisation and */
/* measurement launches cover the jobs due for them; the launches of a step  */
/* are captured once in a hipGraph per work structure and replayed with each */
/* sweep node's grid set to the step's tile count.                            */
/*                                                                            */
/* A step can be left in flight (gf_pool_step_async) while the host admits,   */
/* polls, fetches and releases jobs: these touch only jobs the step does not  */
/* use, and move links on a transfer stream of the pool's own, so the host's  */
/* work overlaps the GPU's.  Results are the same either way.                 */
/* ------------------------------------------------------------------------ */

typedef struct gf_pool_* gf_pool; /* opaque, library-owned */

typedef struct {
    size_t hbm_budget;   /* bytes of device memory the pool may hold for job lattices (its tables and
                            the 33.6 MB staging buffer of admissions and fetches come on top) */
    int32_t max_slots;   /* maximum number of resident jobs, 1..4096 */
    int32_t prec;        /* gf_prec of every job: GF_MIXED or GF_FP64 */
    int32_t check_every; /* sweeps per pool step = every job's measurement cadence, >= 1 */
    int32_t mode;        /* gf_or_mode of every job */
    int32_t tps32, block32, tps64, block64; /* shape of the pool's float32 / float64 overrelaxation
                                               sweeps: lanes per site (1, 2 or 4; 0 = default: 2 for
                                               float32 in 12 reals, 1 for float32 in 8 reals, 1 for
                                               float64) and threads per block (64, 128
                                               or 256; 0 = 128).  Every shape gives bitwise the same
                                               links; gf_pool_autotune picks the fastest for the
                                               resident jobs.  The heat-bath sweeps use one lane per
                                               site and 128-thread blocks. */
    int32_t reals32;     /* storage of the float32 links of a GF_MIXED pool: 12 (or 0) two rows, 8 the
                            8-real representation (gf_set_storage); 12 or 0 for a GF_FP64 pool */
    int32_t cache32, cache64; /* cache policy of the link loads and stores of the float32 / float64
                                 overrelaxation sweeps: 1 plain, 2 non-temporal, 0 = default (float32:
                                 non-temporal in 8 reals, plain in 12 reals; float64: non-temporal); the
                                 same links either way, and an axis of gf_pool_autotune.  The heat-bath
                                 sweeps keep plain accesses for float32, non-temporal for float64. */
} gf_pool_config;

typedef struct {
    uint64_t job_id;
    gf_fix_result result;
    int32_t status; /* GF_OK, or the error that ended the job (e.g. GF_E_NUMERIC); other jobs are unaffected */
    double t_admit; /* seconds on the library's steady clock */
    double t_done;  /* when the pool step in which the job finished was completed */
} gf_pool_done;

/* Create a pool.  hip_stream: a non-default hipStream_t for the pool's steps,
 * or NULL to let the pool create its own (default priority); admissions and
 * fetches use a second stream the pool creates.  Allocates bookkeeping and a
 * 33.6 MB staging buffer; job lattices are allocated on admission. */
gf_status gf_pool_create(const gf_pool_config* cfg, void* hip_stream, gf_pool* out);

/* Wait for the pool's streams and free everything, including unreleased jobs.  NULL is accepted. */
gf_status gf_pool_destroy(gf_pool pool);

/* Device bytes one job of extents dims needs in a pool of precision prec
 * whose float32 links take reals32 reals (12 or 8; 0 = 12). */
gf_status gf_pool_job_bytes(const int32_t dims[4], int32_t prec, int32_t reals32, int64_t* bytes);

/* Admit a job: copy its host canonical links (4*V*18 doubles) into a new
 * resident lattice, then (if anneal_sweeps > 0) run anneal_sweeps heat-bath
 * sweeps from T_start to T_end with Philox key `seed` (as gf_anneal) before the
 * fix-until iteration with params (as gf_fix_until; params->mode must equal the
 * pool's mode).  The links move in chunks through the staging buffer on the
 * transfer stream, beside a step in flight, which the job joins at the next
 * step.  Returns once host_links has been read and, for a job without
 * annealing, its first measurement taken (a non-finite one admits the job,
 * which finishes at once with GF_E_NUMERIC).  GF_E_FULL (nothing changed) when
 * no slot is free or the budget would be exceeded (lattices released during a
 * step in flight count until it is completed); GF_E_ARG for a duplicate job_id
 * or bad arguments.  Syncs the transfer stream. */
gf_status gf_pool_admit(gf_pool pool, uint64_t job_id, const int32_t dims[4], const double* host_links,
                        const gf_fix_params* params, int32_t anneal_sweeps, double T_start, double T_end,
                        uint64_t seed);

/* One pool step (see above): completes a step in flight, then runs the next.  Syncs. */
gf_status gf_pool_step(gf_pool pool);

/* Complete the step in flight (if any: wait for it, free lattices released
 * meanwhile, finish or advance its jobs, so that gf_pool_poll reports those
 * that finished), then plan and launch the next step and return without
 * waiting for it.  Launches nothing when no job is active. */
gf_status gf_pool_step_async(gf_pool pool);

/* Complete the step in flight, if any (as gf_pool_step_async does first).  Syncs. */
gf_status gf_pool_sync(gf_pool pool);

/* Move up to cap jobs that finished since the last poll into out[]; *n = count. */
gf_status gf_pool_poll(gf_pool pool, gf_pool_done* out, int32_t cap, int32_t* n);

/* Download a finished job's links (host canonical array) through the staging
 * buffer on the transfer stream, beside a step in flight, and free its
 * lattice (as gf_pool_release).  Syncs the transfer stream. */
gf_status gf_pool_fetch_links(gf_pool pool, uint64_t job_id, double* host);

/* Free a finished job's lattice without downloading it; while a step is in
 * flight the lattice is freed, and its bytes returned to the budget, when
 * that step is completed (freeing device memory synchronises the device). */
gf_status gf_pool_release(gf_pool pool, uint64_t job_id);

/* Cancel a resident job that has not finished (a step in flight is completed
 * first, so the job may finish in it instead): it takes no further part in
 * pool steps and is reported by the next gf_pool_poll with status
 * GF_E_CANCELLED and its last measured theta and F (converged = 0); its links
 * stay resident until gf_pool_release / gf_pool_fetch_links.  Other jobs are
 * unaffected.  GF_E_STATE if the job has already finished, GF_E_ARG if no
 * such job is resident. */
gf_status gf_pool_cancel(gf_pool pool, uint64_t job_id);

/* Autotuner of the pool's batched overrelaxation sweep (threads per site and
 * block size, Sec. 4 and 5 of the paper tune these at run time; a step in
 * flight is completed first): copies the
 * `kernel` links (GF_FP32: the float32 links and g(x) of a GF_MIXED pool;
 * GF_FP64: the float64 links) of the resident jobs, in slot order and up to
 * scratch_bytes of copies, times one warm-up and n_sweeps sweeps (both
 * colours) of that set for every shape (lanes per site 1, 2, 4; threads per
 * block 64, 128, 256; cache policy plain or non-temporal: 18 shapes) with HIP
 * events, in two rounds over all shapes of which each shape keeps its faster
 * time, writes up to cap entries to table (may be NULL; nontemporal = 0 plain,
 * 1 non-temporal), and makes the fastest the pool's shape and cache policy for
 * that kernel (*chosen, may be NULL).
 * The jobs' links are not changed.  GF_E_STATE if no resident job fits in
 * scratch_bytes.  Allocates and frees the copies.  Syncs. */
gf_status gf_pool_autotune(gf_pool pool, int32_t kernel, int32_t n_sweeps, size_t scratch_bytes,
                           gf_tune_entry* table, int32_t cap, int32_t* n_out, gf_tune_entry* chosen);

/* The pool's current sweep shape (any pointer may be NULL). */
gf_status gf_pool_get_shape(gf_pool pool, int32_t* tps32, int32_t* block32, int32_t* tps64, int32_t* block64);

/* The pool's current cache policy of the float32 / float64 overrelaxation
 * sweeps as in gf_pool_config (1 plain, 2 non-temporal; any pointer may be NULL). */
gf_status gf_pool_get_cache(gf_pool pool, int32_t* cache32, int32_t* cache64);

/* Resident jobs still iterating, finished jobs not yet released, and device
 * bytes held for job lattices (including those released during a step in
 * flight and not yet freed). */
gf_status gf_pool_stats(gf_pool pool, int32_t* active, int32_t* finished, int64_t* bytes_in_use);

/* Bandwidth probe: a plain float4 copy of `bytes` (>= 4096, multiple of 16)
 * between two fresh device buffers, `blocks` blocks of 256 threads striding
 * over it (nontemporal != 0: non-temporal loads and stores), timed over reps
 * launches on the default stream after one warm-up.  *gbps = 2*bytes*reps /
 * time (read + write).  Allocates and frees its buffers.  Syncs. */
gf_status gf_probe_copy(size_t bytes, int32_t reps, int32_t nontemporal, int32_t blocks, double* gbps);

/* Seconds on the library's steady clock (the clock of t_admit / t_done). */
double gf_clock(void);

/* Thread-local text of the last error (never NULL). */
const char* gf_last_error(void);

/* Library version string. */
const char* gf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GF_H */
