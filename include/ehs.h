/*
 * ehs.h -- C ABI of the MI355X half-space spectral Ewald library.
 *
 * Fast summation of the half-space Green's functions of Stokes flow
 * (stokeslet, stresslet, rotlet with their wall images and harmonic
 * corrections), after Srinivasan & Tornberg, "Fast Ewald summation for
 * Green's functions of Stokes flow in a half-space":
 *
 *   u(x_t) = sum_m K(x_t - y_m) s_m - K(x_t - y_m^I) s_m^I
 *                  - x_t3 grad phi_m(x_t) + e_3 phi_m(x_t)
 *
 * (Sec. 3, eq. (v_sum_halfspace) with the potentials of eq. (phi)), split by
 * Ewald's method into a real-space sum over neighbours within r_c (Sec. 5.1)
 * and a Fourier-space part evaluated with Gaussian spreading, zero-padded
 * FFTs, scaling by the truncated-kernel multipliers, inverse FFTs and Gaussian
 * quadrature (Sec. 5.2, Algorithm 1).
 *
 * Normalisation: the kernels are S f = f/r + r(r.f)/r^3, T[g,q] =
 * -6 r (r.g)(r.q)/r^5 and the rotlet 2 W v = 2 (v x r)/r^3 (the paper's
 * 8 pi S, 8 pi T and 4 pi W of Sec. 2 without the constants); the wall is the
 * plane x3 = 0 and all points lie in x3 >= 0.
 *
 * Conventions for every entry point below:
 *  - all array pointers are DEVICE pointers (HIP memory of the context's
 *    device), row-major float64, owned by the caller; the library keeps no
 *    pointer after the call returns;
 *  - `stream` is a hipStream_t passed as void* (NULL: the default stream).
 *    The call returns after enqueueing; results are valid once the stream has
 *    synchronised.  Part of the work may run on a stream of the context's
 *    own (EHS_OPT_OVERLAP), forked from and joined back into `stream` by
 *    events, so that work ordered after the call on `stream` sees all of it.  One blocking device-to-host read (384 bytes: the bounding
 *    box, the validation counts, the strength measure and a histogram of the
 *    target heights) happens inside every call; a cache miss of the truncated-kernel precompute adds one
 *    more synchronisation;
 *  - sizes: 1 <= N < 2^30 sources and 0 <= T < 2^31 targets (else
 *    EHS_EINVAL, before anything is allocated); the workspace, about
 *    45 GB at N = T = 2^24 with ~2000 neighbours at tol 1e-6, bounds N
 *    before that;
 *  - outputs are overwritten, never accumulated;
 *  - a context is not thread safe and calls on one context must not overlap
 *    (they share the context's workspace);
 *  - return value: 0 on success or a negative EHS_E* code (ehs_strerror).
 */
#ifndef EHS_H
#define EHS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EHS_OK 0
#define EHS_EINVAL (-1)  /* null pointer, bad size or parameter */
#define EHS_EDOMAIN (-2) /* a source with y3 <= 0, a target with x3 < 0, or a non-finite input */
#define EHS_ERANGE (-3)  /* no admissible grid for the request (too fine, or eta >= 1) */
#define EHS_ENOMEM (-4)  /* device allocation failed or the memory cap is too small */
#define EHS_EHIP (-5)    /* a HIP runtime error */
#define EHS_ETIMEDOUT (-6) /* ehs_wait: the request has not completed within the timeout */
#define EHS_ETOOBIG (-7)   /* ewald_halfspace_noalloc: the problem does not fit its fixed scratch buffer */

/* kernel families */
#define EHS_STOKESLET 0
#define EHS_STRESSLET 1
#define EHS_ROTLET 2

/* options (ehs_set_option) */
#define EHS_OPT_PRECISION 0 /* 0: auto (FP32 when tol >= 1e-5 and est_fp32 <= tol/2, else FP64), 1: FP64, 2: FP32 */
#define EHS_OPT_TIMING 1    /* 1: record per-stage times into the report (adds a synchronisation) */
#define EHS_OPT_FORCE_M 2   /* > 0: use this M (grid intervals over the box) instead of the estimate */
#define EHS_OPT_FORCE_P 3   /* > 0: use this Gaussian support P (even) */
#define EHS_OPT_FORCE_MT 4  /* > 0: use this total grid size M~ (>= M + P, 7-smooth, even) */
#define EHS_OPT_MEM_CAP 5   /* > 0: bound on the workspace plus the cached octants, in bytes: octants of
                               other grid sizes are released to make room, else EHS_ENOMEM */
#define EHS_OPT_ZSLAB 6     /* > 0: k1 slabs per group of the y / x3 transform pipeline (default: sized for
                               the last-level cache); M~ + 1 keeps the whole grid in one group */
#define EHS_OPT_GATHER_EXTRA 7 /* >= 0 (even): support nodes the quadrature adds to P; -1: default (2 for
                                  FP64, whose quadrature forms the correction gradient, 0 for FP32) */
#define EHS_OPT_DGRID 8     /* FP64: 1 spreads the correction sources as one density with derivative
                               weights, 0 as separate grids, -1 (default) chooses by cost, and only
                               for tol >= 1e-12 (the density's rounding floor is about 1e-13) and
                               where its support fits 30 nodes; with the density the stresslet's
                               Gaussian support P grows by 2, which its second-derivative weights
                               need (1 with a support beyond 30 nodes: EHS_EINVAL) */
#define EHS_OPT_FAIL_PRECOMPUTE 9 /* test hook: > 0 makes the next that many truncated-kernel
                                     productions fail with EHS_EHIP before anything is launched */
#define EHS_OPT_CELL_REACH 10 /* 1..3: real-space cells of side >= r_c / value; 0 (default): chosen
                                 from the targets' density (ehs_report.occupancy) */
#define EHS_OPT_OVERLAP 11  /* 1 (default): the real-space sum runs on a stream of the context's own,
                               beside the grid stages on the caller's stream (joined by events before
                               the quadrature; the results are the same bit for bit); 0: everything on
                               the caller's stream.  With timing on, ms_stage[EHS_ST_REAL] is then the
                               overlapped sum's own time and the stages no longer add up to the total */
#define EHS_OPT_PARTS 12    /* test hook for the split of Sec. 4: 0 (default) the whole sum; 1 only the
                               real-space part (pairs within r_c, their images and corrections, and the
                               stokeslet's self term); 2 only the Fourier part (spreading, transforms,
                               scaling, quadrature).  Parts 1 and 2 add up to part 0 within rounding */
#define EHS_OPT_ADMISSION 13 /* servers only (ehs_server_set_option): 1 (default) smallest request first
                               (by workspace), one slot of two or more kept for requests of at most
                               65,536 points (N + T), the oldest request overtaken at most 8 times;
                               0 first come first served, younger requests overtaking a head that does
                               not fit at most 8 times */

/* stage indices of ehs_report.ms_stage */
#define EHS_ST_BBOX 0       /* bounding box + validation reduction and its readback */
#define EHS_ST_PRECOMP 1    /* truncated-kernel precompute (cache miss only) */
#define EHS_ST_BIN 2        /* cell keys, radix sorts, offsets, sorted copies */
#define EHS_ST_REAL 3       /* real-space sum */
#define EHS_ST_SPREAD 4     /* point keys, sort, records, spreading */
#define EHS_ST_FWDX 5       /* forward x1 pass (real to half spectrum) */
#define EHS_ST_FWDY 6       /* forward x2 pass */
#define EHS_ST_ZSCALE 7     /* fused x3 transform, scaling, inverse x3 transform */
#define EHS_ST_INVY 8       /* inverse x2 pass */
#define EHS_ST_INVX 9       /* inverse x1 pass */
#define EHS_ST_GATHER 10    /* quadrature at the targets + FP64 combination */
#define EHS_ST_TOTAL 11
#define EHS_NSTAGES 12

typedef struct ehs_ctx ehs_ctx;

typedef struct ehs_report {
    int32_t M, P, Mt;       /* grid intervals over the box, Gaussian support, total grid size M~ */
    int32_t precision;      /* 1: FP64, 2: FP32 */
    int32_t Q;              /* phases of the fused x3 pass */
    int32_t nf, nf3;        /* oversampled precompute grid (in-plane, x3) */
    int32_t warnings;       /* bit 0: real-space estimate above tol/2 (r_c too small for xi);
                               bit 1: the precompute ran in this call;
                               bit 2: FP32 requested but its rounding estimate exceeds tol/2 */
    int32_t ncell[3];       /* real-space cells per axis */
    int32_t family;
    double L, h, Lt, eta;   /* box, grid spacing, extended box M~ h, Gaussian shape */
    double xi, r_c, tol;
    double est_real, est_fourier; /* relative truncation estimates (Sec. 6, Tables 1-2) */
    double origin[3];       /* grid origin (the wall is at x3 = 0) */
    double ms_stage[EHS_NSTAGES]; /* stage times when EHS_OPT_TIMING is on, else 0 */
    double workspace_bytes;
    int32_t zslab;          /* k1 slabs per group of the y / x3 transform pipeline */
    int32_t Pg;             /* Gaussian support of the quadrature at the targets (>= P) */
    int32_t Ps;             /* Gaussian support of the spreading (>= P) */
    int32_t dgrid;          /* 1: correction sources spread as one density (FP64) */
    double est_fp32;        /* estimated FP32 rounding error (relative RMS, uniform point sets) */
    int32_t x3_first;       /* first x3 grid node the inverse transforms produce: the quadrature
                               of the lowest target reads no node below it */
    int32_t x3_corr_end;    /* x3 grid nodes from this one up lie above every image's Gaussian
                               support: the correction grids vanish there */
    int32_t cell_reach;     /* real-space cells have side >= r_c / cell_reach and are walked
                               (2 cell_reach + 1)^3 around a target's cell */
    double occupancy;       /* targets per real-space cell of side r_c, averaged over the targets
                               (from their height histogram, x1 and x2 taken as uniform) */
    double pairs_direct;    /* in-range (target, source) pairs of the real-space sum, direct and */
    double pairs_image;     /* image terms (counted when EHS_OPT_TIMING is on, else 0) */
    int32_t free_space;     /* 1: an ewald_freespace_* evaluation */
} ehs_report;

/* Smallest arena a context accepts (the table and bounding-box regions). */
#define EHS_ARENA_MIN_BYTES ((size_t)32 << 20)

/* Create a context on HIP device `hip_device`.
   arena_bytes == 0: the context grows its workspace and its cache of
   truncated-kernel octants (one set per grid size) on demand, with hipMalloc
   inside the calls that need more (EHS_OPT_MEM_CAP bounds both together).
   arena_bytes >= EHS_ARENA_MIN_BYTES: one device region of that size is
   allocated now, and every later evaluation takes its tables, the octants of
   its grid size and its workspace from it -- no allocation on the call path;
   the octants of the last grid size are kept and recomputed when the size
   changes; a problem that does not fit returns EHS_ENOMEM.
   Also resolves, for this device, the scratch of ewald_halfspace_noalloc.
   Returns EHS_OK, EHS_EINVAL (bad device or arena size), EHS_ENOMEM or
   EHS_EHIP; *out is NULL on error. */
int ehs_create(ehs_ctx** out, int hip_device, size_t arena_bytes);
/* Release the context and all its device memory (NULL is allowed). */
void ehs_destroy(ehs_ctx* ctx);
/* Set an EHS_OPT_* option; returns EHS_EINVAL for an unknown option. */
int ehs_set_option(ehs_ctx* ctx, int option, double value);

/*
 * Half-space stokeslet sum (Sec. 3 eq. (v_sum_halfspace) a).
 *   sources: N x 3 positions y_m (y_m3 > 0);  f: N x 3 forces;
 *   targets: T x 3 positions x_t (x_t3 >= 0), may alias `sources`;
 *   xi: Ewald parameter (> 0); r_c: real-space cutoff (> 0);
 *   tol: target relative RMS error in [1e-14, 1e-2];
 *   u_out: T x 3 velocities.
 * A target that coincides exactly with a source omits that source's direct
 * term (p != m of Sec. 2); its image and correction terms are kept.
 */
int ewald_halfspace_stokeslet(ehs_ctx* ctx, const double* sources, const double* f, int64_t N,
                              const double* targets, int64_t T, double xi, double r_c, double tol,
                              double* u_out, void* stream, ehs_report* rep);

/* Half-space stresslet sum (eq. (v_sum_halfspace) b); strengths N x 6 rows
   (g1, g2, g3, q1, q2, q3): strength g then orientation q.  Other arguments
   as for the stokeslet. */
int ewald_halfspace_stresslet(ehs_ctx* ctx, const double* sources, const double* gq, int64_t N,
                              const double* targets, int64_t T, double xi, double r_c, double tol,
                              double* u_out, void* stream, ehs_report* rep);

/* Half-space rotlet sum (eq. (v_sum_halfspace) c); strengths N x 3 torques
   v = g x q (the sum depends on g and q only through g x q). */
int ewald_halfspace_rotlet(ehs_ctx* ctx, const double* sources, const double* v, int64_t N,
                           const double* targets, int64_t T, double xi, double r_c, double tol,
                           double* u_out, void* stream, ehs_report* rep);

/*
 * Allocation-free evaluation, for callers that cannot allocate device memory
 * during a call (tight serving loops, harnesses that forbid hipMalloc).  The
 * same evaluation as ewald_halfspace_{stokeslet,stresslet,rotlet} (family
 * EHS_STOKESLET, EHS_STRESSLET or EHS_ROTLET; strengths N x 3, N x 6 or
 * N x 3; other arguments as there, options such as EHS_OPT_PRECISION from
 * ctx), but every buffer it needs -- stage tables, truncated-kernel octants,
 * grids, cell lists, sort scratch -- comes from one static device array of
 * EHS_NOALLOC_SCRATCH_BYTES per device, held from the library's first use on
 * that device until the process ends.  No hipMalloc, hipFree or other
 * allocating call is made; ctx supplies its device, options and pinned
 * readback buffer (its own workspace and cache are not touched).
 * The octants of the last grid size stay in the scratch and are recomputed
 * when the size changes.  The slab groups of the transform pipeline shrink
 * to fit; a problem that still does not fit returns EHS_ETOOBIG without
 * launching anything (enough for N = 1000 at tol 1e-10 with ~300 neighbours,
 * M~ = 64-80, for each of the three kernels).
 * Every call on a device shares that device's scratch: calls that overlap on
 * one device (other host threads, or other streams not yet synchronised)
 * race and give undefined results.  Each call overwrites every scratch byte
 * it reads before reading it, except the octants and tables it reuses.
 * Stage timing (EHS_OPT_TIMING) is not recorded by this entry point.
 */
#define EHS_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)
int ewald_halfspace_noalloc(ehs_ctx* ctx, int family, const double* sources, const double* strengths, int64_t N,
                            const double* targets, int64_t T, double xi, double r_c, double tol, double* u_out,
                            void* stream, ehs_report* rep);

/* Device memory a context holds: its workspace (or arena) bytes, the bytes
   and number of grid sizes of its octant cache.  Any output may be NULL. */
int ehs_context_memory(const ehs_ctx* ctx, double* workspace_bytes, double* cache_bytes, int* cache_entries);

/*
 * Free-space sums (Sec. 2, eq. (v_sum_free_space)): u(x_t) = sum_m K(x_t - y_m) s_m,
 * the kernels and strength layouts of the half-space entry points above, with
 * no wall: no images, no harmonic corrections, and no restriction on x3 (any
 * finite coordinates).  The same spectral Ewald method on the sources alone:
 * the kernel grid only (3, 6 and 3 forward transforms, 3 inverse), the
 * direct real-space terms only.  The grid keeps the half-space layout, with
 * the points in the lower half of its x3 range and the upper half empty
 * (skipped by the forward passes); the x3 transforms are therefore twice the
 * length a cubic box would need.  Arguments, ownership, synchronisation and
 * errors as for the half-space entry points (EHS_EDOMAIN only for non-finite
 * input).
 */
int ewald_freespace_stokeslet(ehs_ctx* ctx, const double* sources, const double* f, int64_t N,
                              const double* targets, int64_t T, double xi, double r_c, double tol,
                              double* u_out, void* stream, ehs_report* rep);
int ewald_freespace_stresslet(ehs_ctx* ctx, const double* sources, const double* gq, int64_t N,
                              const double* targets, int64_t T, double xi, double r_c, double tol,
                              double* u_out, void* stream, ehs_report* rep);
int ewald_freespace_rotlet(ehs_ctx* ctx, const double* sources, const double* v, int64_t N, const double* targets,
                           int64_t T, double xi, double r_c, double tol, double* u_out, void* stream,
                           ehs_report* rep);

/* Message for an EHS_* code (static storage). */
const char* ehs_strerror(int code);

/*
 * Ewald parameter xi for which the real-space truncation estimate of the
 * half-space sum (Sec. 6, Table 2 with sources and images counted) equals
 * tol/2 relative to sqrt(Q)/L, for cutoff r_c and box size L.  Host-only
 * arithmetic; returns a value > 0, or -1 for bad arguments.
 */
double ehs_xi_for_cutoff(int family, double r_c, double tol, double L);

/*
 * Cutoff r_c at which the real-space truncation estimate (as above) equals
 * `est` for the Ewald parameter xi and box size L: the inverse of
 * ehs_xi_for_cutoff in the other variable.  Host-only arithmetic; returns
 * -1 for bad arguments or when est is not reached for xi r_c in [1, 100].
 */
double ehs_cutoff_for_estimate(int family, double xi, double est, double L);

/*
 * Runtime-optimal Ewald parameter (the tuning procedure of Sec. 7): the two
 * truncation errors are held where the starting point (xi0, r_c0) puts them
 * while xi is perturbed, so that xi r_c and k_inf / xi stay (nearly)
 * constant and only the division of the work between the real-space sum
 * and the grid changes.  Candidates are xi = xi0 2^(k/8): r_c is the cutoff
 * with the starting point's real-space estimate (ehs_cutoff_for_estimate)
 * and the planner picks the grid from tol as always.  The search times
 * k = 0, then k = -2 and k = +2, and walks in steps of 2 in the faster
 * direction while the time falls; last it times the two neighbours k +- 1
 * of the fastest.  A walk stops at max_evals candidates (1..64), at a cutoff
 * above half the box, where no grid is admissible or the workspace does
 * not fit (EHS_ERANGE / EHS_ENOMEM of a candidate end the walk, they are not
 * returned), or, with FP32 forced (EHS_OPT_PRECISION 2), where the FP32
 * rounding estimate exceeds tol/2 (report warning bit 2) and the starting
 * point's did not.  Each candidate is evaluated once untimed (workspace and
 * multiplier precompute, which the paper's timings exclude too) and then
 * twice, timed on the host around a synchronised `stream`; its time is the
 * faster of the two.
 *   arguments as for the single-call entry points of `family` (0 stokeslet,
 *   1 stresslet, 2 rotlet; strengths N x 3, N x 6, N x 3), T >= 1;
 *   u_out: T x 3, on return the result at the chosen parameters;
 *   best: host array of 3, on return (xi, r_c, milliseconds) of the fastest
 *   candidate; trace (host, nullable): 3 max_evals values, (xi, r_c, ms) of
 *   every timed candidate in the order tried, their count in *ntrace
 *   (nullable); rep (nullable): the report of the final evaluation.
 * Synchronises `stream` repeatedly; returns 0 or the first error of an
 * evaluation other than the two that end the walk.  The context keeps the
 * multipliers of every grid size tried (as after any evaluation) and a
 * workspace sized for the largest candidate, until it is destroyed.
 */
int ehs_tune(ehs_ctx* ctx, int family, const double* sources, const double* strengths, int64_t N,
             const double* targets, int64_t T, double xi0, double r_c0, double tol, int max_evals,
             double* u_out, double* best, double* trace, int* ntrace, void* stream, ehs_report* rep);

/*
 * Parameter selection only (host arithmetic, no device work): the plan that
 * an evaluation would use for N sources, T targets in the bounding box
 * [lo, hi] (x3 of the box measured from the wall), strength measure Q (sum of
 * squared strength norms: |f|^2, |g|^2 |q|^2 or |v|^2), xi, r_c and tol.
 * precision: 0 auto, 1 FP64, 2 FP32.  Fills rep (workspace_bytes = bytes of
 * the workspace the evaluation would allocate).
 */
int ehs_plan_query(int family, int64_t N, int64_t T, const double* lo, const double* hi, double Q, double xi,
                   double r_c, double tol, int precision, ehs_report* rep);

/*
 * Truncated Green's function transforms of Sec. 5.2 evaluated on the host:
 * kind 0: H^R(k) = 8 pi sin^2(R k / 2) / k^2, the transform of (1/r) 1[r < R];
 * kind 1: the transform of the biharmonic kernel shifted by a constant,
 * (r - R) 1[r < R]: 4 pi [2 cos Rk + Rk sin Rk - 2] / k^4 (series near
 * k = 0).  The shift is invisible to the second and third derivatives
 * through which the biharmonic kernel enters.
 */
double ehs_truncated_kernel_hat(int kind, double k, double R);

/*
 * Unit-test entry: `nl` independent in-place-style FFTs of length n on the
 * context's device (in, out: device arrays of nl * n interleaved complex
 * values, float64 when fp32 == 0 else float32).  Unnormalised; inverse != 0
 * uses exp(+2 pi i k t / n).  n must factor into 2, 3, 5, 7.
 */
int ehs_debug_line_fft(ehs_ctx* ctx, int n, int nl, const void* in, void* out, int inverse, int fp32,
                       void* stream);

/*
 * Unit-test entry for the Gaussian spreading and quadrature (steps 5 and 10
 * of Algorithm 1): one evaluation exactly like ewald_halfspace_<family>
 * (free_space == 0) or ewald_freespace_<family> (free_space == 1), with
 * the same arguments, options and report, and two taps:
 *  - spread_out != NULL (device, spread_elems FP64 values): the grids as
 *    spread, before any transform, converted to FP64;
 *  - quad_in != NULL (device, quad_elems FP64 values): the grids the
 *    quadrature reads are replaced by these (converted to the evaluation's
 *    precision), and the real-space part is left out, so u_out holds the
 *    quadrature of quad_in alone.
 * Each grid is M~ x M~ x 2M~ values (report Mt), x1 fastest then x2 then
 * x3, node (i, j, l) at origin + h (i, j, l); the grids follow one another.
 * n_grids (may be NULL) receives the number of spread grids and of
 * quadrature grids of the plan:
 *  - spread grids: the kernel strengths at the sources and at their images
 *    (free space: sources only), then the correction sources at the images,
 *    either as separate grids or (report dgrid == 1) as one density with
 *    derivative weights;
 *  - quadrature grids: FP64 half space: the three velocity grids and the
 *    correction potential phi, whose gradient the quadrature takes with
 *    derivative weights; FP32 half space: the three velocity grids and the
 *    three grids of grad phi; free space: the three velocity grids.
 * A buffer below ngrids * M~^2 * 2M~ values gives EHS_EINVAL after the plan
 * (call once with NULL buffers to learn M~ and the counts).  Contexts
 * created with arena_bytes > 0 give EHS_EINVAL.  Not safe against other
 * calls on the same context at the same time.
 */
int ehs_debug_grid_taps(ehs_ctx* ctx, int family, int free_space, const double* sources, const double* strengths,
                        int64_t N, const double* targets, int64_t T, double xi, double r_c, double tol,
                        double* u_out, double* spread_out, int64_t spread_elems, const double* quad_in,
                        int64_t quad_elems, int32_t* n_grids, void* stream, ehs_report* report);

/*
 * Serving: continuous batching of many summation requests on one device.
 *
 * A server owns one device arena of `arena_bytes`.  Each request's workspace
 * (grids, cell lists, sort scratch) is carved from it when the request is
 * admitted and returned when it completes; the truncated-kernel multipliers
 * (one set per grid size M~) are cached in the same arena and shared by all
 * requests, evicted least recently used when no running request needs them.
 * `nslots` requests (1..16) run at once, each on its own stream and host
 * worker thread, so their device work overlaps.  A request is admitted as
 * soon as a slot is free and its footprint (workspace plus the multipliers it
 * still lacks) fits the arena; younger requests may overtake a queued request
 * that does not fit, a bounded number of times.  The arithmetic of a request
 * is exactly that of the single-call entry points with the same arguments.
 * There is no paper counterpart: the serving layer is an extension.
 */
typedef struct ehs_server ehs_server;

typedef struct ehs_request {
    int32_t family;    /* EHS_STOKESLET, EHS_STRESSLET or EHS_ROTLET */
    int32_t precision; /* 0 auto (FP32 when tol >= 1e-5 and the FP32 rounding estimate is at most
                          tol/2, else FP64), 1 FP64, 2 FP32 */
    int64_t N, T;
    /* device pointers, layouts as in ewald_halfspace_*; inputs must be complete
       on the device before ehs_submit, and every pointer stays valid and
       untouched until ehs_wait has returned the request */
    const double* sources;
    const double* strengths;
    const double* targets;
    double xi, r_c, tol;
    double* u_out;     /* T x 3, written by the request */
} ehs_request;

typedef struct ehs_request_status {
    int32_t code;          /* EHS_OK or the request's error */
    int32_t slot;          /* slot that ran it (-1: never admitted) */
    double t_submit_ms;    /* host steady clock, ms since the server was created */
    double t_admit_ms;     /* admission (slot and memory granted) */
    double t_done_ms;      /* results complete on the device and visible */
    double gpu_ms;         /* device time from the request's first to last operation */
    double footprint_bytes; /* arena bytes it needed: workspace plus its multipliers */
    ehs_report report;     /* the plan it ran with (ms_stage not filled) */
} ehs_request_status;

typedef struct ehs_server_stats {
    int64_t submitted, completed, failed, rejected;
    int32_t nslots, queued, running, cache_entries;
    int64_t cache_hits, cache_misses, evictions;
    double arena_bytes, arena_used, arena_peak, cache_bytes;
} ehs_serve_stats;

/* Create a server on `hip_device` with one arena of `arena_bytes` (allocated
   now) and `nslots` slots.  Returns EHS_OK, EHS_EINVAL, EHS_ENOMEM or
   EHS_EHIP; *out is NULL on error. */
int ehs_server_create(ehs_server** out, int hip_device, size_t arena_bytes, int nslots);
/* Wait for every submitted request to complete, then release the server and
   its arena.  Tickets not yet collected with ehs_wait are discarded. */
void ehs_server_destroy(ehs_server* srv);
/* Validate and plan a request (one small blocking readback for the bounding
   box, as in the single-call path) and queue it.  Argument and domain errors
   are returned here (EHS_EINVAL, EHS_EDOMAIN, EHS_ERANGE), as is EHS_ENOMEM
   when the request could never fit the arena; on EHS_OK *ticket identifies
   it.  Thread safe. */
int ehs_submit(ehs_server* srv, const ehs_request* req, uint64_t* ticket);
/* Wait up to timeout_ms (negative: no limit) for a request.  Returns
   EHS_ETIMEDOUT if it is still queued or running (the ticket stays valid);
   otherwise fills *status (may be NULL), releases the ticket and returns the
   request's own code.  EHS_EINVAL for an unknown ticket.  Thread safe. */
int ehs_wait(ehs_server* srv, uint64_t ticket, int timeout_ms, ehs_request_status* status);
/* Counters and arena occupancy.  Thread safe. */
int ehs_server_stats(ehs_server* srv, ehs_serve_stats* out);
/* Server options: EHS_OPT_ADMISSION (the admission rule, above) and
   EHS_OPT_FAIL_PRECOMPUTE (the next `value` octant productions fail with
   EHS_EHIP, for tests of the failure path); EHS_EINVAL for any other.
   Thread safe. */
int ehs_server_set_option(ehs_server* srv, int option, double value);

#ifdef __cplusplus
}
#endif
#endif /* EHS_H */
