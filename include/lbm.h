/*
 * lbm.h -- C ABI of the MI355X limited lattice Boltzmann step.
 *
 * One time step is the LBGK step of Brownlee, Gorban & Levesley,
 * "Nonequilibrium entropy limiters in lattice Boltzmann methods"
 * (Physica A; arXiv:0704.0043), eq. (lbgkLB) of Sec. 4.2:
 *   free flight (Sec. 2) -> moments rho, u (eq. macro_dis) -> quasiequilibrium
 *   f* (eqs. polyeq1d, entropiceq1d, polyeq2d, maxwellian of Sec. 4.1) ->
 *   over-relaxation f' = f* + (2 beta - 1)(f* - f) (eq. collLBGK) ->
 *   nonequilibrium entropy Delta S(f') = sum f' ln(f'/f*) (eqs. locaNEQentropy,
 *   Kul, DelS) -> limiter f -> f* + phi (f' - f*) (eq. LimGenF) with
 *   entropy trimming (Sec. 3.2 Ehrenfests' step, Sec. 3.4 eq. entrHom) and/or
 *   the median entropy filter (Sec. 3.5, cavity stencils of Sec. 4.4).
 *
 * Units are lattice units (dx = dt = 1).  Populations are laid out as
 * structure-of-arrays planes f[i][y][x], x fastest; for D1Q3 ny = 1.
 * Velocity order: D1Q3 {0, -1, +1}; D2Q9 {rest, E, N, W, S, NE, NW, SW, SE}.
 *
 * Conventions shared by all functions:
 *  - Every function returns an int status: LBM_OK (0) or a negative code.
 *    On error, lbm_last_error(ctx) holds a message (ctx may be NULL for
 *    errors raised before a context exists; then a thread-local message is
 *    kept).  No function aborts or exits the process.
 *  - Host arrays are owned by the caller.  Inputs are copied during the
 *    call; outputs are written into caller-allocated arrays of the stated
 *    size.  Device memory is owned by the library unless the caller passes
 *    a workspace (then the caller keeps ownership and must keep it alive
 *    until lbm_destroy).
 *  - A context is used by one host thread at a time.
 *  - The "state at step t" is the post-free-flight (pre-collision) state
 *    f(x, t) of eq. (lbgkLB).  lbm_step is asynchronous with respect to the
 *    host (stream ordered); functions documented "sync" wait for the stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 3

#if defined(__GNUC__)
#define LBM_API __attribute__((visibility("default")))
#else
#define LBM_API
#endif

/* status codes */
#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument (sizes, beta, delta, enums, NULL) */
#define LBM_ENOMEM (-2)    /* device allocation failed or workspace too small */
#define LBM_EDEVICE (-3)   /* a HIP runtime error; message in lbm_last_error */
#define LBM_EUNSTABLE (-4) /* at a stats point: non-finite moments, or, with the exact Delta S
                              and neither trimming nor the positivity rule, a non-positive
                              population (Delta S = +inf, eq. DelS undefined) */
#define LBM_ERANGE (-5)    /* domain index out of range */

/* lattice (Sec. 4.1) */
enum lbm_lattice { LBM_D1Q3 = 1, LBM_D2Q9 = 2 };
/* quasiequilibrium: polynomial (polyeq1d/polyeq2d) or entropic
 * (entropiceq1d/maxwellian).  The D1Q3 entropic movers are taken with the
 * velocity they are labelled by: f*(v=+-1) = (rho/6)(+-3u - 1 + 2 sqrt(1+3u^2)). */
enum lbm_qe { LBM_QE_POLYNOMIAL = 0, LBM_QE_ENTROPIC = 1 };
/* limiter families, a bit mask: trimming (Sec. 3.2/3.4), median filter
 * (Sec. 3.5), and the ensemble-dependent limiters, which use the mean
 * E = E(Delta S') over the domain's fluid nodes of the same step:
 *   ENS_THRESHOLD  Delta S_t = max(ens_c E, delta_ens), homothety above it
 *                  (Sec. 4.3.2 with eq. entrHom)
 *   ENS_SMOOTH     phi = 1 / (1 + a Delta S^ens_k), a = delta_ens / E^ens_k
 *                  (eq. smooth1)
 *   ENS_RATIONAL   phi = (1 + r^(k - 1/2)) / (1 + r^k), r = Delta S / (ens_c E),
 *                  k = ens_k, kept <= 1 (eq. phiExamp)
 *   ENS_BUDGET     Delta S_t = max(Delta S_0, delta_ens) with Delta S_0 solving
 *                  sum max(Delta S - Delta S_0, 0) = ens_c [1 - (2 beta - 1)^2]
 *                  sum Delta S on the domain's values (eq. EntThresh), found by
 *                  a radix selection over the values' bit patterns whose
 *                  bucket sums are exact integers: the threshold does not
 *                  depend on the order of the additions (run to run equal).
 *                  No budget (ens_c = 0) puts it at the largest value; a
 *                  budget beyond sum Delta S puts it at 0
 * When several are on, phi is the smallest of their factors. */
enum lbm_limiter { LBM_LIM_NONE = 0, LBM_LIM_TRIM = 1, LBM_LIM_MEDIAN = 2, LBM_LIM_ENS_THRESHOLD = 4,
                   LBM_LIM_ENS_SMOOTH = 8, LBM_LIM_ENS_RATIONAL = 16, LBM_LIM_ENS_BUDGET = 32,
                   LBM_LIM_POSITIVITY = 64 };
/* LBM_LIM_POSITIVITY, the positivity rule (Sec. 2.1): a post-collision state
 * with a negative population is moved to the closest non-negative state on
 * the line through it and f*, phi = min f*_i / (f*_i - f'_i) over f'_i < 0.
 * On D2Q9 it combines with the median or ensemble limiters only with the
 * exact Delta S (LBM_EINVAL otherwise). */
/* collision: LBGK (eq. collLBGK), or ELBM (eqs. elbm, elbmLB): f' = f +
 * alpha beta (f* - f), alpha the nontrivial root of S((1 - alpha) f +
 * alpha f*) = S(f), found per node to full precision, never lowering the
 * entropy; when no such state is non-negative, the positivity rule (alpha at
 * the positivity boundary).  ELBM needs LBM_QE_ENTROPIC. */
enum lbm_collision { LBM_COLL_LBGK = 0, LBM_COLL_ELBM = 1 };
/* trimming: homothety to Delta S_t = delta (eq. entrHom) or Ehrenfests' step
 * f -> f* (Sec. 3.2) at sites with Delta S > delta */
enum lbm_trimmode { LBM_TRIM_HOMOTHETY = 0, LBM_TRIM_EHRENFEST = 1 };
/* median tolerance: FLOOR uses Delta S_t = max(Delta S_med, delta);
 * GATE corrects to Delta S_med only where Delta S > delta */
enum lbm_medmode { LBM_MED_FLOOR_DELTA = 0, LBM_MED_GATE_DELTA = 1 };
/* Delta S form: EXACT = sum f ln(f/f*) (eq. DelS / Kul), QUADRATIC =
 * sum (f - f*)^2 / (2 f*) (its second-order expansion, Sec. 3.6) */
enum lbm_dsform { LBM_DS_EXACT = 0, LBM_DS_QUADRATIC = 1 };
/* boundaries: periodic; lid-driven cavity with on-node bounce-back walls and
 * a constant equilibrium lid (Sec. 4.4.1); 1-D tube with half-way
 * bounce-back ends (Sec. 4.3); lid-driven cavity with diffusive Maxwell walls
 * (Sec. 4.4.2): a non-corner boundary node keeps what free flight brought,
 * except the populations pointing into the fluid, which become
 * gamma f*_i(1, u_wall) with gamma = (mass that arrived from the fluid) /
 * (mass of those f*_i); the lid moves with (lid_ux, 0), the other walls rest,
 * corners reflect every population; boundary nodes do not collide. */
enum lbm_bc { LBM_BC_PERIODIC = 0, LBM_BC_CAVITY = 1, LBM_BC_TUBE_ENDS = 2, LBM_BC_CAVITY_DIFFUSIVE = 3 };
/* population storage.  F64 stores f.  The others store the shift
 * g_i = f_i - w_i rho0 (w_i the lattice weights at rest) and compute in FP32;
 * global reductions are FP64 in every mode. */
enum lbm_storage { LBM_F64 = 0, LBM_F32 = 1, LBM_F16_SHIFT = 2, LBM_BF16_SHIFT = 3 };

/* limiter mask bits reported per node by lbm_limiter_mask */
#define LBM_MASK_TRIM 1u     /* Delta S' > trimming threshold */
#define LBM_MASK_MEDIAN 2u   /* median filter corrected the site */
#define LBM_MASK_NONPOS 4u   /* a population or f* was <= 0 (Delta S = +inf) */
#define LBM_MASK_NOTFLUID 8u /* wall or lid node: no collision, no limiter */
#define LBM_MASK_ENSEMBLE 16u /* an ensemble-dependent limiter moved the node (phi < 1) */
#define LBM_MASK_POSITIVITY 32u /* the positivity rule acted (limiter, or ELBM without a root) */

/* run flags */
#define LBM_RUN_RECORD 1u    /* keep per-node mask and Delta S' of every step */
#define LBM_RUN_ENTROPY 2u   /* also accumulate sum S(f) (Sec. 4.3.1) */
#define LBM_RUN_NO_GRAPH 4u  /* launch steps one by one (no captured graphs) */
#define LBM_RUN_NO_TUNE 8u   /* no timing of shapes: narrow row blocks where a domain allows
                                them, tile_h (or 64) for the second pass */
#define LBM_RUN_ADAPTIVE 16u /* D2Q9 LBGK domains with the median filter and no ensemble-
                                dependent limiter, tile_x other than 248: keep both forms of
                                the step, the two kernels (shapes tuned as usual) and the
                                fused step (tile height tuned; 8 rows with LBM_RUN_NO_TUNE),
                                and choose between them while the run goes.  At every
                                multiple of graph_chunk steps that lbm_step reaches, the
                                number of nodes the median filter moved in the step just
                                run is queued for reading back, and the form of the next
                                graph_chunk steps is chosen from the number queued at the
                                previous such point: the fused step once the filter moves
                                more than 0.5 % of the fluid nodes, the two kernels again
                                below 0.1 %; the two kernels first.  lbm_step then waits
                                for the stream to pass the previous point (it runs at most
                                about two chunks ahead).  The choice depends on the states
                                at those steps only (not on how the steps are split into
                                calls); the two forms take the same decisions and agree to
                                rounding (see tile_x = 248).  Else LBM_EINVAL */

/* One simulation domain.  All domains of one context share lattice, qe,
 * ds_form and bc (they run in the same kernel); sizes, beta, limiter and
 * thresholds may differ per domain. */
typedef struct {
    uint32_t struct_size;       /* = sizeof(lbm_domain_desc) */
    int32_t lattice;            /* enum lbm_lattice */
    int32_t nx, ny;             /* grid nodes; ny = 1 for D1Q3.  Cavity: nx, ny >= 4 */
    double beta;                /* over-relaxation, 0 <= beta <= 1 (eq. collLBGK) */
    int32_t qe;                 /* enum lbm_qe */
    int32_t limiter;            /* bit mask of enum lbm_limiter */
    int32_t trim_mode;          /* enum lbm_trimmode */
    int32_t median_mode;        /* enum lbm_medmode */
    int32_t ds_form;            /* enum lbm_dsform */
    int32_t bc;                 /* enum lbm_bc */
    double delta_trim;          /* trimming threshold delta >= 0 */
    double delta_median;        /* median tolerance delta >= 0 */
    double rho0;                /* reference density: storage shift, cavity lid density */
    double lid_ux;              /* cavity lid velocity u0 (lid state f*(rho0, (u0, 0))) */
    const double* rho_init;     /* nullable host [ny*nx]: initial density (default rho0) */
    const double* u_init;       /* nullable host [dim][ny*nx]: initial velocity (default 0) */
    const double* f_init;       /* nullable host [Q][ny*nx]: initial state, overrides rho/u */
    int32_t probe_x, probe_y;   /* node whose (ux, uy) is recorded each step; -1 = none */
    double ens_c;               /* ensemble limiters: c of the threshold c E, alpha of
                                   the rational phi, delta_0 of the budget; >= 0 */
    double ens_k;               /* exponent k of the smooth (> 0) and rational (>= 1/2) phi */
    double delta_ens;           /* floor delta of the thresholds; delta of a = delta / E^k */
    int32_t collision;          /* enum lbm_collision; same in every domain of a context */
    int32_t homothety;          /* 0: a homothety to Delta S_t scales f' - f* by sqrt(Delta S_t /
                                   Delta S') (eq. entrHom, exact in the quadratic form); 1: with
                                   the exact Delta S, by the root phi of Delta S(f* + phi (f' -
                                   f*)) = Delta S_t (Sec. 3.6); trimming, median, threshold and
                                   budget limiters */
    int64_t top_k;              /* > 0: trimming only at the top_k nodes of largest finite
                                   Delta S' above delta_trim (Sec. 3.2; ties at the k-th value
                                   included, Delta S' = +inf always), by a radix selection each
                                   step; not with LBM_LIM_ENS_BUDGET; 0: every node above delta */
} lbm_domain_desc;

typedef struct {
    uint32_t struct_size;       /* = sizeof(lbm_run_desc) */
    int32_t storage;            /* enum lbm_storage */
    int32_t device;             /* HIP device ordinal */
    int32_t stats_every;        /* >0: lbm_step synchronises every k steps and
                                   returns LBM_EUNSTABLE as lbm_entropy_stats does */
    int32_t tile_x;             /* D2Q9 collision row blocks (one node per thread, 256 per
                                   workgroup): 256 = one row of 256 columns per workgroup;
                                   64 = for a domain at most 128 wide, the narrowest of 64
                                   or 128 columns that spans its rows, with 4 or 2 rows per
                                   workgroup (wider domains keep 256); 0 = chosen by the
                                   autotuner (see lbm_create); 248 = the fused step: one kernel
                                   does the collision and the median filter (Sec. 3.5) over
                                   tiles of 248 columns (four waves of 62 owned columns each;
                                   LBGK domains with the median filter and no ensemble-dependent
                                   limiter only, else LBM_EINVAL).  Its cost does not depend on
                                   how many nodes the filter moves; the two kernels cost less
                                   while few move and more when many do (each moved node's
                                   stored state is read and written again).  The decisions are
                                   the same; a moved node's state is formed once as
                                   f* - phi c d (phi the smallest factor, eq. LimGenF), so its
                                   populations agree with the two-kernel step to rounding */
    int32_t tile_y;             /* 0 (or 1) */
    int32_t tile_h;             /* rows per D2Q9 second-pass tile (1..64); 0 = chosen by the
                                   autotuner among 16, 32 and 64 (64 without a second pass).
                                   With tile_x = 248: rows per fused tile (1..128), 0 = chosen
                                   among 4, 8, 16, 32 and 64 */
    uint32_t flags;             /* LBM_RUN_* */
    int32_t probe_capacity;     /* samples kept per probe (ring buffer), 0 = 4096 */
    int32_t graph_chunk;        /* longest captured step sequence, 1..4096, 0 = 64: lbm_create
                                   captures, for each starting parity, one graph of graph_chunk
                                   steps and one of each power of two below it, and lbm_step
                                   runs any count as replays of these (e.g. 20 = 16 + 4) */
    void* stream;               /* hipStream_t to run on; NULL = library-owned stream */
    void* workspace;            /* nullable device buffer (caller-owned) */
    size_t workspace_bytes;     /* its size; must be >= lbm_workspace_bytes() */
} lbm_run_desc;

typedef struct {
    uint32_t struct_size;       /* = sizeof(lbm_entropy_stats_t) */
    int64_t step;               /* number of completed steps; the sums below
                                   describe the last one (its input state) */
    double mass, mom_x, mom_y;  /* sum rho, sum rho u over all nodes */
    double sum_dS_pre;          /* sum over fluid nodes of Delta S(f) before collision */
    double sum_dS_post;         /* ... of Delta S(f') after collision */
    double max_dS;              /* max Delta S(f') (finite values) */
    double mean_dS;             /* sum_dS_post / n_fluid */
    double lbgk_production;     /* [1 - (2 beta - 1)^2] sum_dS_pre (Sec. 3.4) */
    double limiter_production;  /* sum (Delta S(f') - Delta S(f_limited)) (eq. LimEntLim) */
    double total_entropy;       /* sum S(f), S = -sum f ln(f/W); NaN unless LBM_RUN_ENTROPY */
    int64_t n_trimmed, n_filtered, n_nonpositive, n_nonfinite, n_fluid;
    int64_t n_ensemble;         /* nodes an ensemble-dependent limiter moved */
    double ens_threshold;       /* Delta S_t of ENS_BUDGET, else of ENS_THRESHOLD (0 if off) */
    int64_t n_positivity;       /* nodes the positivity rule moved (limiter, or ELBM without a root) */
} lbm_entropy_stats_t;

typedef struct lbm_ctx lbm_ctx;

/* Device bytes a context needs (for a caller-provided workspace). */
LBM_API int lbm_workspace_bytes(const lbm_domain_desc* domains, int32_t n_domains,
                        const lbm_run_desc* run, size_t* bytes);

/* Create a context: validates the descriptors, allocates (or carves the
 * workspace into) population buffers, builds f(x, 0) (f_init, or f*(rho, u))
 * and the work tables, and captures the step graphs.  D2Q9 autotuner: unless
 * LBM_RUN_NO_TUNE or fixed by tile_x / tile_h, the candidate shapes (row
 * blocks of 256 columns or narrow ones; second-pass tiles of 16, 32 or 64
 * rows; with tile_x = 248 the fused tile heights) are timed with HIP events
 * on a few steps that all read the initial state (which they leave
 * unchanged), each scored by a step as it stands plus one whose second pass
 * walks every tile, and the fastest is kept; the choice is
 * cached for the process under the descriptors, so later contexts of the
 * same problem reuse it.  The shapes do not change the fields or E(Delta S');
 * the FP64 sums the second pass adds to (limiter production) can differ in
 * the last bits.  Errors: EINVAL, ENOMEM, EDEVICE.  On error *out is NULL and
 * nothing is leaked. */
LBM_API int lbm_create(const lbm_domain_desc* domains, int32_t n_domains,
               const lbm_run_desc* run, lbm_ctx** out);

/* Advance every domain by n_steps >= 0 time steps (async, stream ordered),
 * as replays of the graphs captured at creation (unless LBM_RUN_NO_GRAPH).
 * With LBM_RUN_ADAPTIVE it waits, at each multiple of graph_chunk steps,
 * until the stream has passed the previous one. */
LBM_API int lbm_step(lbm_ctx* ctx, int64_t n_steps);

/* Wait for all queued work. */
LBM_API int lbm_synchronize(lbm_ctx* ctx);

/* sync.  rho [ny*nx], u [dim][ny*nx] (dim = 1 for D1Q3) of the current state;
 * either pointer may be NULL. */
LBM_API int lbm_moments(lbm_ctx* ctx, int32_t domain, double* rho, double* u);

/* sync.  Global sums of the last completed step (FP64).  Returns
 * LBM_EUNSTABLE (with *out filled) when n_nonfinite > 0, or when
 * n_nonpositive > 0 in a domain with the exact Delta S and neither trimming
 * nor the positivity rule (nothing sent those nodes back into the domain of
 * the entropy). */
LBM_API int lbm_entropy_stats(lbm_ctx* ctx, int32_t domain, lbm_entropy_stats_t* out);

/* sync.  Current state f[Q][ny*nx] as FP64 (reduced storage is widened). */
LBM_API int lbm_get_populations(lbm_ctx* ctx, int32_t domain, double* f);

/* sync.  Replace the current state with f[Q][ny*nx] (rounded to storage). */
LBM_API int lbm_set_populations(lbm_ctx* ctx, int32_t domain, const double* f);

/* sync.  Per-node limiter mask (LBM_MASK_* bits) and Delta S(f') of the last
 * step, [ny*nx] each; either pointer may be NULL.  Needs LBM_RUN_RECORD,
 * else LBM_EINVAL. */
LBM_API int lbm_limiter_mask(lbm_ctx* ctx, int32_t domain, uint8_t* mask, double* dS);

/* sync.  Probe samples (ux, uy) pairs, oldest first: writes
 * min(steps done, capacity, max_samples) pairs into uv[2*max_samples]. */
LBM_API int lbm_probe_trace(lbm_ctx* ctx, int32_t domain, float* uv, int64_t max_samples,
                    int64_t* n_written);

/* Shape in use (with LBM_RUN_ADAPTIVE, of the form the last step ran, or
 * the next step runs after a choice).  D2Q9: columns of the first domain's
 * collision row blocks (256, or 64 / 128 for a narrow domain), their rows
 * per workgroup, and the rows of a second-pass tile; the fused step: 248, 1
 * and the rows of a fused tile.  D1Q3: 254, 1, 1. */
LBM_API int lbm_tile_config(const lbm_ctx* ctx, int32_t* tile_x, int32_t* tile_y, int32_t* tile_h);

/* sync; profiling aid outside the method.  Advances the state by n_steps
 * (1..4096) like lbm_step, but launches every step eagerly (no graph) with
 * HIP events around each kernel on the context's stream, and writes the
 * average duration in milliseconds of the collision kernel to ms[0] and of
 * the rest of the step to ms[1]: the ensemble reductions and selection (when
 * an ensemble-dependent limiter is on) and the second pass (median filter,
 * ensemble factors); 0 when no second pass runs.  The stats of the
 * last step stay readable afterwards.  ms is a
 * caller-owned host array of 2 doubles.  LBM_EINVAL for a bad count or a
 * NULL pointer. */
LBM_API int lbm_kernel_times(lbm_ctx* ctx, int64_t n_steps, double* ms);

/* Release everything the context owns.  NULL is accepted. */
LBM_API void lbm_destroy(lbm_ctx* ctx);

/* Bytes of the static device array behind lbm_step_static (per GPU). */
#define LBM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
/* doubles written to lbm_step_static's stats array */
#define LBM_STATIC_NSTATS 14

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): advance
 * one domain by n_steps with the kernels of lbm_step, on population buffers
 * the caller owns, without any allocation.  Every other array a step uses
 * (the domain view, the work tables, the reduction partials, the Delta S'
 * plane, the step counters, the stats) lives in one
 * static device array of LBM_STATIC_SCRATCH_BYTES, one per GPU, which the
 * library holds until the process ends.  All calls on one GPU share it:
 * calls that overlap in time on one GPU (from two host threads, or on two
 * streams) race and give wrong results; calls in stream order are safe.
 * Each call clears what must start at zero (counters, stats, the
 * selection histogram) with its own kernels and launches nothing else, so a
 * call can be captured into a HIP graph.
 *   domain   one domain, as for lbm_create; f_init, rho_init and u_init must
 *            be NULL and probe_x, probe_y -1 (else LBM_EINVAL).
 *   storage  enum lbm_storage: the element type of f0 and f1.
 *   stream   hipStream_t to run on (NULL: the null stream); the device is
 *            the calling thread's current device.
 *   f0, f1   two distinct device buffers of Q * nx * ny elements of the
 *            storage type, planes [i][y][x] without padding (plane =
 *            nx * ny); F64 holds populations, the other types the shift
 *            g_i = f_i - w_i rho0.  A buffer holds the populations as they
 *            leave the nodes, before free flight: plane i at node x holds
 *            f_i(x + v_i) of the state f(x, t) of eq. (lbgkLB) (wrapped on a
 *            periodic grid; off a non-periodic edge, f_opp(i)(x)), which is
 *            how lbm_set_populations stores a state.  f0 holds the state at
 *            entry; step t reads f0 when t is even and f1 when odd and
 *            writes the other, so after n_steps the state is in f0 for even
 *            n_steps and in f1 for odd.  Caller-owned.
 *   n_steps  >= 0 (0 launches nothing).
 *   stats    nullable device array of LBM_STATIC_NSTATS doubles: the FP64
 *            sums of the last step in the order mass, mom_x, mom_y,
 *            sum_dS_pre, sum_dS_post, max_dS, limiter_production,
 *            n_trimmed, n_filtered, n_nonpositive, n_nonfinite, n_fluid,
 *            n_ensemble, n_positivity (as in lbm_entropy_stats_t).
 * Asynchronous (stream ordered).  Errors: LBM_EINVAL (descriptor, buffers,
 * n_steps < 0); LBM_ENOMEM when the domain needs more scratch than
 * LBM_STATIC_SCRATCH_BYTES (D2Q9 in FP32 with the median filter needs about
 * 4.7 bytes per node: up to some 14 million nodes; FP64 about 8.7); these
 * are detected before anything is launched; LBM_EDEVICE for a HIP error.
 * The message is in lbm_last_error(NULL). */
LBM_API int lbm_step_static(const lbm_domain_desc* domain, int32_t storage, void* stream, void* f0, void* f1,
                            int64_t n_steps, double* stats);

LBM_API const char* lbm_last_error(const lbm_ctx* ctx);
LBM_API const char* lbm_strerror(int code);

/* beta for kinematic viscosity nu with c_s^2 = 1/3: nu = (1/3)(1/(2 beta) - 1/2),
 * i.e. beta = 1/(6 nu + 1) (the LBGK viscosity of Sec. 2 for these lattices). */
LBM_API double lbm_beta_from_nu(double nu);

LBM_API int lbm_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
