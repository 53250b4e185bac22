/*
 * oracle.h -- plain FP64 CPU reference of the limited lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and oracle.c are the slow, obviously
 * correct checker that the GPU library is compared against.  Nothing in the
 * product library includes, links or calls them; only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load liboracle.so.
 *
 * Brownlee, Gorban, Levesley, "Nonequilibrium entropy limiters in lattice
 * Boltzmann methods" (Physica A, arXiv:0704.0043):
 *   - lattices and quasiequilibria: Sec. 4.1, eqs. (entropiceq1d), (polyeq1d),
 *     (maxwellian), (polyeq2d), moments eq. (macro_dis)
 *   - LBGK collision: eq. (collLBGK), Sec. 4.2 eq. (lbgkLB)
 *   - nonequilibrium entropy: eq. (locaNEQentropy), (Kul), (DelS) and its
 *     quadratic approximation (Sec. 3.6)
 *   - entropy trimming: Sec. 3.2 (Ehrenfests' step), Sec. 3.4 eq. (entrHom)
 *   - median entropy filter: Sec. 3.5, cavity stencil rule of Sec. 4.4
 *   - free flight: Sec. 2; bounce-back walls and constant lid: Sec. 4.4.1
 *
 * The median step (stencils with their periodic wrap, the FLOOR / GATE
 * decision on the post-collision Delta S, the landing on the target) is
 * checked against an independent restatement in the tests, and planted
 * mistakes in copies of this file are shown to fail those checks.  Still a
 * reading of the paper, with no printed value to check it against: which
 * nodes form the near-wall and corner stencils of the cavity (Sec. 4.4: three
 * nodes along a neighbouring wall, self plus two inner axis neighbours next
 * to a corner) and the lid density rho0; only the vortex centres of Table 1
 * (to within a node or two) constrain that reading.
 *
 * Layout: populations f[i*n + y*nx + x], n = nx*ny, x fastest (ny = 1 for
 * D1Q3).  The state passed in and out of orc_step is the post-streaming
 * (pre-collision) state f(x, t) of eq. (lbgkLB).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D1Q3 = 1, ORC_D2Q9 = 2 };
enum { ORC_QE_POLY = 0, ORC_QE_ENTROPIC = 1 };
enum { ORC_DS_EXACT = 0, ORC_DS_QUADRATIC = 1 };
/* limiter bits: trimming (Sec. 3.2), median filter (Sec. 3.5), and the
 * ensemble-dependent limiters, which use the mean E(Delta S) over the fluid
 * nodes: threshold max(c E, delta) (Sec. 4.3.2), smooth phi = 1/(1 + a DS^k)
 * with a = delta / E^k (eq. smooth1), the rational phi of eq. (phiExamp),
 * and the entropy-budget threshold of eq. (EntThresh) */
enum { ORC_LIM_TRIM = 1, ORC_LIM_MEDIAN = 2, ORC_LIM_ENS_THRESHOLD = 4, ORC_LIM_ENS_SMOOTH = 8,
       ORC_LIM_ENS_RATIONAL = 16, ORC_LIM_ENS_BUDGET = 32, ORC_LIM_POSITIVITY = 64 };
/* collision: LBGK (eq. collLBGK) or ELBM (eq. elbm, entropic f* only) */
enum { ORC_COLL_LBGK = 0, ORC_COLL_ELBM = 1 };
enum { ORC_TRIM_HOMOTHETY = 0, ORC_TRIM_EHRENFEST = 1 };
enum { ORC_MED_FLOOR = 0, ORC_MED_GATE = 1 };
/* boundaries: periodic; lid-driven cavity with on-node bounce-back walls and
 * an equilibrium lid (Sec. 4.4.1); 1-D tube with reflecting ends (Sec. 4.3);
 * lid-driven cavity with diffusive Maxwell walls (Sec. 4.4.2) */
enum { ORC_BC_PERIODIC = 0, ORC_BC_CAVITY = 1, ORC_BC_TUBE = 2, ORC_BC_CAVITY_DIFFUSIVE = 3 };

/* mask bits written per node by orc_step */
enum { ORC_MASK_TRIM = 1, ORC_MASK_MEDIAN = 2, ORC_MASK_NONPOS = 4,
       ORC_MASK_NOTFLUID = 8, ORC_MASK_ENSEMBLE = 16, ORC_MASK_POSITIVITY = 32 };

typedef struct {
    int32_t lattice, nx, ny;
    double beta;
    int32_t qe, ds_form, limiter, trim_mode, median_mode, bc;
    double delta_trim, delta_median;
    double rho0, lid_ux;    /* cavity lid: f*(rho0, (lid_ux, 0)) */
    int32_t entropy;        /* nonzero: also sum S(f) over fluid nodes */
    /* ensemble limiters: ens_c is c of the threshold c E, alpha of eq.
     * (phiExamp), delta_0 of eq. (EntThresh); ens_k the exponent k of eqs.
     * (smooth1) and (phiExamp); delta_ens the floor delta of the thresholds
     * and the delta of a = delta / E^k */
    double ens_c, ens_k, delta_ens;
    int32_t collision;      /* ORC_COLL_LBGK or ORC_COLL_ELBM */
    /* homothety to a threshold Delta S_t (trimming, median, threshold and
     * budget limiters): 0: phi = sqrt(Delta S_t / Delta S') (eq. entrHom,
     * exact in the quadratic form); 1: the root of
     * Delta S(f* + phi (f' - f*)) = Delta S_t (Sec. 3.6, exact form) */
    int32_t homothety;
    /* trimming at most at the top_k nodes of largest finite Delta S' > delta
     * (ties at the k-th value included; nodes with Delta S' = +inf always);
     * 0: every node above delta (Sec. 3.2) */
    int64_t top_k;
} orc_params;

typedef struct {
    double mass, mom_x, mom_y;
    double sum_dS_pre, sum_dS_post, max_dS;
    double lbgk_production, limiter_production, total_entropy;
    int64_t n_trimmed, n_filtered, n_nonpositive, n_nonfinite, n_fluid;
    int64_t n_ensemble;     /* nodes an ensemble limiter moved (phi < 1) */
    double mean_dS;         /* E(Delta S'): sum_dS_post / n_fluid */
    double ens_threshold;   /* Delta S_t of the budget limiter, else of the threshold limiter, else 0 */
    int64_t n_positivity;   /* nodes where the positivity rule acted (limiter, or ELBM without a root) */
} orc_stats;

/* threads the per-node loops of orc_step run on (1 unless built with OpenMP,
 * which only the CPU-baseline timing build is) */
int    orc_threads(void);
int    orc_q(int32_t lattice);
/* velocity components and entropy weights W_i of the paper's lattices */
void   orc_velocity(int32_t lattice, int32_t i, int32_t* vx, int32_t* vy);
int    orc_opposite(int32_t lattice, int32_t i);
/* f* for given rho, u (uy ignored for D1Q3); fstar has Q entries */
void   orc_equilibrium(int32_t lattice, int32_t qe, double rho, double ux,
                       double uy, double* fstar);
/* Delta S(f) relative to fstar; +inf when a logarithm is undefined */
double orc_delta_s(int32_t q, int32_t form, const double* f,
                   const double* fstar);
/* h(x) = (1+x) ln(1+x) - x, the per-population entropy kernel */
double orc_h(double x);
/* alpha of the ELBM step for f with entropic f* (Q entries each); sets
 * *posrule when the equation has no root short of the positivity boundary */
double orc_elbm_alpha(int32_t q, const double* f, const double* fstar, int32_t* posrule);
/* S(f) = -sum f_i ln(f_i / W_i) with the paper's W */
double orc_entropy(int32_t lattice, const double* f);
double orc_median(const double* v, int32_t n);
/* one LBGK step + limiter + free flight; mask, dS (Delta S of the
 * post-collision state) and dS_lim (Delta S of the limited state, the same
 * form) may be NULL */
int    orc_step(const orc_params* p, double* f, orc_stats* st, uint8_t* mask,
                double* dS, double* dS_lim);
/* free flight only: f = stream(o) (edge reflection at non-periodic edges) */
int    orc_stream(const orc_params* p, const double* o, double* f);
/* f = f*(rho, u) at every node; u is [dim][n] */
int    orc_init_equilibrium(const orc_params* p, const double* rho,
                            const double* u, double* f);

#ifdef __cplusplus
}
#endif
#endif
