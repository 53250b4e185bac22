/*
 * oracle.c -- plain FP64 CPU reference of the limited lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Loops in row-major node order,
 * no blocking or fusion: each function follows one formula of Brownlee,
 * Gorban & Levesley (arXiv:0704.0043) so that it can be checked against the
 * paper by eye.  Built with -O2 -ffp-contract=off.  The per-node loops carry
 * OpenMP pragmas: the build the tests use ignores them (no -fopenmp); a
 * separate build that only times the CPU baseline honours them.  The global
 * sums are formed afterwards from per-node terms in row-major order, so both
 * builds give the same bits.
 *
 * Readings of points where the paper is silent or garbled:
 *   - D1Q3 entropic f*: the printed left/right movers contradict the velocity
 *     labels of Sec. 4.1; the mover with velocity v = +-1 is taken as
 *     (rho/6)(+-3u - 1 + 2 sqrt(1+3u^2)), the 1-D factor of eq. (maxwellian).
 *   - Quadratic Delta S carries the factor 1/2 of the Taylor expansion
 *     (Sec. 3.6 prints it without).
 *   - The limiter acts on the post-collision state f' (Sec. 4.3.2: the limiter
 *     is a post-processing step immediately after collision).
 *   - Non-positive populations make the logarithm undefined: Delta S = +inf,
 *     so every enabled limiter returns the site to f*.
 *   - Free flight off the edge of a non-periodic grid is reflected into the
 *     same node's opposite population (half-way bounce-back at the tube ends;
 *     at cavity wall nodes it only touches populations that never reach the
 *     fluid).  With this rule free flight is a permutation.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- lattices (Sec. 4.1) ------------------------------------------------ */

/* D1Q3: static, left-moving (v = -1), right-moving (v = +1) in the paper's
 * order f1, f2, f3 (0-based here).  Entropy weights from
 * H = f1 log(f1/4) + f2 log f2 + f3 log f3. */
static const int D1_VX[3] = {0, -1, 1};
static const int D1_OPP[3] = {0, 2, 1};
static const double D1_W[3] = {4.0, 1.0, 1.0};

/* D2Q9: rest, E, N, W, S, NE, NW, SW, SE with weights 4/9, 1/9, 1/36. */
static const int D2_VX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int D2_VY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int D2_OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double D2_W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                               1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* threads the per-node loops run on (1 unless built with OpenMP) */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_q(int32_t lattice)
{
    if (lattice == ORC_D1Q3) return 3;
    if (lattice == ORC_D2Q9) return 9;
    return 0;
}

void orc_velocity(int32_t lattice, int32_t i, int32_t* vx, int32_t* vy)
{
    if (lattice == ORC_D1Q3) {
        *vx = D1_VX[i];
        *vy = 0;
    } else {
        *vx = D2_VX[i];
        *vy = D2_VY[i];
    }
}

int orc_opposite(int32_t lattice, int32_t i)
{
    return lattice == ORC_D1Q3 ? D1_OPP[i] : D2_OPP[i];
}

/* ---- quasiequilibria (Sec. 4.1) ----------------------------------------- */

void orc_equilibrium(int32_t lattice, int32_t qe, double rho, double ux,
                     double uy, double* fstar)
{
    if (lattice == ORC_D1Q3) {
        double u = ux;
        if (qe == ORC_QE_POLY) {
            /* eq. (polyeq1d) */
            fstar[0] = 2.0 * rho / 3.0 * (1.0 - 3.0 * u * u / 2.0);
            fstar[1] = rho / 6.0 * (1.0 - 3.0 * u + 3.0 * u * u);
            fstar[2] = rho / 6.0 * (1.0 + 3.0 * u + 3.0 * u * u);
        } else {
            /* eq. (entropiceq1d), movers assigned by their velocity */
            double s = sqrt(1.0 + 3.0 * u * u);
            fstar[0] = 2.0 * rho / 3.0 * (2.0 - s);
            fstar[1] = rho / 6.0 * (-3.0 * u - 1.0 + 2.0 * s);
            fstar[2] = rho / 6.0 * (3.0 * u - 1.0 + 2.0 * s);
        }
        return;
    }
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        if (qe == ORC_QE_POLY) {
            /* eq. (polyeq2d) */
            double cu = D2_VX[i] * ux + D2_VY[i] * uy;
            fstar[i] = rho * D2_W[i] *
                       (1.0 + 3.0 * cu + 9.0 * cu * cu / 2.0 - 3.0 * uu / 2.0);
        } else {
            /* eq. (maxwellian): product over the two axes */
            double prod = 1.0;
            double u[2] = {ux, uy};
            int v[2] = {D2_VX[i], D2_VY[i]};
            for (int j = 0; j < 2; ++j) {
                double s = sqrt(1.0 + 3.0 * u[j] * u[j]);
                double base = (2.0 * u[j] + s) / (1.0 - u[j]);
                double power = 1.0;
                if (v[j] == 1) power = base;
                if (v[j] == -1) power = 1.0 / base;
                prod *= (2.0 - s) * power;
            }
            fstar[i] = rho * D2_W[i] * prod;
        }
    }
}

/* ---- nonequilibrium entropy (Sec. 3.2, 3.6) ----------------------------- */

/* h(x) = (1+x) ln(1+x) - x.  With x_i = (f_i - f*_i)/f*_i,
 *   sum_i f_i ln(f_i/f*_i) = sum_i f*_i h(x_i) + sum_i (f_i - f*_i),
 * and the last sum vanishes because f and f* share their moments, so
 * eq. (DelS) equals sum_i f*_i h(x_i).  For small |x| the closed form
 * cancels, so its Taylor series sum_{n>=2} (-1)^n x^n / (n(n-1)) is used. */
double orc_h(double x)
{
    if (fabs(x) < 0.05) {
        double sum = 0.0;
        double power = x * x;
        for (int n = 2; n < 60; ++n) {
            double term = power / ((double)n * (double)(n - 1));
            if (n % 2 == 0)
                sum += term;
            else
                sum -= term;
            if (fabs(term) <= 1e-20 * fabs(sum)) break;
            power *= x;
        }
        return sum;
    }
    return (1.0 + x) * log1p(x) - x;
}

double orc_delta_s(int32_t q, int32_t form, const double* f,
                   const double* fstar)
{
    for (int i = 0; i < q; ++i)
        if (isnan(f[i]) || isnan(fstar[i])) return NAN;
    for (int i = 0; i < q; ++i)
        if (!(fstar[i] > 0.0)) return INFINITY;
    double sum = 0.0;
    if (form == ORC_DS_QUADRATIC) {
        /* sum_i (f_i - f*_i)^2 / (2 f*_i) */
        for (int i = 0; i < q; ++i) {
            double d = f[i] - fstar[i];
            sum += 0.5 * d * d / fstar[i];
        }
        return sum;
    }
    for (int i = 0; i < q; ++i)
        if (!(f[i] > 0.0)) return INFINITY;
    for (int i = 0; i < q; ++i)
        sum += fstar[i] * orc_h((f[i] - fstar[i]) / fstar[i]);
    return sum;
}

double orc_entropy(int32_t lattice, const double* f)
{
    int q = orc_q(lattice);
    const double* w = lattice == ORC_D1Q3 ? D1_W : D2_W;
    double s = 0.0;
    for (int i = 0; i < q; ++i) {
        if (!(f[i] > 0.0)) return NAN;
        s -= f[i] * log(f[i] / w[i]);
    }
    return s;
}

/* ---- ELBM collision (eqs. (elbm), (elbmLB), (entropy_estimate)) -----------
 * F(f) = (1 - beta) f + beta f~ with f~ = (1 - alpha) f + alpha f*, alpha the
 * nontrivial root of S(f~) = S(f).  With the entropic f*, ln(f*_i / W_i) is a
 * combination of the conserved quantities, so for every state g on the line
 * through f and f* (they share the moments) S(f*) - S(g) = sum g ln(g / f*)
 * = sum f*_i h(x_i(g)), x(g) = (g - f*) / f*.  The deviation of f~ is
 * (1 - alpha) x, so the equation reads
 *     sum f*_i h((1 - alpha) x_i) = sum f*_i h(x_i),
 * the same equation as a difference of entropies, but one that keeps its
 * precision when f is close to f*.  It is solved by bisection in alpha on
 * [1, alpha_max] to 1e-15, where alpha_max is the positivity boundary of f~
 * (the first population of f~ reaching 0); the lower end of the final
 * bracket is returned, so the entropy does not decrease.  When the equation
 * has no root short of alpha_max, the positivity rule: f~ stops on the
 * positivity boundary (alpha = alpha_max). */

/* h with its limit h(-1) = 1 (a population at exactly zero) */
static double h_closed(double x)
{
    return x <= -1.0 ? 1.0 : orc_h(x);
}

double orc_elbm_alpha(int32_t q, const double* f, const double* fstar, int32_t* posrule)
{
    double x[9], target = 0.0, smax = INFINITY;
    *posrule = 0;
    for (int i = 0; i < q; ++i) {
        x[i] = (f[i] - fstar[i]) / fstar[i];
        if (x[i] > 0.0 && 1.0 / x[i] < smax) smax = 1.0 / x[i];
    }
    if (!isfinite(smax)) return 2.0;             /* f = f*: every alpha gives f */
    int nonpos = 0;
    for (int i = 0; i < q; ++i) {
        if (x[i] <= -1.0) nonpos = 1;
        target += fstar[i] * h_closed(x[i]);
    }
    /* in s = alpha - 1: G(s) = sum f* h(-s x) - target, G(0) < 0, increasing */
    double g_max = -target;
    for (int i = 0; i < q; ++i) g_max += fstar[i] * h_closed(-smax * x[i]);
    if (nonpos || g_max < 0.0) {
        /* no state of entropy S(f) on the non-negative part of the line (or f
         * itself has no entropy): positivity rule */
        *posrule = 1;
        return 1.0 + smax;
    }
    double lo = 0.0, hi = smax;
    while (hi - lo > 1e-15) {
        const double mid = 0.5 * (lo + hi);
        double g = -target;
        for (int i = 0; i < q; ++i) g += fstar[i] * h_closed(-mid * x[i]);
        if (g <= 0.0) lo = mid;
        else hi = mid;
        if (mid == lo && mid == hi) break;
    }
    return 1.0 + lo;
}

/* Homothety toward f* down to Delta S = t (eq. entrHom): phi = sqrt(t / d),
 * which reaches t exactly in the quadratic form; with p->homothety and the
 * exact form, the root of Delta S(f* + phi (f' - f*)) = t (Sec. 3.6), by
 * bisection on [0, 1] to 1e-15, taking the lower end (the limited state does
 * not exceed t).  Delta S' = +inf gives 0. */
static double homothety_phi(const orc_params* p, int q, const double* fpost, const double* fs, double d, double t)
{
    if (!isfinite(d)) return 0.0;
    if (!p->homothety || p->ds_form == ORC_DS_QUADRATIC) return sqrt(t / d);
    double lo = 0.0, hi = 1.0, g[9];
    while (hi - lo > 1e-15) {
        const double mid = 0.5 * (lo + hi);
        for (int i = 0; i < q; ++i) g[i] = fs[i] + mid * (fpost[i] - fs[i]);
        if (orc_delta_s(q, ORC_DS_EXACT, g, fs) <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

/* Sec. 3.5: sort the neighbourhood, take the middle value. */
double orc_median(const double* v, int32_t n)
{
    double a[27];
    for (int i = 0; i < n; ++i) a[i] = v[i];
    for (int i = 1; i < n; ++i) {
        double key = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > key) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = key;
    }
    return a[n / 2];
}

/* ---- grid helpers -------------------------------------------------------- */

enum { NODE_FLUID = 0, NODE_WALL = 1, NODE_LID = 2 };

static int node_type(const orc_params* p, int x, int y)
{
    if (p->bc != ORC_BC_CAVITY && p->bc != ORC_BC_CAVITY_DIFFUSIVE) return NODE_FLUID;
    if (x == 0 || x == p->nx - 1 || y == 0) return NODE_WALL;
    if (y == p->ny - 1) return NODE_LID;
    return NODE_FLUID;
}

static int wrap(int a, int n)
{
    return ((a % n) + n) % n;
}

static int check_params(const orc_params* p)
{
    if (p->lattice != ORC_D1Q3 && p->lattice != ORC_D2Q9) return -1;
    if (p->nx < 1 || p->ny < 1) return -1;
    if (p->lattice == ORC_D1Q3 && p->ny != 1) return -1;
    if (!(p->beta >= 0.0 && p->beta <= 1.0)) return -1;
    if (!(p->delta_trim >= 0.0) || !(p->delta_median >= 0.0)) return -1;
    if (p->limiter & (ORC_LIM_ENS_THRESHOLD | ORC_LIM_ENS_SMOOTH | ORC_LIM_ENS_RATIONAL | ORC_LIM_ENS_BUDGET)) {
        if (!(p->delta_ens >= 0.0) || !(p->ens_c >= 0.0) || !(p->ens_k > 0.0)) return -1;
        if ((p->limiter & ORC_LIM_ENS_RATIONAL) && !(p->ens_c > 0.0 && p->ens_k >= 0.5)) return -1;
    }
    if (p->collision != ORC_COLL_LBGK && p->collision != ORC_COLL_ELBM) return -1;
    if (p->homothety != 0 && p->homothety != 1) return -1;
    if (p->top_k < 0) return -1;
    if (p->collision == ORC_COLL_ELBM && p->qe != ORC_QE_ENTROPIC) return -1;
    if (p->bc == ORC_BC_CAVITY || p->bc == ORC_BC_CAVITY_DIFFUSIVE) {
        if (p->lattice != ORC_D2Q9 || p->nx < 4 || p->ny < 4) return -1;
    } else if (p->bc == ORC_BC_TUBE) {
        if (p->lattice != ORC_D1Q3 || p->nx < 2) return -1;
    } else if (p->bc != ORC_BC_PERIODIC) {
        return -1;
    }
    return 0;
}

/* Median stencil of node (x, y); returns the number of points (0: the node
 * is not filtered).  Cavity rule of Sec. 4.4: boundary nodes are not
 * filtered, nodes next to the boundary use three nodes along the boundary
 * (next to two walls: the node and its two inner axis neighbours), all other
 * nodes the 3x3 neighbourhood. */
static int median_stencil(const orc_params* p, int x, int y, int* sx, int* sy)
{
    int nx = p->nx, ny = p->ny;
    if (p->lattice == ORC_D1Q3) {
        if (p->bc == ORC_BC_TUBE && (x == 0 || x == nx - 1)) return 0;
        for (int k = 0; k < 3; ++k) {
            sx[k] = wrap(x - 1 + k, nx);
            sy[k] = 0;
        }
        return 3;
    }
    if (p->bc == ORC_BC_PERIODIC) {
        int k = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                sx[k] = wrap(x + dx, nx);
                sy[k] = wrap(y + dy, ny);
                ++k;
            }
        return 9;
    }
    if (node_type(p, x, y) != NODE_FLUID) return 0;
    int near_l = x == 1, near_r = x == nx - 2;
    int near_b = y == 1, near_t = y == ny - 2;
    if ((near_l || near_r) && (near_b || near_t)) {
        int ix = near_l ? 1 : -1;
        int iy = near_b ? 1 : -1;
        sx[0] = x;      sy[0] = y;
        sx[1] = x + ix; sy[1] = y;
        sx[2] = x;      sy[2] = y + iy;
        return 3;
    }
    if (near_l || near_r) {
        for (int k = 0; k < 3; ++k) {
            sx[k] = x;
            sy[k] = y - 1 + k;
        }
        return 3;
    }
    if (near_b || near_t) {
        for (int k = 0; k < 3; ++k) {
            sx[k] = x - 1 + k;
            sy[k] = y;
        }
        return 3;
    }
    int k = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            sx[k] = x + dx;
            sy[k] = y + dy;
            ++k;
        }
    return 9;
}

/* ---- free flight (Sec. 2) ------------------------------------------------ */

int orc_stream(const orc_params* p, const double* o, double* f)
{
    if (check_params(p)) return -1;
    int q = orc_q(p->lattice), nx = p->nx, ny = p->ny, n = nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < q; ++i) {
                int vx, vy;
                orc_velocity(p->lattice, i, &vx, &vy);
                int tx = x + vx, ty = y + vy;
                double val = o[i * n + y * nx + x];
                if (p->bc == ORC_BC_PERIODIC) {
                    tx = wrap(tx, nx);
                    ty = wrap(ty, ny);
                    f[i * n + ty * nx + tx] = val;
                } else if (tx >= 0 && tx < nx && ty >= 0 && ty < ny) {
                    f[i * n + ty * nx + tx] = val;
                } else {
                    /* leaves the grid: comes back reversed at the same node */
                    int j = orc_opposite(p->lattice, i);
                    f[j * n + y * nx + x] = val;
                }
            }
    return 0;
}

int orc_init_equilibrium(const orc_params* p, const double* rho,
                         const double* u, double* f)
{
    if (check_params(p)) return -1;
    int q = orc_q(p->lattice), n = p->nx * p->ny;
    double fs[9];
    for (int s = 0; s < n; ++s) {
        double uy = p->lattice == ORC_D2Q9 ? u[n + s] : 0.0;
        orc_equilibrium(p->lattice, p->qe, rho[s], u[s], uy, fs);
        for (int i = 0; i < q; ++i) f[i * n + s] = fs[i];
    }
    return 0;
}

/* ---- diffusive Maxwell walls (Sec. 4.4.2) --------------------------------
 * A boundary node that is not a corner keeps the populations that arrived
 * along the wall or from the fluid; those that point into the fluid (a
 * positive component along the wall's inward normal) are replaced by
 * gamma f*_i(1, u_wall), with gamma the ratio of the mass that arrived from
 * the fluid (populations with a negative normal component) to the mass of
 * those quasiequilibrium populations: the wall returns what it received,
 * distributed as the quasiequilibrium of the wall's velocity.  The density of
 * the wall's f* cancels in gamma, so it is 1.  The lid moves with (u0, 0),
 * the other walls rest.  A corner reflects every population (there the rule
 * coincides with bounce-back).  No collision at boundary nodes. */
static void diffusive_wall(const orc_params* p, int x, int y, const double* fl, double* out)
{
    const int nx = p->nx, ny = p->ny;
    if ((x == 0 || x == nx - 1) && (y == 0 || y == ny - 1)) {
        for (int i = 0; i < 9; ++i) out[i] = fl[orc_opposite(ORC_D2Q9, i)];
        return;
    }
    int mx = 0, my = 0;
    double uw = 0.0;
    if (y == 0) {
        my = 1;
    } else if (y == ny - 1) {
        my = -1;
        uw = p->lid_ux;
    } else if (x == 0) {
        mx = 1;
    } else {
        mx = -1;
    }
    double fs[9];
    orc_equilibrium(ORC_D2Q9, p->qe, 1.0, uw, 0.0, fs);
    double sum_in = 0.0, sum_arrived = 0.0;
    for (int i = 0; i < 9; ++i) {
        int vx, vy;
        orc_velocity(ORC_D2Q9, i, &vx, &vy);
        const int d = vx * mx + vy * my;
        if (d > 0) sum_in += fs[i];
        if (d < 0) sum_arrived += fl[i];
    }
    const double gamma = sum_arrived / sum_in;
    for (int i = 0; i < 9; ++i) {
        int vx, vy;
        orc_velocity(ORC_D2Q9, i, &vx, &vy);
        out[i] = vx * mx + vy * my > 0 ? gamma * fs[i] : fl[i];
    }
}

/* ---- one time step -------------------------------------------------------
 * eq. (lbgkLB): collide every fluid node toward f*, apply the limiter to the
 * post-collision state (eq. (LimGenF) with the trimming or median rule),
 * then free flight.  Cavity walls: bounce-back (reverse all populations, no
 * collision); lid nodes: set to f*(rho0, (u0, 0)) (Sec. 4.4.1). */
static int cmp_descending(const void* a, const void* b)
{
    const double x = *(const double*)a, y = *(const double*)b;
    return (x < y) - (x > y);
}

/* eq. (EntThresh) on the empirical distribution of the m finite values d
 * (sorted here in descending order): the Delta S0 >= 0 with
 * sum_x max(d_x - Delta S0, 0) = budget.  The left side is continuous and
 * decreasing in Delta S0, linear between consecutive sorted values: with the
 * k largest values above Delta S0 it reads S_k - k Delta S0. */
static double budget_threshold(double* d, int m, double budget)
{
    if (m == 0) return 0.0;
    qsort(d, (size_t)m, sizeof(double), cmp_descending);
    if (!(budget > 0.0)) return d[0];
    double sum = 0.0;
    for (int k = 1; k <= m; ++k) {
        sum += d[k - 1];
        const double next = k < m ? d[k] : 0.0;
        const double t = (sum - budget) / k;
        if (t >= next) return t > 0.0 ? t : 0.0;
    }
    return 0.0;
}

int orc_step(const orc_params* p, double* f, orc_stats* st, uint8_t* mask,
             double* dS, double* dS_lim)
{
    if (check_params(p)) return -1;
    const int q = orc_q(p->lattice), nx = p->nx, ny = p->ny, n = nx * ny;
    const double c = 2.0 * p->beta - 1.0;

    double* fst = (double*)malloc(sizeof(double) * q * n);
    double* fpost = (double*)malloc(sizeof(double) * q * n);
    double* o = (double*)malloc(sizeof(double) * q * n);
    double* dpre = (double*)malloc(sizeof(double) * n);
    double* dpost = (double*)malloc(sizeof(double) * n);
    uint8_t* m = (uint8_t*)calloc(n, 1);
    /* per-node terms of the global sums, summed in row-major order after
     * each pass (the per-node loops are then independent of each other) */
    double* srho = (double*)malloc(sizeof(double) * n);
    double* sjx = (double*)malloc(sizeof(double) * n);
    double* sjy = (double*)malloc(sizeof(double) * n);
    double* sent = (double*)malloc(sizeof(double) * n);
    double* slim = (double*)malloc(sizeof(double) * n);
    uint8_t* npos = (uint8_t*)calloc(n, 1);     /* positivity rule acted (0..2 times) */
    uint8_t* limon = (uint8_t*)calloc(n, 1);    /* slim holds a term */
    if (!fst || !fpost || !o || !dpre || !dpost || !m || !srho || !sjx || !sjy || !sent || !slim || !npos ||
        !limon) {
        free(fst); free(fpost); free(o); free(dpre); free(dpost); free(m);
        free(srho); free(sjx); free(sjy); free(sent); free(slim); free(npos); free(limon);
        return -2;
    }

    orc_stats s;
    memset(&s, 0, sizeof(s));
    if (dS_lim)
        for (int k = 0; k < n; ++k) dS_lim[k] = 0.0;
    s.total_entropy = p->entropy ? 0.0 : NAN;

    /* pass 1: moments, collision, Delta S of every node */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int site = y * nx + x;
            double fl[9], fs[9], fp[9];
            double rho = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < q; ++i) {
                int vx, vy;
                orc_velocity(p->lattice, i, &vx, &vy);
                fl[i] = f[i * n + site];
                rho += fl[i];
                jx += vx * fl[i];
                jy += vy * fl[i];
            }
            srho[site] = rho;
            sjx[site] = jx;
            sjy[site] = jy;
            sent[site] = NAN;
            dpre[site] = 0.0;
            dpost[site] = 0.0;
            int type = node_type(p, x, y);
            if (type != NODE_FLUID && p->bc == ORC_BC_CAVITY_DIFFUSIVE) {
                diffusive_wall(p, x, y, fl, fp);
                for (int i = 0; i < q; ++i) o[i * n + site] = fp[i];
                m[site] = ORC_MASK_NOTFLUID;
                continue;
            }
            if (type == NODE_WALL) {
                for (int i = 0; i < q; ++i)
                    o[i * n + site] = fl[orc_opposite(p->lattice, i)];
                m[site] = ORC_MASK_NOTFLUID;
                continue;
            }
            if (type == NODE_LID) {
                orc_equilibrium(p->lattice, p->qe, p->rho0, p->lid_ux, 0.0, fs);
                for (int i = 0; i < q; ++i) o[i * n + site] = fs[i];
                m[site] = ORC_MASK_NOTFLUID;
                continue;
            }
            double ux = jx / rho, uy = jy / rho;   /* eq. (macro_dis) */
            orc_equilibrium(p->lattice, p->qe, rho, ux, uy, fs);
            if (p->collision == ORC_COLL_ELBM) {
                /* eq. (elbmLB): f + alpha beta (f* - f) */
                int32_t pr = 0;
                const double alpha = orc_elbm_alpha(q, fl, fs, &pr);
                for (int i = 0; i < q; ++i) fp[i] = fl[i] + alpha * p->beta * (fs[i] - fl[i]);
                if (pr) {
                    m[site] |= ORC_MASK_POSITIVITY;
                    npos[site]++;
                }
            } else {
                for (int i = 0; i < q; ++i)      /* eq. (collLBGK) */
                    fp[i] = fs[i] + c * (fs[i] - fl[i]);
            }
            dpre[site] = orc_delta_s(q, p->ds_form, fl, fs);
            dpost[site] = orc_delta_s(q, p->ds_form, fp, fs);
            for (int i = 0; i < q; ++i) {
                fst[i * n + site] = fs[i];
                fpost[i * n + site] = fp[i];
            }
            if (p->entropy) sent[site] = orc_entropy(p->lattice, fl);
        }
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int site = y * nx + x;
            s.mass += srho[site];
            s.mom_x += sjx[site];
            s.mom_y += sjy[site];
            if (!isfinite(srho[site]) || !isfinite(sjx[site]) || !isfinite(sjy[site])) s.n_nonfinite++;
            if (node_type(p, x, y) == NODE_FLUID) s.n_fluid++;
            if (isfinite(sent[site])) s.total_entropy += sent[site];
        }

    /* ensemble quantities of the post-collision Delta S (Sec. 3.3, 3.4):
     * E = mean over the fluid nodes (non-finite values left out of the sum),
     * and the thresholds of the ensemble limiters */
    const int ens = p->limiter & (ORC_LIM_ENS_THRESHOLD | ORC_LIM_ENS_SMOOTH | ORC_LIM_ENS_RATIONAL |
                                  ORC_LIM_ENS_BUDGET);
    double mean_ds = 0.0, t_thresh = 0.0, t_budget = 0.0;
    {
        double sum = 0.0;
        int64_t nf = 0, nfin = 0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (node_type(p, x, y) != NODE_FLUID) continue;
                nf++;
                if (isfinite(dpost[y * nx + x])) {
                    sum += dpost[y * nx + x];
                    nfin++;
                }
            }
        mean_ds = nf > 0 ? sum / (double)nf : 0.0;
        t_thresh = p->ens_c * mean_ds > p->delta_ens ? p->ens_c * mean_ds : p->delta_ens;
        if (p->limiter & ORC_LIM_ENS_BUDGET) {
            double* vals = (double*)malloc(sizeof(double) * (nfin > 0 ? nfin : 1));
            int mv = 0;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    if (node_type(p, x, y) == NODE_FLUID && isfinite(dpost[y * nx + x]))
                        vals[mv++] = dpost[y * nx + x];
            const double b = p->ens_c * (1.0 - c * c) * sum;
            const double s0 = budget_threshold(vals, mv, b);
            free(vals);
            t_budget = s0 > p->delta_ens ? s0 : p->delta_ens;
        }
    }

    /* top-k trimming (Sec. 3.2): the k-th largest finite Delta S' above
     * delta; trimming then acts where Delta S' >= that value */
    double topk_value = -INFINITY;
    if ((p->limiter & ORC_LIM_TRIM) && p->top_k > 0) {
        double* vals = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
        int mv = 0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const double d = dpost[y * nx + x];
                if (node_type(p, x, y) == NODE_FLUID && isfinite(d) && d > p->delta_trim) vals[mv++] = d;
            }
        if (mv > p->top_k) {
            qsort(vals, (size_t)mv, sizeof(double), cmp_descending);
            topk_value = vals[p->top_k - 1];
        }
        free(vals);
    }

    /* pass 2: limiter on the post-collision state */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int site = y * nx + x;
            if (node_type(p, x, y) != NODE_FLUID) continue;
            double d = dpost[site];
            double dp = dpre[site];
            if (isinf(d) || isinf(dp)) m[site] |= ORC_MASK_NONPOS;
            double phi = 1.0;
            double fpn[9], fsn[9];              /* f' and f* of this node */
            for (int i = 0; i < q; ++i) {
                fpn[i] = fpost[i * n + site];
                fsn[i] = fst[i * n + site];
            }
            if (p->limiter & ORC_LIM_TRIM) {
                /* eq. (entrHom) with Delta S_t = delta, or an Ehrenfests' step */
                double t = p->delta_trim;
                if (d > t && (isinf(d) || d >= topk_value)) {
                    m[site] |= ORC_MASK_TRIM;
                    double pt = p->trim_mode == ORC_TRIM_EHRENFEST
                                    ? 0.0
                                    : homothety_phi(p, q, fpn, fsn, d, t);
                    if (pt < phi) phi = pt;
                }
            }
            if (p->limiter & ORC_LIM_MEDIAN) {
                int sx[9], sy[9];
                int k = median_stencil(p, x, y, sx, sy);
                if (k > 0) {
                    double vals[9];
                    for (int a = 0; a < k; ++a) vals[a] = dpost[sy[a] * nx + sx[a]];
                    double med = orc_median(vals, k);
                    int hit;
                    double t;
                    if (p->median_mode == ORC_MED_GATE) {
                        hit = d > p->delta_median && d > med;
                        t = med;
                    } else {
                        t = med > p->delta_median ? med : p->delta_median;
                        hit = d > t;
                    }
                    if (hit) {
                        m[site] |= ORC_MASK_MEDIAN;
                        double pm = homothety_phi(p, q, fpn, fsn, d, t);
                        if (pm < phi) phi = pm;
                    }
                }
            }
            if (ens) {
                double pe = 1.0;
                if ((p->limiter & ORC_LIM_ENS_THRESHOLD) && d > t_thresh) {
                    const double v = homothety_phi(p, q, fpn, fsn, d, t_thresh);   /* eq. (entrHom) */
                    if (v < pe) pe = v;
                }
                if ((p->limiter & ORC_LIM_ENS_BUDGET) && d > t_budget) {
                    const double v = homothety_phi(p, q, fpn, fsn, d, t_budget);
                    if (v < pe) pe = v;
                }
                if ((p->limiter & ORC_LIM_ENS_SMOOTH) && mean_ds > 0.0 && d > 0.0) {
                    /* eq. (smooth1) with a = delta / E^k */
                    const double a = p->delta_ens / pow(mean_ds, p->ens_k);
                    const double v = isinf(d) ? 0.0 : 1.0 / (1.0 + a * pow(d, p->ens_k));
                    if (v < pe) pe = v;
                }
                if ((p->limiter & ORC_LIM_ENS_RATIONAL) && mean_ds > 0.0 && d > 0.0) {
                    /* eq. (phiExamp), r = Delta S / (alpha E); only entropic
                     * adjustments are kept (phi <= 1) */
                    double v = 0.0;
                    if (!isinf(d)) {
                        const double r = d / (p->ens_c * mean_ds);
                        v = (1.0 + pow(r, p->ens_k - 0.5)) / (1.0 + pow(r, p->ens_k));
                    }
                    if (v < pe) pe = v;
                }
                if (pe < 1.0) {
                    m[site] |= ORC_MASK_ENSEMBLE;
                    if (pe < phi) phi = pe;
                }
            }
            if (p->limiter & ORC_LIM_POSITIVITY) {
                /* positivity rule (Sec. 2.1): a post-collision state with a
                 * negative population goes to the closest non-negative state
                 * on the line through it and f*, where the first population
                 * reaches 0: phi = min f*_i / (f*_i - f'_i) over f'_i < 0 */
                double pp = 1.0;
                for (int i = 0; i < q; ++i) {
                    const double a = fpost[i * n + site], b = fst[i * n + site];
                    if (a < 0.0) {
                        const double v = b / (b - a);
                        if (v < pp) pp = v;
                    }
                }
                if (pp < 1.0) {
                    m[site] |= ORC_MASK_POSITIVITY;
                    npos[site]++;
                    if (pp < phi) phi = pp;
                }
            }
            double fs[9], fl[9];
            for (int i = 0; i < q; ++i) {       /* eq. (LimGenF) */
                fs[i] = fst[i * n + site];
                fl[i] = fs[i] + phi * (fpost[i * n + site] - fs[i]);
                o[i * n + site] = fl[i];
            }
            const double after = phi < 1.0 ? orc_delta_s(q, p->ds_form, fl, fs) : d;
            if (phi < 1.0 && isfinite(d)) {
                slim[site] = d - after;
                limon[site] = 1;
            }
            if (dS_lim) dS_lim[site] = after;
        }
    double max_ds = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int site = y * nx + x;
            s.n_positivity += npos[site];
            if (node_type(p, x, y) != NODE_FLUID) continue;
            const double d = dpost[site], dp = dpre[site];
            if (m[site] & ORC_MASK_NONPOS) s.n_nonpositive++;
            if (isfinite(dp)) s.sum_dS_pre += dp;
            if (isfinite(d)) {
                s.sum_dS_post += d;
                if (d > max_ds) max_ds = d;
            }
            if (m[site] & ORC_MASK_TRIM) s.n_trimmed++;
            if (m[site] & ORC_MASK_MEDIAN) s.n_filtered++;
            if (m[site] & ORC_MASK_ENSEMBLE) s.n_ensemble++;
            if (limon[site]) s.limiter_production += slim[site];
        }
    s.max_dS = max_ds;
    s.lbgk_production = (1.0 - c * c) * s.sum_dS_pre;
    s.mean_dS = mean_ds;
    s.ens_threshold = (p->limiter & ORC_LIM_ENS_BUDGET) ? t_budget
                      : (p->limiter & ORC_LIM_ENS_THRESHOLD) ? t_thresh : 0.0;

    /* pass 3: free flight */
    orc_stream(p, o, f);

    if (st) *st = s;
    if (mask) memcpy(mask, m, n);
    if (dS) memcpy(dS, dpost, sizeof(double) * n);
    free(fst); free(fpost); free(o); free(dpre); free(dpost); free(m);
    free(srho); free(sjx); free(sjy); free(sent); free(slim); free(npos); free(limon);
    return 0;
}
