// Device building blocks of the limited LBGK step (gfx950).
//
// Arithmetic is FP64 for FP64 storage and FP32 for the shifted FP32/FP16/BF16
// storage.  Populations are handled in shift form g_i = f_i - w_i * shift
// (shift = rho0 for reduced storage, 0 for FP64), so that the equilibrium and
// the nonequilibrium part are computed without cancellation:
//   rho = shift + sum g_i,   g*_i = w_i (sum g + rho E_i(u)),   d_i = g_i - g*_i
// where E_i = f*_i / (rho w_i) - 1 is the "equilibrium excess" of the
// quasiequilibria of Sec. 4.1.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_common.h"

namespace lbm {

// ---- lattices (Sec. 4.1) ----------------------------------------------------
// D2Q9 order: rest, E, N, W, S, NE, NW, SW, SE.  D1Q3 order: rest, v=-1, v=+1.
template <int LAT>
struct Lat;

template <>
struct Lat<kD2Q9> {
    static constexpr int Q = 9;
    __host__ __device__ static constexpr int vx(int i)
    {
        return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0;
    }
    __host__ __device__ static constexpr int vy(int i)
    {
        return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0;
    }
    __host__ __device__ static constexpr int opp(int i)
    {
        return i == 0 ? 0 : (i <= 4 ? (i + 1) % 4 + 1 : (i - 3) % 4 + 5);
    }
    // weights of the rest state (polynomial equilibrium at u = 0)
    __host__ __device__ static constexpr double w(int i)
    {
        return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    // W_i of the entropy S = -sum f ln(f/W) (same numbers for D2Q9)
    __host__ __device__ static constexpr double went(int i) { return w(i); }
};

template <>
struct Lat<kD1Q3> {
    static constexpr int Q = 3;
    __host__ __device__ static constexpr int vx(int i) { return i == 0 ? 0 : (i == 1 ? -1 : 1); }
    __host__ __device__ static constexpr int vy(int) { return 0; }
    __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : 3 - i; }
    __host__ __device__ static constexpr double w(int i) { return i == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
    // H = f1 log(f1/4) + f2 log f2 + f3 log f3
    __host__ __device__ static constexpr double went(int i) { return i == 0 ? 4.0 : 1.0; }
};

// ---- storage ---------------------------------------------------------------
// Pointers into the population buffers are read from the domain table, so
// the compiler cannot infer their address space; they are cast to global
// (address space 1) so that loads and stores use global_* instructions
// (flat ones would also count against the LDS wait counter).
#define LBM_GLOBAL __attribute__((address_space(1)))
template <class T>
using gptr = LBM_GLOBAL T*;
template <class T>
__device__ inline gptr<T> to_global(void* p) { return (gptr<T>)p; }
template <class T>
__device__ inline gptr<const T> to_global(const void* p) { return (gptr<const T>)p; }

// Value held by the lane D = -1 (left) or +1 (right) positions away in the
// same wave, by a DPP wave shift (wave_shr:1 = 0x138 moves lane i-1 to lane i,
// wave_shl:1 = 0x130 moves lane i+1 to lane i).  The lane at the end of the
// wave keeps its own value; callers replace it.  Convergent: every active lane
// must execute it.
template <int D>
__device__ __forceinline__ int lane_shift_i(int v)
{
    static_assert(D == 1 || D == -1, "neighbour lanes only");
    return __builtin_amdgcn_update_dpp(v, v, D < 0 ? 0x138 : 0x130, 0xF, 0xF, false);
}
template <int D>
__device__ __forceinline__ float lane_shift(float v)
{
    return __builtin_bit_cast(float, lane_shift_i<D>(__builtin_bit_cast(int, v)));
}
template <int D>
__device__ __forceinline__ double lane_shift(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = lane_shift_i<D>(int(b & 0xffffffffll)), hi = lane_shift_i<D>(int(b >> 32));
    return __builtin_bit_cast(double, (long long)(unsigned(lo)) | ((long long)hi << 32));
}

// Sum (MAX = false) or maximum (MAX = true) of v over the 64 lanes of a wave,
// complete in lane 63: an inclusive scan inside each row of 16 lanes by DPP
// row shifts 1, 2, 4, 8 (0x111..0x118; a lane whose source lies before its
// row takes the identity), then the totals of rows 0 and 2 carried into
// rows 1 and 3 (row_bcast:15, 0x142, row mask 0b1010) and the total of rows
// 0-1 into rows 2-3 (row_bcast:31, 0x143, row mask 0b1100).  Six VALU
// operations, each with its DPP source folded in; every lane of the wave
// must be active.
template <int CTRL, int RMASK>
__device__ __forceinline__ int dpp_id(int id, int v)
{
    return __builtin_amdgcn_update_dpp(id, v, CTRL, RMASK, 0xF, false);
}
template <bool MAX, int CTRL, int RMASK>
__device__ __forceinline__ float scan_step(float v)
{
    constexpr int id = MAX ? int(0xff800000u) : 0;        // -inf or +0
    const float o = __builtin_bit_cast(float, dpp_id<CTRL, RMASK>(id, __builtin_bit_cast(int, v)));
    return MAX ? __builtin_fmaxf(v, o) : v + o;
}
template <bool MAX, int CTRL, int RMASK>
__device__ __forceinline__ double scan_step(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    constexpr int id_hi = MAX ? int(0xfff00000u) : 0;      // -inf or +0
    const int lo = dpp_id<CTRL, RMASK>(0, int(b & 0xffffffffll)), hi = dpp_id<CTRL, RMASK>(id_hi, int(b >> 32));
    const double o = __builtin_bit_cast(double, (long long)(unsigned(lo)) | ((long long)hi << 32));
    return MAX ? fmax(v, o) : v + o;
}
template <bool MAX, class S>
__device__ __forceinline__ S wave_reduce(S v)
{
    v = scan_step<MAX, 0x111, 0xF>(v);
    v = scan_step<MAX, 0x112, 0xF>(v);
    v = scan_step<MAX, 0x114, 0xF>(v);
    v = scan_step<MAX, 0x118, 0xF>(v);
    v = scan_step<MAX, 0x142, 0xA>(v);
    v = scan_step<MAX, 0x143, 0xC>(v);
    return v;
}

// uniform base (SGPRs) + 32-bit byte offset (VGPR): lets the compiler use
// the global_load/store "saddr + voffset" form instead of 64-bit lane addresses
template <class T>
__device__ __forceinline__ gptr<const T> at_bytes(gptr<const T> base, unsigned off)
{
    return (gptr<const T>)((gptr<const char>)base + off);
}
template <class T>
__device__ __forceinline__ gptr<T> at_bytes(gptr<T> base, unsigned off)
{
    return (gptr<T>)((gptr<char>)base + off);
}

template <class T>
struct Store;

template <>
struct Store<double> {
    using A = double;
    __device__ static A ld(gptr<const double> p) { return *p; }
    __device__ static void st(gptr<double> p, A v) { *p = v; }
    __device__ static void st_stream(gptr<double> p, A v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<float> {
    using A = float;
    __device__ static A ld(gptr<const float> p) { return *p; }
    __device__ static void st(gptr<float> p, A v) { *p = v; }
    // streaming store (nontemporal hint): the state written by a step is not
    // read again within it
    __device__ static void st_stream(gptr<float> p, A v) { __builtin_nontemporal_store(v, p); }
};
// FP16 / BF16 storage uses the compiler's native _Float16 and __bf16 types
// (round to nearest even on store).
template <>
struct Store<_Float16> {
    using A = float;
    __device__ static A ld(gptr<const _Float16> p) { return float(*p); }
    __device__ static void st(gptr<_Float16> p, A v) { *p = (_Float16)v; }
    __device__ static void st_stream(gptr<_Float16> p, A v) { __builtin_nontemporal_store((_Float16)v, p); }
};
template <>
struct Store<__bf16> {
    using A = float;
    __device__ static A ld(gptr<const __bf16> p) { return float(*p); }
    __device__ static void st(gptr<__bf16> p, A v) { *p = (__bf16)v; }
    // the nontemporal store of the 16-bit pattern (the builtin takes no __bf16)
    __device__ static void st_stream(gptr<__bf16> p, A v)
    {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, (__bf16)v),
                                    reinterpret_cast<gptr<unsigned short>>(p));
    }
};

// ---- arithmetic helpers ------------------------------------------------------
// FP64: IEEE division and square root.  FP32: the hardware reciprocal and
// square root (about 1 ulp), well inside the FP32 error budget.
__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double sqrt_(double x) { return sqrt(x); }
__device__ inline double pow_(double x, double y) { return pow(x, y); }
__device__ inline float pow_(float x, float y) { return powf(x, y); }
__device__ inline float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double log1p_(double x) { return log1p(x); }
__device__ inline float log1p_(float x) { return log1pf(x); }
__device__ inline double log_(double x) { return log(x); }
__device__ inline float log_(float x) { return logf(x); }

__device__ inline float med3(float a, float b, float c) { return __builtin_amdgcn_fmed3f(a, b, c); }
__device__ inline double med3(double a, double b, double c) { return fmax(fmin(a, b), fmin(fmax(a, b), c)); }
template <class A>
__device__ inline A min3(A a, A b, A c) { return fmin(fmin(a, b), c); }
template <class A>
__device__ inline A max3(A a, A b, A c) { return fmax(fmax(a, b), c); }

// Median of a 3x3 block: sort each row (min / med / max), then the median of
// all nine is med3(max of row minima, med of row medians, min of row maxima).
template <class A>
__device__ inline A median9(A a0, A a1, A a2, A a3, A a4, A a5, A a6, A a7, A a8)
{
    A lo = max3(min3(a0, a1, a2), min3(a3, a4, a5), min3(a6, a7, a8));
    A mi = med3(med3(a0, a1, a2), med3(a3, a4, a5), med3(a6, a7, a8));
    A hi = min3(max3(a0, a1, a2), max3(a3, a4, a5), max3(a6, a7, a8));
    return med3(lo, mi, hi);
}

// h(x) = (1 + x) ln(1 + x) - x, so that sum f ln(f/f*) = sum f* h((f - f*)/f*)
// when f and f* share their moments (eq. DelS).  Near x = 0 the closed form
// cancels; there the alternating series x^2 sum_k (-x)^k / ((k+1)(k+2)) is
// summed in Horner form.  The first omitted term bounds the truncation:
// below 1e-17 relative for |x| <= 0.1 in FP64 (16 terms); in FP32 below
// 1.4e-8 for |x| <= 1/8 (7 terms, the usual case) and 1.4e-9 for
// |x| <= 0.5 (22 terms).
__device__ inline double hkern(double x)
{
    if (fabs(x) <= 0.1) {
        double p = 1.0 / (16.0 * 17.0);
#pragma unroll
        for (int k = 14; k >= 0; --k) p = 1.0 / ((k + 1.0) * (k + 2.0)) - x * p;
        return x * x * p;
    }
    return (1.0 + x) * log1p(x) - x;
}
__device__ inline float hkern(float x)
{
    if (fabsf(x) <= 0.125f) {
        float p = 1.0f / (7.0f * 8.0f);
#pragma unroll
        for (int k = 5; k >= 0; --k) p = 1.0f / ((k + 1.0f) * (k + 2.0f)) - x * p;
        return x * x * p;
    }
    if (fabsf(x) <= 0.5f) {
        float p = 1.0f / (22.0f * 23.0f);
#pragma unroll
        for (int k = 20; k >= 0; --k) p = 1.0f / ((k + 1.0f) * (k + 2.0f)) - x * p;
        return x * x * p;
    }
    return (1.0f + x) * log1pf(x) - x;
}

// h(x) with its derivative h'(x) = ln(1 + x).  Where hkern sums the series,
// the logarithm follows from h itself, (1 + x) ln(1 + x) = h(x) + x, with no
// cancellation (h is second order in x); elsewhere it is the logarithm that
// h is built from.  h(-1) = 1 with h'(-1) = -inf (a population at zero).
template <class A>
__device__ inline A hkern_slope(A x, A& dh)
{
    constexpr A series = sizeof(A) == 8 ? A(0.1) : A(0.5);
    if (x <= A(-1)) {
        dh = -A(__builtin_huge_val());
        return A(1);
    }
    if (fabs(x) <= series) {
        const A h = hkern(x);
        dh = (h + x) * rcp(A(1) + x);
        return h;
    }
    const A l = log1p_(x);
    dh = l;
    return (A(1) + x) * l - x;
}

// ---- quasiequilibria, excess form -------------------------------------------
// One axis of the entropic equilibrium: f*(v) / (rho w_v) = A B^v with
// A = 2 - s, B = (2u + s)/(1 - u), s = sqrt(1 + 3u^2) (eq. maxwellian; the
// D1Q3 equilibrium of eq. entropiceq1d is the same factor).  Returned as
// X_v = A B^v - 1 for v = 0, -1, +1 using s - 1 = 3u^2/(1 + s) and
// 1/B = (s - 2u)/(1 + u).
template <class A>
__device__ inline void axis_excess(A u, A& x0, A& xm, A& xp)
{
    A s = sqrt_(A(1) + A(3) * u * u);
    A q = A(3) * u * u * rcp(A(1) + s);   // s - 1
    A a = -q;                               // A - 1
    A bp = (A(3) * u + q) * rcp(A(1) - u);  // B - 1
    A bm = (q - A(3) * u) * rcp(A(1) + u);  // 1/B - 1
    x0 = a;
    xm = a + bm + a * bm;
    xp = a + bp + a * bp;
}

template <int LAT, int QE, class A>
__device__ __forceinline__ void eq_excess(A ux, A uy, A (&E)[Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    if constexpr (QE == kPoly) {
        // eqs. (polyeq1d), (polyeq2d): 1 + 3 c + 9 c^2 / 2 - 3 u^2 / 2, c = v.u
        A base = A(-1.5) * (ux * ux + uy * uy);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            A cu = A(L::vx(i)) * ux + A(L::vy(i)) * uy;
            E[i] = base + cu * (A(3) + A(4.5) * cu);
        }
    } else {
        A x0, xm, xp, y0 = 0, ym = 0, yp = 0;
        axis_excess(ux, x0, xm, xp);
        if constexpr (LAT == kD2Q9) axis_excess(uy, y0, ym, yp);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            A X = L::vx(i) == 0 ? x0 : (L::vx(i) > 0 ? xp : xm);
            if constexpr (LAT == kD2Q9) {
                A Y = L::vy(i) == 0 ? y0 : (L::vy(i) > 0 ? yp : ym);
                E[i] = X + Y + X * Y;
            } else {
                E[i] = X;
            }
        }
    }
}

// ---- one site: moments, f*, collision, nonequilibrium entropy ---------------
template <int LAT, class A>
struct SiteState {
    static constexpr int Q = Lat<LAT>::Q;
    A gs[Q];      // shifted equilibrium g*_i = f*_i - w_i shift
    A d[Q];       // nonequilibrium part g_i - g*_i = f_i - f*_i
    A dpost;      // Delta S(f'), +inf when undefined
    A c;          // f' - f* = -c d: 2 beta - 1 (LBGK), alpha beta - 1 (ELBM)
    bool posrule; // ELBM: no root short of the positivity boundary
};

struct SiteScalars {
    double dr, jx, jy;   // moments (FP64 for the reductions)
    double dpre;
    float ux, uy;
    bool nonpos;
};

// ---- FP32 equilibrium without a coherent drift ------------------------------
// In FP32 the moments are sums of O(0.1) shifts whose result is much smaller
// (the shift removes only the rest state), and the lattice weights 4/9, 1/9,
// 1/36 (2/3, 1/6 in 1-D) round to one mantissa with the same relative error
// e = 7.45e-9: the equilibrium's momentum then comes out as (1 + 2e) j, and
// the sums' rounding lands alike at neighbouring nodes.  Both errors repeat
// at every step of a slowly varying flow and add up (1e-5 of the velocity
// after 1e3 steps of a lid-driven cavity), where an unbiased rounding of the
// stored state alone stays near 1e-7.  So the FP32 path forms mass and
// momentum in FP64 (the nine FP32 terms and their sums and differences are
// exact there unless their magnitudes span more than 2^25; the result is
// rounded to FP32 once) and takes the momentum term with coefficients whose
// identity sum_i a_i v_i v_i = 1 holds exactly in binary: a = fl(1/3) on the
// axes and (1 - 2 fl(1/3)) / 4 (exactly representable) on the diagonals of
// D2Q9, 1/2 in D1Q3.  The entropic f* (square roots and reciprocals) is
// brought back to the node's mass and momentum afterwards along the same
// coefficients.  FP64 adds issue at the rate of unpacked FP32 ones on this
// part, so the nine conversions and sixteen adds cost less than the
// error-free FP32 transformations that give the same result.

// mass sum_i g_i and momentum sum_i v_i g_i of FP32 terms, formed in FP64 and
// rounded once.  D2Q9: sums and differences of opposite populations first
// (the diagonal difference g5 - g7 serves both components).
template <int LAT>
__device__ __forceinline__ void comp_moments(const float (&g)[Lat<LAT>::Q], float& dr, float& jx, float& jy)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    double d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = double(g[i]);
    if constexpr (LAT == kD2Q9) {
        dr = float((((d[1] + d[3]) + (d[2] + d[4])) + ((d[5] + d[7]) + (d[6] + d[8]))) + d[0]);
        const double d13 = d[1] - d[3], d24 = d[2] - d[4], d57 = d[5] - d[7], d86 = d[8] - d[6];
        jx = float((d13 + d57) + d86);
        jy = float((d24 + d57) - d86);
    } else {
        dr = float((d[1] + d[2]) + d[0]);
        jx = float(d[2] - d[1]);
        jy = 0.0f;
    }
}

// momentum coefficient a_i = 3 w_i of population i, with sum_i a_i v_i v_i = 1
// exactly in FP32
template <int LAT>
__device__ __forceinline__ float mom_coef(int i)
{
    if constexpr (LAT == kD2Q9) {
        constexpr float a1 = 0.333333343267440796f;        // fl(1/3) = 11184811 2^-25
        constexpr float a5 = 0.0833333283662796021f;       // (1 - 2 a1) / 4 = 5592405 2^-26
        return i == 0 ? 0.0f : (i <= 4 ? a1 : a5);
    } else {
        return i == 0 ? 0.0f : 0.5f;
    }
}

// Moments (eq. macro_dis) and the shifted equilibrium g*_i = f*_i - w_i shift
// of a state g in shift form.  Also used on a limited state: the limiter keeps
// rho and u, so its f* is the one it was limited toward.
template <int LAT, int QE, class A>
__device__ __forceinline__ void moments_equilibrium(const A (&g)[Lat<LAT>::Q], A shift, A& dr, A& jx, A& jy, A& rho,
                                                    A& ux, A& uy, A (&gs)[Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    constexpr bool fp32 = sizeof(A) == 4;
    if constexpr (fp32) {
        comp_moments<LAT>(g, dr, jx, jy);
    } else {
        dr = 0;
        jx = 0;
        jy = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            dr += g[i];
            if (L::vx(i) > 0) jx += g[i];
            if (L::vx(i) < 0) jx -= g[i];
            if (L::vy(i) > 0) jy += g[i];
            if (L::vy(i) < 0) jy -= g[i];
        }
    }
    rho = shift + dr;
    const A inv = rcp(rho);
    ux = jx * inv;
    uy = jy * inv;
    if constexpr (QE == kPoly && fp32) {
        // w_i (dr + rho (9 (v_i.u)^2 / 2 - 3 u^2 / 2)) + a_i v_i.j; a velocity
        // and its opposite share the even part and take the odd one with
        // opposite signs (v.u and v.j change sign exactly)
        const A base = A(-1.5) * (ux * ux + uy * uy);
        auto dot = [](int vx, int vy, A x, A y) -> A {
            const A xs = vx > 0 ? x : -x, ys = vy > 0 ? y : -y;
            return vx == 0 ? ys : (vy == 0 ? xs : xs + ys);
        };
        gs[0] = A(L::w(0)) * (dr + rho * base);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (L::opp(i) < i) continue;   // each pair once, from its first member
            const A cu = dot(L::vx(i), L::vy(i), ux, uy);
            const A cj = dot(L::vx(i), L::vy(i), jx, jy);
            const A even = A(L::w(i)) * (dr + rho * (base + A(4.5) * cu * cu));
            gs[i] = __builtin_fmaf(mom_coef<LAT>(i), cj, even);
            gs[L::opp(i)] = __builtin_fmaf(mom_coef<LAT>(i), -cj, even);
        }
        return;
    }
    A E[Q];
    if constexpr (QE == kPoly) {
        // rho E_i = 3 v_i.j + rho (9 (v_i.u)^2 / 2 - 3 u^2 / 2): the linear
        // term is taken from j itself, so the momentum of f* is j up to the
        // rounding of sums, whatever the rounding of u = j / rho
        const A base = A(-1.5) * (ux * ux + uy * uy);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const A cu = A(L::vx(i)) * ux + A(L::vy(i)) * uy;
            const A cj = A(L::vx(i)) * jx + A(L::vy(i)) * jy;
            E[i] = A(3) * cj + rho * (base + A(4.5) * cu * cu);
        }
    } else {
        eq_excess<LAT, QE>(ux, uy, E);
#pragma unroll
        for (int i = 0; i < Q; ++i) E[i] = rho * E[i];
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) gs[i] = A(L::w(i)) * (dr + E[i]);
    if constexpr (fp32) {
        // entropic f* in FP32: bring the equilibrium's mass and momentum
        // (summed without loss) back to the node's, along w_i and the exact
        // momentum coefficients
        float dre, jxe, jye;
        comp_moments<LAT>(gs, dre, jxe, jye);
        const float dd = dr - dre, dx = jx - jxe, dy = jy - jye;
        // v_i . (dx, dy) by signs (the components are 0 or +-1): the same
        // values as the products, without multiplying by them
        auto vdot = [&](int i) -> A {
            const int vx = L::vx(i), vy = L::vy(i);
            const A xs = vx > 0 ? dx : -dx, ys = vy > 0 ? dy : -dy;
            return vx == 0 ? (vy == 0 ? A(0) : ys) : (vy == 0 ? xs : xs + ys);
        };
        gs[0] += A(L::w(0)) * dd;
#pragma unroll
        for (int i = 1; i < Q; ++i) gs[i] += A(L::w(i)) * dd + mom_coef<LAT>(i) * vdot(i);
    }
}

// h with its limit h(-1) = 1 (a population at exactly zero)
template <class A>
__device__ __forceinline__ A h_closed(A y)
{
    return y <= A(-1) ? A(1) : hkern(y);
}

// ELBM (eqs. elbm, entropy_estimate): alpha, the nontrivial root of
// S(f~) = S(f) for f~ = (1 - alpha) f + alpha f*.  With the entropic f*,
// S(f*) - S(g) = sum f*_i h(x_i(g)) on the line through f and f*, and f~ has
// the deviation (1 - alpha) x, so in s = alpha - 1 the equation is
// G(s) = sum f*_i h(-s x_i) - sum f*_i h(x_i) = 0 with G convex and
// increasing on [0, s_max], s_max the positivity boundary of f~, and
// G(0) < 0.  Newton from the LBGK mirror s = 1 corrected by the cubic term
// of h (h(y) = y^2/2 - y^3/6 + O(y^4) puts the root at
// s = 1 - sum f*_i x_i^3 / (3 sum f*_i x_i^2) + O(x^2)), kept inside the bracket
// (bisection when a step leaves it), until G is at the rounding level of its
// sums; the result is moved down to a point with G <= 0, so the entropy does
// not decrease.  A root short of s_max exists iff G(s_max) >= 0; that is
// evaluated only when no iterate has found G > 0 by the time a step leaves
// the bracket (on a convex G, a Newton step from a point with G < 0 lands at
// or beyond the root).  No root (or a state f without entropy): the
// positivity rule, s = s_max.
template <int Q, class A>
__device__ A elbm_alpha(const A (&fs)[Q], const A (&x)[Q], bool& posrule)
{
    constexpr A eps = sizeof(A) == 8 ? A(2.220446049250313e-16) : A(1.1920929e-7);
    const A inf = A(__builtin_huge_val());
    A smax = inf, target = A(0), m2 = A(0), m3 = A(0);
    bool nonpos = false;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (x[i] > A(0)) smax = fmin(smax, A(1) / x[i]);
        nonpos |= x[i] <= A(-1);
        target += fs[i] * h_closed(x[i]);
        const A fx2 = fs[i] * x[i] * x[i];
        m2 += fx2;
        m3 += fx2 * x[i];
    }
    posrule = false;
    if (!(smax < inf)) return A(2);        // f = f*: every alpha gives f
    if (nonpos) {
        posrule = true;
        return A(1) + smax;
    }
    // G(s) and G'(s) = -sum f*_i x_i ln(1 - s x_i)
    auto eval = [&](A s, A& dg) {
        A g = -target;
        dg = A(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            A dh;
            g += fs[i] * hkern_slope(-s * x[i], dh);
            dg -= fs[i] * x[i] * dh;
        }
        return g;
    };
    A s = A(1);
    if (m2 > A(0)) {
        const A c = m3 / (A(3) * m2);
        if (fabs(c) < A(0.5)) s -= c;
    }
    A lo = A(0), hi = smax;
    s = fmin(s, A(0.5) * smax);
    A g = A(0), dg;
    bool at_s = false;      // g = G(s)
    bool above = false;     // some G > 0 seen, or G(s_max) >= 0: a root lies in [lo, hi]
    bool settled = false;   // converged (residual or step at the rounding level)
    for (int it = 0; it < 60; ++it) {
        g = eval(s, dg);
        at_s = true;
        // at the rounding level of the sums: the root is as good as it gets
        if (fabs(g) <= A(4) * eps * target) {
            settled = true;
            break;
        }
        if (g <= A(0)) {
            lo = s;
        } else {
            hi = s;
            above = true;
        }
        A sn = s - g / dg;
        if (!(sn > lo && sn < hi)) {
            if (!above) {
                A d;
                if (eval(smax, d) < A(0)) {
                    posrule = true;
                    return A(1) + smax;
                }
                above = true;
            }
            sn = A(0.5) * (lo + hi);
        }
        const bool done = fabs(sn - s) <= A(2) * eps * s;
        s = sn;
        at_s = false;
        if (done) {
            settled = true;
            break;
        }
    }
    A d;
    if (!settled && !above && eval(smax, d) < A(0)) {
        posrule = true;
        return A(1) + smax;
    }
    A gs = at_s ? g : eval(s, d);
    for (int k = 0; k < 4 && gs > A(0); ++k) {
        s *= A(1) - A(2) * eps;
        gs = eval(s, d);
    }
    if (gs > A(0)) s = lo;
    return A(1) + s;
}

template <int LAT, int QE, int DS, bool ELBM = false, class A>
__device__ __forceinline__ void collide_site(const A (&g)[Lat<LAT>::Q], A shift, A c, SiteState<LAT, A>& o,
                                    SiteScalars& sc, bool want_pre)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    A dr, jx, jy, rho, ux, uy;
    moments_equilibrium<LAT, QE>(g, shift, dr, jx, jy, rho, ux, uy, o.gs);
    A fs[Q];
    bool fs_ok = true, pre_ok = true, post_ok = true;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        fs[i] = A(L::w(i)) * shift + o.gs[i];
        o.d[i] = g[i] - o.gs[i];
        fs_ok &= fs[i] > A(0);
        pre_ok &= (g[i] + A(L::w(i)) * shift) > A(0);
    }
    o.posrule = false;
    if constexpr (ELBM) {
        // eq. (elbmLB): f' = f + alpha beta (f* - f) = f* - (alpha beta - 1) d,
        // beta = (c + 1) / 2
        A xe[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) xe[i] = o.d[i] / fs[i];
        const A alpha = elbm_alpha<Q>(fs, xe, o.posrule);
        c = alpha * (A(0.5) * (c + A(1))) - A(1);
    }
    o.c = c;
#pragma unroll
    for (int i = 0; i < Q; ++i) post_ok &= (fs[i] - c * o.d[i]) > A(0);
    A dpre = 0, dpost = 0;
    if constexpr (DS == kQuad) {
        // sum (f - f*)^2 / (2 f*); after collision f' - f* = -c d (eq. collLBGK)
#pragma unroll
        for (int i = 0; i < Q; ++i) dpre += o.d[i] * o.d[i] * rcp(fs[i]);
        dpre *= A(0.5);
        dpost = c * c * dpre;
        pre_ok = post_ok = true;
    } else {
        A x[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) x[i] = o.d[i] * rcp(fs[i]);
        if (want_pre) {
#pragma unroll
            for (int i = 0; i < Q; ++i) dpre += fs[i] * hkern(x[i]);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) dpost += fs[i] * hkern(-c * x[i]);
    }
    const A inf = A(__builtin_huge_val());
    if (!fs_ok) pre_ok = post_ok = false;
    o.dpost = post_ok ? dpost : inf;
    sc.dpre = pre_ok ? double(dpre) : double(inf);
    sc.nonpos = !(pre_ok && post_ok);
    // non-finite moments or velocity (e.g. rho = 0) propagate as NaN
    if (!(isfinite(rho) && isfinite(ux) && isfinite(uy))) {
        o.dpost = A(__builtin_nan(""));
        sc.dpre = __builtin_nan("");
        sc.nonpos = false;
    }
    sc.dr = double(dr);
    sc.jx = double(jx);
    sc.jy = double(jy);
    sc.ux = float(ux);
    sc.uy = float(uy);
}

// positivity rule (Sec. 2.1): the largest phi with f* + phi (f' - f*) >= 0,
// min f*_i / (f*_i - f'_i) over the populations with f'_i < 0; 1 when none
template <int LAT, class A>
__device__ __forceinline__ A positivity_phi(const SiteState<LAT, A>& o, A shift)
{
    using L = Lat<LAT>;
    A pp = A(1);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const A fs = A(L::w(i)) * shift + o.gs[i];
        const A fp = fs - o.c * o.d[i];
        if (fp < A(0)) pp = fmin(pp, fs / (fs - fp));
    }
    return pp;
}

// Delta S of f* + s (f' - f*) = f* - s c d, used for the limiter's entropy
// production (eq. LimEntLim).
template <int LAT, int DS, class A>
__device__ __forceinline__ A delta_s_scaled(const SiteState<LAT, A>& o, A shift, A c, A s)
{
    using L = Lat<LAT>;
    if constexpr (DS == kQuad) {
        return s * s * o.dpost;
    } else {
        A sum = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            A fs = A(L::w(i)) * shift + o.gs[i];
            sum += fs * hkern(-s * c * o.d[i] * rcp(fs));
        }
        return sum;
    }
}

// S(f) = -sum f ln(f/W) (Sec. 4.3.1), NaN when a population is not positive
template <int LAT, class A>
__device__ inline double entropy_site(const A (&g)[Lat<LAT>::Q], A shift)
{
    using L = Lat<LAT>;
    A s = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        A f = g[i] + A(L::w(i)) * shift;
        if (!(f > A(0))) return __builtin_nan("");
        s -= f * log_(f * A(1.0 / L::went(i)));
    }
    return double(s);
}

// ---- limiter -----------------------------------------------------------------
// phi for one fluid site (eq. LimGenF): trimming (eq. entrHom / Ehrenfests'
// step) and the median filter (Sec. 3.5); both on -> the smaller phi.
template <class A>
__device__ __forceinline__ A limiter_phi(A dpost, bool has_med, A med, const DomainDev& D, unsigned& mask, A& tgt)
{
    A phi = A(1);
    tgt = A(__builtin_huge_val());
    if (D.limiter & kLimTrim) {
        A t = A(D.delta_trim);
        if (dpost > t) {
            mask |= kMaskTrim;
            A p = D.trim_mode ? A(0) : sqrt_(t * rcp(dpost));
            phi = fmin(phi, p);
            if (!D.trim_mode) tgt = fmin(tgt, t);
        }
    }
    if ((D.limiter & kLimMedian) && has_med) {
        A dm = A(D.delta_median);
        bool hit;
        A t;
        if (D.median_mode) {
            hit = dpost > dm && dpost > med;
            t = med;
        } else {
            t = fmax(med, dm);
            hit = dpost > t;
        }
        if (hit) {
            mask |= kMaskMedian;
            phi = fmin(phi, sqrt_(t * rcp(dpost)));
            tgt = fmin(tgt, t);
        }
    }
    return phi;
}

// ---- statistics ----------------------------------------------------------------
// Per-thread running sums over the (at most 64) nodes a thread visits, kept
// in type S: FP64 in FP64 mode, FP32 in the reduced-storage modes (a
// 64-term FP32 sum of FP32 site values loses nothing that matters); the
// workgroup, tile, domain and global reductions are FP64.  The second D2Q9
// pass keeps the limiter's entropy production in FP64 (type SL): a thread
// there sums over a tile's column, whose height is a launch choice, and in
// FP64 that choice changes the sum only at FP64 rounding.
template <class S, class SL = S>
struct AccT {
    S mass = 0, jx = 0, jy = 0, dpre = 0, dpost = 0, ent = 0, maxd = 0;
    SL lim = 0;
    int trim = 0, filt = 0, nonpos = 0, nonfin = 0, fluid = 0, above = 0, ens = 0, pos = 0;

    __device__ void moments(const SiteScalars& s)
    {
        mass += S(s.dr);
        jx += S(s.jx);
        jy += S(s.jy);
        if (!(isfinite(s.dr) && isfinite(s.jx) && isfinite(s.jy))) ++nonfin;
    }
    template <class A>
    __device__ void fluid_site(const SiteScalars& s, A site_dpost)
    {
        ++fluid;
        if (s.nonpos) ++nonpos;
        if (isfinite(s.dpre)) dpre += S(s.dpre);
        const S dp = S(site_dpost);
        if (isfinite(dp)) {
            dpost += dp;
            maxd = fmax(maxd, dp);
        }
    }
};
using Acc = AccT<double>;

// Deterministic workgroup reduction of the accumulators into one partial
// (fixed butterfly inside each wave, then waves in order).
template <class S, class SL>
__device__ inline void store_partial(const AccT<S, SL>& acc, double* out, double* lds /* [4 * kNStat] */)
{
    double v[kNStat] = {double(acc.mass), double(acc.jx), double(acc.jy), double(acc.dpre), double(acc.dpost),
                        double(acc.maxd), double(acc.lim), double(acc.ent), double(acc.trim), double(acc.filt),
                        double(acc.nonpos), double(acc.nonfin), double(acc.fluid), double(acc.above),
                        double(acc.ens), double(acc.pos)};
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < kNStat; ++k) {
            double o = __shfl_xor(v[k], off, 64);
            v[k] = (k == kSMax) ? fmax(v[k], o) : v[k] + o;
        }
    }
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kNStat; ++k) lds[wave * kNStat + k] = v[k];
    }
    __syncthreads();
    if (tid < kNStat) {
        const int nw = (blockDim.x * blockDim.y) >> 6;
        double s = lds[tid];
        for (int w = 1; w < nw; ++w) s = (tid == kSMax) ? fmax(s, lds[w * kNStat + tid]) : s + lds[w * kNStat + tid];
        out[tid] = s;
    }
}

// The same, plus the rn <= kMaxTileH partials rp[0], rp[rstride kNStat], ...
// written by an earlier kernel: they are fetched by the whole workgroup at
// once, summed in fixed segments of eight, and the segments added after the
// waves in order.  rowbuf holds kMaxTileH * kNStat + 8 * kNStat doubles.
template <class S>
__device__ inline void store_partial_rows(const AccT<S>& acc, double* out, double* lds, const double* rp, int rn,
                                          long long rstride, double* rowbuf)
{
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nthr = blockDim.x * blockDim.y;
    for (int e = tid; e < rn * kNStat; e += nthr) {
        const int j = e / kNStat, k = e - j * kNStat;
        rowbuf[e] = rp[j * rstride * kNStat + k];
    }
    double v[kNStat] = {double(acc.mass), double(acc.jx), double(acc.jy), double(acc.dpre), double(acc.dpost),
                        double(acc.maxd), double(acc.lim), double(acc.ent), double(acc.trim), double(acc.filt),
                        double(acc.nonpos), double(acc.nonfin), double(acc.fluid), double(acc.above),
                        double(acc.ens), double(acc.pos)};
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < kNStat; ++k) {
            double o = __shfl_xor(v[k], off, 64);
            v[k] = (k == kSMax) ? fmax(v[k], o) : v[k] + o;
        }
    }
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kNStat; ++k) lds[wave * kNStat + k] = v[k];
    }
    __syncthreads();
    double* seg = rowbuf + kMaxTileH * kNStat;     // [kNStat][8]
    if (tid < 8 * kNStat) {
        const int k = tid >> 3, g = tid & 7;
        double s = k == kSMax ? -__builtin_huge_val() : 0.0;
        for (int j = 8 * g; j < rn && j < 8 * g + 8; ++j) {
            const double r = rowbuf[j * kNStat + k];
            s = (k == kSMax) ? fmax(s, r) : s + r;
        }
        seg[tid] = s;
    }
    __syncthreads();
    if (tid < kNStat) {
        const int nw = nthr >> 6;
        double s = lds[tid];
        for (int w = 1; w < nw; ++w) s = (tid == kSMax) ? fmax(s, lds[w * kNStat + tid]) : s + lds[w * kNStat + tid];
#pragma unroll
        for (int g = 0; g < 8; ++g) s = (tid == kSMax) ? fmax(s, seg[tid * 8 + g]) : s + seg[tid * 8 + g];
        out[tid] = s;
    }
}

// Partials of a workgroup whose threads hold at most one node each, covering
// `nrow` rows of `wpr` waves each (a row of 64 wpr columns): the sums (FP32
// for reduced storage, FP64 for FP64 storage) by a fixed DPP scan in each
// wave (the limiter and entropy sums only in waves that hold one), the 0/1
// counts by ballots; then for each row its waves combined in FP64 in order,
// written to out + r * stride (r < nrow).  kSAbove is a bit mask there: bit
// w is set when wave w of the row holds a node above the median tolerance
// (the median pass reads which waves stored Delta S').
template <class S>
__device__ inline void node_partial_rows(const AccT<S>& acc, double* out, long long stride, int wpr, int nrow,
                                         double* lds /* [4 * kNStat] */)
{
    S v[8] = {acc.mass, acc.jx, acc.jy, acc.dpre, acc.dpost, acc.maxd, acc.lim, acc.ent};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k == kSLim || k == kSEnt) {
            if (!__ballot(v[k] != S(0))) continue;     // uniform: the wave holds none
        }
        v[k] = k == kSMax ? wave_reduce<true>(v[k]) : wave_reduce<false>(v[k]);
    }
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    // counts of a wave fit 32 bits; wpr is a power of two
    auto count = [](bool b) { return double(unsigned(__popcll(__ballot(b)))); };
    const double cnt[8] = {count(acc.trim != 0), count(acc.filt != 0), count(acc.nonpos != 0),
                           count(acc.nonfin != 0), count(acc.fluid != 0),
                           __ballot(acc.above != 0) ? double(1u << (unsigned(wave) & unsigned(wpr - 1))) : 0.0,
                           count(acc.ens != 0), count(acc.pos != 0)};
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < 8; ++k) lds[wave * kNStat + k] = double(v[k]);
#pragma unroll
        for (int k = 0; k < 8; ++k) lds[wave * kNStat + 8 + k] = cnt[k];
    }
    __syncthreads();
    if (tid < nrow * kNStat) {
        const int r = tid / kNStat, k = tid - r * kNStat;
        const double* row = lds + r * wpr * kNStat;
        double s = row[k];
        for (int w = 1; w < wpr; ++w) s = (k == kSMax) ? fmax(s, row[w * kNStat + k]) : s + row[w * kNStat + k];
        out[r * stride * kNStat + k] = s;
    }
}

// Second-pass limiter terms of a node with Delta S' = d, from this step's
// E(Delta S') and thresholds (ens[kNEns]): `tgt`, the smallest homothety
// target Delta S_t among the limiters that act (threshold and budget: eq.
// entrHom above Delta S_t; top-k trimming in homothety mode: delta), and
// `fac`, the smallest factor given as phi itself (smooth: eq. (smooth1) with
// a = delta / E^k; rational: eq. (phiExamp) with r = d / (alpha E), kept <= 1;
// top-k Ehrenfests' step: 0).  The node's factor is min(fac, phi(tgt)), with
// phi(tgt) = sqrt(tgt / d) in the quadratic reading of the homothety.
// +inf (a non-positive population) gives 0; NaN moves nothing.
struct SecondHit {
    unsigned bits = 0;
    int ens = 0, trim = 0;
};
template <class A>
__device__ __forceinline__ void ens_terms(const DomainDev& D, const double* ens, A d, A& tgt, A& fac, SecondHit& h)
{
    const int lim = D.limiter;
    bool e = false;
    if ((lim & kLimEnsThresh) && d > A(ens[kEThresh])) {
        tgt = fmin(tgt, A(ens[kEThresh]));
        e = true;
    }
    if ((lim & kLimEnsBudget) && d > A(ens[kEBudget])) {
        tgt = fmin(tgt, A(ens[kEBudget]));
        e = true;
    }
    const double mean = ens[kEMean];
    if ((lim & kLimEnsSmooth) && mean > 0.0 && d > A(0)) {
        const A v = isinf(d) ? A(0) : A(1) / (A(1) + A(ens[kESmoothA]) * pow_(d, A(D.ens_k)));
        if (v < A(1)) {
            fac = fmin(fac, v);
            e = true;
        }
    }
    if ((lim & kLimEnsRational) && mean > 0.0 && d > A(0)) {
        A v = A(0);
        if (!isinf(d)) {
            const A r = d / A(D.ens_c * mean);
            v = (A(1) + pow_(r, A(D.ens_k - 0.5))) / (A(1) + pow_(r, A(D.ens_k)));
        }
        if (v < A(1)) {
            fac = fmin(fac, v);
            e = true;
        }
    }
    if (e) {
        h.bits |= kMaskEns;
        ++h.ens;
    }
    if ((lim & kLimTopK) && d > A(D.delta_trim) && (isinf(d) || d >= A(ens[kETopk]))) {
        h.bits |= kMaskTrim;
        ++h.trim;
        if (D.trim_mode) fac = A(0);
        else tgt = fmin(tgt, A(D.delta_trim));
    }
}

// Root p >= 0 of F(p) = sum f*_i h(p x_i) = t (the Kullback Delta S of the
// state whose deviation from f* is p x), F convex and increasing: Newton
// from p0 inside [lo, hi] (bisection when a step leaves the bracket), then
// moved down to F(p) <= t.  Used for the homothety to Delta S_t with the
// exact Delta S (Sec. 3.6: phi with S(f* + phi (f - f*)) = S(f*) - Delta S_t).
template <int Q, class A>
__device__ A kullback_scale(const A (&fs)[Q], const A (&x)[Q], A t, A p0, A lo, A hi)
{
    constexpr A eps = sizeof(A) == 8 ? A(2.220446049250313e-16) : A(1.1920929e-7);
    // F(p) - t and F'(p) = sum f*_i x_i ln(1 + p x_i)
    auto eval = [&](A p, A& df) {
        A f = -t;
        df = A(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            A dh;
            f += fs[i] * hkern_slope(p * x[i], dh);
            df += fs[i] * x[i] * dh;
        }
        return f;
    };
    A p = fmin(fmax(p0, lo), hi);
    A f = A(0), df;
    bool at_p = false;      // f = F(p) - t
    for (int it = 0; it < 60; ++it) {
        f = eval(p, df);
        at_p = true;
        if (fabs(f) <= A(4) * eps * t) break;
        if (f <= A(0)) lo = p;
        else hi = p;
        A pn = p - f / df;
        if (!(pn > lo && pn < hi)) pn = A(0.5) * (lo + hi);
        const bool done = fabs(pn - p) <= A(2) * eps * p;
        p = pn;
        at_p = false;
        if (done) break;
    }
    A d;
    A fp = at_p ? f : eval(p, d);
    for (int k = 0; k < 4 && fp > A(0); ++k) {
        p *= A(1) - A(2) * eps;
        fp = eval(p, d);
    }
    if (fp > A(0)) p = lo;
    return p;
}

// exact homothety of a post-collision state (f' - f* = -c d) to Delta S = t
template <int LAT, class A>
__device__ __forceinline__ A exact_homothety(const SiteState<LAT, A>& o, A shift, A t, A dpost)
{
    using L = Lat<LAT>;
    A fs[L::Q], x[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        fs[i] = A(L::w(i)) * shift + o.gs[i];
        x[i] = -o.c * o.d[i] / fs[i];
    }
    return kullback_scale<L::Q>(fs, x, t, sqrt_(t * rcp(dpost)), A(0), A(1));
}

constexpr int kSmallDomainTiles = 32;

__device__ inline void reduce_partials(const StepArgs& a, int parity, long long step, double* lds)
{
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nthr = blockDim.x * blockDim.y;
    // set 0: collision partials per group (D2Q9: summed from the rows on
    // demand); set 1: the second pass per tile, when it ran
    const double* part = a.partials + (long long)parity * 2 * a.pstride * kNStat;
    // the fused step writes set 1 only
    const int set0 = a.fused ? 1 : 0, nsets = (a.median_pass || a.fused) ? 2 : 1;
    // domains with few slots: one thread each, slots summed in order
    for (int d = tid; d < a.ndomains; d += nthr) {
        const DomainDev& D = a.dom[d];
        // the rule depends on the groups only, so that set 0 is summed in the
        // same order whatever the tile height (set 1 adds zeros to its slots)
        if (D.group_count > kSmallDomainTiles) continue;
        double v[kNStat];
#pragma unroll
        for (int k = 0; k < kNStat; ++k) v[k] = 0;
        for (int set = set0; set < nsets; ++set) {
            const int first = set ? D.tile_first : D.group_first, count = set ? D.tile_count : D.group_count;
            for (int t = 0; t < count; ++t) {
                const double* p = part + ((long long)set * a.pstride + first + t) * kNStat;
#pragma unroll
                for (int k = 0; k < kNStat; ++k) v[k] = (k == kSMax) ? fmax(v[k], p[k]) : v[k] + p[k];
            }
        }
#pragma unroll
        for (int k = 0; k < kNStat; ++k) D.stats[k] = v[k];
        D.stats[kNStat] = double(step);
    }
    // large domains: the whole workgroup, fixed slices then a fixed tree
    for (int d = 0; d < a.ndomains; ++d) {
        const DomainDev& D = a.dom[d];
        if (D.group_count <= kSmallDomainTiles) continue;
        double v[kNStat];
#pragma unroll
        for (int k = 0; k < kNStat; ++k) v[k] = 0;
        for (int set = set0; set < nsets; ++set) {
            const int first = set ? D.tile_first : D.group_first, count = set ? D.tile_count : D.group_count;
            for (int t = tid; t < count; t += nthr) {
                const double* p = part + ((long long)set * a.pstride + first + t) * kNStat;
#pragma unroll
                for (int k = 0; k < kNStat; ++k) v[k] = (k == kSMax) ? fmax(v[k], p[k]) : v[k] + p[k];
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int k = 0; k < kNStat; ++k) {
                double o = __shfl_xor(v[k], off, 64);
                v[k] = (k == kSMax) ? fmax(v[k], o) : v[k] + o;
            }
        }
        const int wave = tid >> 6, lane = tid & 63;
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < kNStat; ++k) lds[wave * kNStat + k] = v[k];
        }
        __syncthreads();
        if (tid < kNStat) {
            const int nw = nthr >> 6;
            double s = lds[tid];
            for (int w = 1; w < nw; ++w) s = (tid == kSMax) ? fmax(s, lds[w * kNStat + tid]) : s + lds[w * kNStat + tid];
            D.stats[tid] = s;
        }
        if (tid == 0) D.stats[kNStat] = double(step);
        __syncthreads();
    }
}

__host__ __device__ inline int wrapi(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

}  // namespace lbm
