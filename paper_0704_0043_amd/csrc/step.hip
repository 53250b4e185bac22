// Fused limited LBGK step kernels for gfx950.
//
// Compiled once per population storage type (LBM_ST = 0..3).  One launch is
// one time step of every domain in the tile table: free flight (pull form,
// read from buffer `parity`), moments, f*, over-relaxation, Delta S(f'),
// trimming and/or the median filter, and the store of the limited
// post-collision state into the other buffer.  The last workgroup of the grid
// reduces the previous step's per-tile FP64 partials into the domain stats.
//
// Memory layout: SoA planes buf[i * plane + y * nx + x].  Each D2Q9 workgroup
// owns a strip of TX columns and rows [y0, y1) and walks down it with TY rows
// per iteration ("sliding window"): Delta S' of the current row block goes
// into an LDS ring of four row blocks, so the 3x3 median of a row needs no
// recomputation of its neighbours; the two halo columns of the strip are
// computed once per tile before the walk.  Loads of the next row block are
// issued before the current block is processed.
#include "lbm_device.h"

#ifndef LBM_ST
#define LBM_ST 1
#endif
#if LBM_ST == 0
using StT = double;
#define LBM_SUFFIX st0
#elif LBM_ST == 1
using StT = float;
#define LBM_SUFFIX st1
#elif LBM_ST == 2
using StT = _Float16;
#define LBM_SUFFIX st2
#else
using StT = __bf16;
#define LBM_SUFFIX st3
#endif
#define LBM_CAT2(a, b) a##_##b
#define LBM_CAT(a, b) LBM_CAT2(a, b)

namespace lbm {

// Pull free flight: the population i arriving at (x, y) left (x - vx, y - vy)
// one step earlier.  Off a non-periodic edge the value is the node's own
// opposite population (reflection), which makes free flight a permutation.
template <int LAT, int BC, class T>
__device__ inline void gather(gptr<const T> src, long long plane, int nx, int ny, int x, int y,
                              typename Store<T>::A (&g)[Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    if constexpr (BC == kPeriodic) {
        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        unsigned r0 = unsigned(y) * unsigned(nx), rm = r0, rp = r0;
        if constexpr (LAT == kD2Q9) {
            rm = unsigned(y == 0 ? ny - 1 : y - 1) * unsigned(nx);
            rp = unsigned(y == ny - 1 ? 0 : y + 1) * unsigned(nx);
        }
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int xs = L::vx(i) > 0 ? xm : (L::vx(i) < 0 ? xp : x);
            const unsigned rs = L::vy(i) > 0 ? rm : (L::vy(i) < 0 ? rp : r0);
            g[i] = Store<T>::ld(src + i * plane + (rs + unsigned(xs)));
        }
    } else {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int xs = x - L::vx(i), ys = y - L::vy(i);
            const bool in = xs >= 0 && xs < nx && ys >= 0 && ys < ny;
            const long long off = in ? (i * plane + (unsigned(ys) * unsigned(nx) + unsigned(xs)))
                                     : (L::opp(i) * plane + (unsigned(y) * unsigned(nx) + unsigned(x)));
            g[i] = Store<T>::ld(src + off);
        }
    }
}

// node classes of the cavity (Sec. 4.4.1): walls x = 0, x = nx-1, y = 0
// (corners included), lid y = ny-1, fluid elsewhere
enum { kNodeFluid = 0, kNodeWall = 1, kNodeLid = 2, kNodeNone = 3 };

template <int BC>
__device__ inline int node_class(int x, int y, int nx, int ny)
{
    if constexpr (BC != kCavity) {
        return kNodeFluid;
    } else {
        if (x == 0 || x == nx - 1 || y == 0) return kNodeWall;
        if (y == ny - 1) return kNodeLid;
        return kNodeFluid;
    }
}

// reduction workgroup: previous step's partials -> stats, advance the counter
__device__ inline void reduce_block(const StepArgs& a, double* red)
{
    const long long step = a.counter[a.parity];
    if (step > 0) reduce_partials(a, 1 - a.parity, step, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) a.counter[1 - a.parity] = step + 1;
}

template <class T, int QE, int DS, int BC>
__global__ void __launch_bounds__(kThreads) k_step2d(StepArgs a)
{
    using A = typename Store<T>::A;
    constexpr int LAT = kD2Q9;
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    __shared__ A ring[4 * (kThreads + 8)];
    __shared__ A halo[2 * (kMaxTileH + 2)];
    __shared__ double red[4 * kNStat];

    if (int(blockIdx.x) == a.ntiles) {
        reduce_block(a, red);
        return;
    }
    const Tile t = a.tiles[blockIdx.x];
    const DomainDev& D = a.dom[t.domain];
    const int TX = blockDim.x, TY = blockDim.y;
    const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * TX + lx;
    const int nx = D.nx, ny = D.ny;
    const int x0 = t.x0, y0 = t.y0, y1 = t.y1;
    const int ncols = min(TX, nx - x0);
    const int hrows = y1 - y0 + 2;
    const long long plane = D.plane;
    const gptr<const T> src = to_global<T>(static_cast<const void*>(D.buf[a.parity]));
    const gptr<T> dst = to_global<T>(D.buf[1 - a.parity]);
    const A shift = A(D.shift), c = A(D.c);
    const bool record = a.flags & kFlagRecord;
    const bool want_ent = a.flags & kFlagEntropy;
    const long long step = a.counter[a.parity];

    // halo columns x0 - 1 and x0 + ncols for rows y0 - 1 .. y1: Delta S' only
    for (int s = tid; s < 2 * hrows; s += kThreads) {
        const int side = s >= hrows;
        int hx = side ? x0 + ncols : x0 - 1;
        int hy = y0 - 1 + (s - side * hrows);
        A val = A(0);
        bool fluid;
        if constexpr (BC == kPeriodic) {
            hx = wrapi(hx, nx);
            hy = wrapi(hy, ny);
            fluid = true;
        } else {
            fluid = hx >= 1 && hx <= nx - 2 && hy >= 1 && hy <= ny - 2;
        }
        if (fluid) {
            A g[Q];
            gather<LAT, BC>(src, plane, nx, ny, hx, hy, g);
            SiteState<LAT, A> st;
            SiteScalars sc;
            collide_site<LAT, QE, DS>(g, shift, c, st, sc, false);
            val = st.dpost;
        }
        halo[s] = val;
    }
    __syncthreads();

    Acc acc;
    const int x = x0 + lx;
    const bool colok = lx < ncols;
    const int nb = (hrows + TY - 1) / TY;
    const int ringw = TX + 2;
    const int ringrows = 4 * TY;

    auto row_of = [&](int rel) { return y0 - 1 + rel; };
    auto row_ok = [&](int rel) {
        const int r = row_of(rel);
        if (rel >= hrows) return false;
        if constexpr (BC == kPeriodic) return true;
        return r >= 0 && r < ny;
    };
    auto wrap_row = [&](int r) {
        if constexpr (BC == kPeriodic) return wrapi(r, ny);
        return r;
    };

    A gcur[Q], gnext[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) gcur[i] = gnext[i] = A(0);
    if (colok && row_ok(ly)) gather<LAT, BC>(src, plane, nx, ny, x, wrap_row(row_of(ly)), gcur);

    SiteState<LAT, A> P, N;
    int clsP = kNodeNone, clsN = kNodeNone;
    bool nonposP = false, nonposN = false;

    for (int b = 0; b <= nb; ++b) {
        const int rel = b * TY + ly;
        if (b < nb) {
            if (b + 1 < nb && colok && row_ok(rel + TY))
                gather<LAT, BC>(src, plane, nx, ny, x, wrap_row(row_of(rel + TY)), gnext);
            const int cr = row_of(rel);
            const int yy = wrap_row(cr);
            clsN = (colok && row_ok(rel)) ? node_class<BC>(x, yy, nx, ny) : kNodeNone;
            const bool owned = clsN != kNodeNone && cr >= y0 && cr < y1;
            A dsv = A(0);
            nonposN = false;
            if (clsN == kNodeFluid) {
                SiteScalars sc;
                collide_site<LAT, QE, DS>(gcur, shift, c, N, sc, owned);
                dsv = N.dpost;
                nonposN = sc.nonpos;
                if (owned) {
                    acc.moments(sc);
                    acc.fluid_site(sc, N.dpost);
                    if (want_ent) {
                        const double e = entropy_site<LAT>(gcur, shift);
                        if (isfinite(e)) acc.ent += e;
                    }
                    if (x == D.probe_x && yy == D.probe_y) {
                        const gptr<float> p = to_global<float>(D.probe) + 2 * (step % D.probe_cap);
                        p[0] = sc.ux;
                        p[1] = sc.uy;
                    }
                }
            } else if (clsN != kNodeNone) {
                // wall or lid node: keep the arriving populations for the output phase
#pragma unroll
                for (int i = 0; i < Q; ++i) N.gs[i] = gcur[i];
                if (owned) {
                    SiteScalars sc;
                    double dr = 0, jx = 0, jy = 0;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        dr += double(gcur[i]);
                        jx += L::vx(i) * double(gcur[i]);
                        jy += L::vy(i) * double(gcur[i]);
                    }
                    sc.dr = dr;
                    sc.jx = jx;
                    sc.jy = jy;
                    acc.moments(sc);
                }
            }
            const int slot = rel % ringrows;
            ring[slot * ringw + 1 + lx] = dsv;
            if (lx == 0 && rel < hrows) {
                ring[slot * ringw] = halo[rel];
                ring[slot * ringw + ncols + 1] = halo[hrows + rel];
            }
        }
        __syncthreads();
        if (b >= 1) {
            const int relo = rel - TY;
            const int orow = row_of(relo);
            if (colok && orow >= y0 && orow < y1 && clsP != kNodeNone) {
                const unsigned obase = unsigned(orow) * unsigned(nx) + unsigned(x);
                unsigned mask = 0;
                A dsrec = A(0);
                if (clsP == kNodeFluid) {
                    A med = A(0);
                    bool has_med = false;
                    if (D.limiter & kLimMedian) {
                        const A* rb = ring + ((relo + ringrows - 1) % ringrows) * ringw + lx;
                        const A* rc = ring + (relo % ringrows) * ringw + lx;
                        const A* ra = ring + ((relo + 1) % ringrows) * ringw + lx;
                        const A v00 = rb[0], v01 = rb[1], v02 = rb[2];
                        const A v10 = rc[0], v11 = rc[1], v12 = rc[2];
                        const A v20 = ra[0], v21 = ra[1], v22 = ra[2];
                        has_med = true;
                        if constexpr (BC == kPeriodic) {
                            med = median9(v00, v01, v02, v10, v11, v12, v20, v21, v22);
                        } else {
                            // Sec. 4.4 stencils: three nodes along a neighbouring wall,
                            // two inner axis neighbours next to a corner
                            const bool nl = x == 1, nr = x == nx - 2, nbm = orow == 1, nt = orow == ny - 2;
                            if ((nl || nr) && (nbm || nt))
                                med = med3(v11, nl ? v12 : v10, nbm ? v21 : v01);
                            else if (nl || nr)
                                med = med3(v01, v11, v21);
                            else if (nbm || nt)
                                med = med3(v10, v11, v12);
                            else
                                med = median9(v00, v01, v02, v10, v11, v12, v20, v21, v22);
                        }
                    }
                    const A phi = limiter_phi(P.dpost, has_med, med, D, mask);
                    const A k = phi * c;
#pragma unroll
                    for (int i = 0; i < Q; ++i) Store<T>::st(dst + i * plane + obase, P.gs[i] - k * P.d[i]);
                    if (mask & kMaskTrim) ++acc.trim;
                    if (mask & kMaskMedian) ++acc.filt;
                    if (phi < A(1) && isfinite(P.dpost))
                        acc.lim += double(P.dpost - delta_s_scaled<LAT, DS>(P, shift, c, phi));
                    if (nonposP) mask |= kMaskNonpos;
                    dsrec = P.dpost;
                } else if (clsP == kNodeWall) {
                    // bounce-back: every population leaves reversed, no collision
#pragma unroll
                    for (int i = 0; i < Q; ++i) Store<T>::st(dst + i * plane + obase, P.gs[L::opp(i)]);
                    mask = kMaskNotFluid;
                } else {
                    // lid: f*(rho0, (u0, 0)) in shift form
                    A E[Q];
                    eq_excess<LAT, QE>(A(D.lid_ux), A(0), E);
                    const A r0 = A(D.rho0);
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        Store<T>::st(dst + i * plane + obase, A(L::w(i)) * ((r0 - shift) + r0 * E[i]));
                    mask = kMaskNotFluid;
                }
                if (record) {
                    to_global<unsigned char>(D.mask)[obase] = (unsigned char)mask;
                    to_global<double>(D.dS)[obase] = double(dsrec);
                }
            }
        }
        P = N;
        clsP = clsN;
        nonposP = nonposN;
#pragma unroll
        for (int i = 0; i < Q; ++i) gcur[i] = gnext[i];
    }
    store_partial(acc, a.partials + ((long long)a.parity * a.ntiles + xcd_spatial(blockIdx.x, a.ntiles)) * kNStat,
                  red);
}

// D1Q3: each workgroup computes Delta S' at kThreads consecutive sites and
// updates the kThreads - 2 inner ones (3-point median, Sec. 4.3.2).
template <class T, int QE, int DS, int BC>
__global__ void __launch_bounds__(kThreads) k_step1d(StepArgs a)
{
    using A = typename Store<T>::A;
    constexpr int LAT = kD1Q3;
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    __shared__ A ds[kThreads];
    __shared__ double red[4 * kNStat];

    if (int(blockIdx.x) == a.ntiles) {
        reduce_block(a, red);
        return;
    }
    const Tile t = a.tiles[blockIdx.x];
    const DomainDev& D = a.dom[t.domain];
    const int tid = threadIdx.x;
    const int nx = D.nx;
    const long long plane = D.plane;
    const gptr<const T> src = to_global<T>(static_cast<const void*>(D.buf[a.parity]));
    const gptr<T> dst = to_global<T>(D.buf[1 - a.parity]);
    const A shift = A(D.shift), c = A(D.c);
    const long long step = a.counter[a.parity];

    const int xr = t.x0 - 1 + tid;
    const bool inside = BC == kPeriodic ? true : (xr >= 0 && xr < nx);
    const int x = BC == kPeriodic ? wrapi(xr, nx) : xr;
    const bool owned = tid >= 1 && tid <= kThreads - 2 && xr < nx && xr < t.x0 + a.tile_w;

    Acc acc;
    A g[Q];
    SiteState<LAT, A> S;
    SiteScalars sc;
    A dsv = A(0);
    if (inside) {
        gather<LAT, BC>(src, plane, nx, 1, x, 0, g);
        collide_site<LAT, QE, DS>(g, shift, c, S, sc, owned);
        dsv = S.dpost;
        if (owned) {
            acc.moments(sc);
            acc.fluid_site(sc, S.dpost);
            if (a.flags & kFlagEntropy) {
                const double e = entropy_site<LAT>(g, shift);
                if (isfinite(e)) acc.ent += e;
            }
            if (x == D.probe_x) {
                const gptr<float> p = to_global<float>(D.probe) + 2 * (step % D.probe_cap);
                p[0] = sc.ux;
                p[1] = 0.0f;
            }
        }
    }
    ds[tid] = dsv;
    __syncthreads();
    if (owned) {
        unsigned mask = 0;
        const bool has_med = (D.limiter & kLimMedian) && (BC == kPeriodic || (x >= 1 && x <= nx - 2));
        const A med = has_med ? med3(ds[tid - 1], ds[tid], ds[tid + 1]) : A(0);
        const A phi = limiter_phi(S.dpost, has_med, med, D, mask);
        const A k = phi * c;
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<T>::st(dst + i * plane + x, S.gs[i] - k * S.d[i]);
        if (mask & kMaskTrim) ++acc.trim;
        if (mask & kMaskMedian) ++acc.filt;
        if (phi < A(1) && isfinite(S.dpost)) acc.lim += double(S.dpost - delta_s_scaled<LAT, DS>(S, shift, c, phi));
        if (sc.nonpos) mask |= kMaskNonpos;
        if (a.flags & kFlagRecord) {
            to_global<unsigned char>(D.mask)[x] = (unsigned char)mask;
            to_global<double>(D.dS)[x] = double(S.dpost);
        }
    }
    store_partial(acc, a.partials + ((long long)a.parity * a.ntiles + xcd_spatial(blockIdx.x, a.ntiles)) * kNStat,
                  red);
}

// one instantiation per (quasiequilibrium, Delta S form, boundary) in use:
// the 2-D kernel serves periodic and cavity grids, the 1-D one periodic and tube
#define LBM_CASE(KER, Q_, D_, B_, ...) \
    case Q_ * 100 + D_ * 10 + B_: hipLaunchKernelGGL((KER<StT, Q_, D_, B_>), __VA_ARGS__); break;
#define LBM_DISPATCH(KER, B0, B1, ...)                                                                 \
    do {                                                                                               \
        switch (qe * 100 + ds * 10 + bc) {                                                             \
            LBM_CASE(KER, 0, 0, B0, __VA_ARGS__)                                                       \
            LBM_CASE(KER, 0, 0, B1, __VA_ARGS__)                                                       \
            LBM_CASE(KER, 0, 1, B0, __VA_ARGS__)                                                       \
            LBM_CASE(KER, 0, 1, B1, __VA_ARGS__)                                                       \
            LBM_CASE(KER, 1, 0, B0, __VA_ARGS__)                                                       \
            LBM_CASE(KER, 1, 0, B1, __VA_ARGS__)                                                       \
            LBM_CASE(KER, 1, 1, B0, __VA_ARGS__)                                                       \
            LBM_CASE(KER, 1, 1, B1, __VA_ARGS__)                                                       \
        default: return hipErrorInvalidValue;                                                          \
        }                                                                                              \
    } while (0)

hipError_t LBM_CAT(launch_step2d, LBM_SUFFIX)(int qe, int ds, int bc, const StepArgs& a, int tx, int ty,
                                             hipStream_t s)
{
    if (tx * ty != kThreads) return hipErrorInvalidValue;
    LBM_DISPATCH(k_step2d, 0, 1, dim3(a.ntiles + 1), dim3(tx, ty), 0, s, a);
    return hipGetLastError();
}

hipError_t LBM_CAT(launch_step1d, LBM_SUFFIX)(int qe, int ds, int bc, const StepArgs& a, hipStream_t s)
{
    LBM_DISPATCH(k_step1d, 0, 2, dim3(a.ntiles + 1), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace lbm
