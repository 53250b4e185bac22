// Fused limited LBGK step kernels for gfx950.
//
// Compiled once per population storage type (LBM_ST = 0..3).  A D2Q9 time
// step of every domain is one launch of the collision kernel and, when a
// limiter needs more than the node itself, one launch of the second pass:
//
//  collision: one thread per node, one workgroup per row segment of 256
//    columns, segments in row-major order, so the whole grid streams through
//    a narrow band of rows at a time.  Free flight (pull form, read from
//    buffer `parity`), moments, f*, the collision (LBGK, or ELBM in its own
//    instantiation), Delta S', the trimming and positivity factors (they
//    depend on the node alone), and the store of the limited post-collision
//    state into the other buffer.  With the median filter or an
//    ensemble-dependent limiter on, Delta S' also goes to a plane of its own.
//    Each workgroup leaves one partial of the reduction terms; the FP64
//    global sums are formed from these on demand, when the stats are read.
//  second pass: the 3x3 median of that plane and the ensemble-dependent
//    factors (thresholds from this step's E(Delta S') and selections) decide
//    which nodes move further; their stored limited states are rescaled
//    toward f* in place.
//
// The collision kernel is a plain streaming pass with aligned loads and
// stores and no barrier before its epilogue, the access pattern that
// sustains the highest HBM bandwidth on this part.
#include <type_traits>

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

// spatial tile of a workgroup: blocks are spread over the XCDs so that each
// XCD runs one contiguous stretch of tiles (rows sharing halo lines hit the
// same L2).  `first` is the block id of tile 0.
__device__ inline int tile_of_block(const StepArgs& a, int first)
{
    return xcd_spatial(int(blockIdx.x) - first, a.ntiles);
}

// per-tile FP64 partials: set 0 = collision rows (summed on demand; the D1Q3
// kernel writes it directly), set 1 = median pass
__device__ inline double* partial_slot(const StepArgs& a, int set, int tile)
{
    return a.partials + (((long long)a.parity * 2 + set) * a.pstride + tile) * kNStat;
}

// trimming factor of one node (it depends on the node alone, Sec. 3.2/3.4)
template <class A, class DD>
__device__ __forceinline__ A trim_phi(const DD& D, A dpost, unsigned& mask)
{
    A phi = A(1);
    if ((D.limiter & kLimTrim) && dpost > A(D.delta_trim)) {
        mask |= kMaskTrim;
        phi = D.trim_mode ? A(0) : sqrt_(A(D.delta_trim) * rcp(dpost));
    }
    return phi;
}

// Columns of one thread: pull sources of movers with vx = +1, 0, -1 as byte
// offsets (periodic wrap), and the thread's own column.
template <class T, int BC>
struct Cols {
    unsigned m, c, p, own;
    int x;
    bool ok;
    __device__ Cols(int x_, int nx, bool in) : x(x_), ok(in)
    {
        constexpr unsigned es = sizeof(T);
        if constexpr (BC == kPeriodic) {
            m = es * unsigned(x == 0 ? nx - 1 : x - 1);
            p = es * unsigned(x == nx - 1 ? 0 : x + 1);
        } else {
            m = es * unsigned(x - 1);
            p = es * unsigned(x + 1);
        }
        c = es * unsigned(x);
        own = c;
    }
};

// pull free flight of node (x, y): population i arriving there left
// (x - vx, y - vy); off a non-periodic edge it is the node's own opposite
// population (reflection: free flight stays a permutation)
template <int BC, class T>
__device__ __forceinline__ void gather2d(gptr<const T> src, long long plane, int nx, int ny, const Cols<T, BC>& cl,
                                         int y, typename Store<T>::A (&g)[9])
{
    using L = Lat<kD2Q9>;
    if constexpr (BC == kPeriodic) {
        const long long r0 = (long long)y * nx;
        const long long rm = (long long)(y == 0 ? ny - 1 : y - 1) * nx;
        const long long rp = (long long)(y == ny - 1 ? 0 : y + 1) * nx;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const long long rs = L::vy(i) > 0 ? rm : (L::vy(i) < 0 ? rp : r0);
            const unsigned cs = L::vx(i) > 0 ? cl.m : (L::vx(i) < 0 ? cl.p : cl.c);
            g[i] = Store<T>::ld(at_bytes(src + (i * plane + rs), cs));
        }
    } else {
        // A wave covers one row (callers keep it so), so the source rows are
        // scalars, clamped at the domain's edges like the lanes' columns; the
        // loads are then those of the periodic case.  A source off the domain
        // (at wall and lid nodes only) is replaced by the node's own opposite
        // population, loaded afterwards for those lanes alone.
        const int yw = __builtin_amdgcn_readfirstlane(y);
        const long long r0 = (long long)yw * nx;
        const long long rm = yw > 0 ? r0 - nx : r0;
        const long long rp = yw < ny - 1 ? r0 + nx : r0;
        constexpr unsigned es = sizeof(T);
        const int x = cl.x;
        const unsigned cc = es * unsigned(x);
        const unsigned cm = x > 0 ? cc - es : cc;
        const unsigned cp = x < nx - 1 ? cc + es : cc;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const long long rs = L::vy(i) > 0 ? rm : (L::vy(i) < 0 ? rp : r0);
            const unsigned cs = L::vx(i) > 0 ? cm : (L::vx(i) < 0 ? cp : cc);
            g[i] = Store<T>::ld(at_bytes(src + (i * plane + rs), cs));
        }
        const bool xm = x > 0, xp = x < nx - 1, ym = yw > 0, yp = yw < ny - 1;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const bool in = (L::vx(i) > 0 ? xm : (L::vx(i) < 0 ? xp : true)) &&
                            (L::vy(i) > 0 ? ym : (L::vy(i) < 0 ? yp : true));
            if (!in) g[i] = Store<T>::ld(at_bytes(src + (L::opp(i) * plane + r0), cc));
        }
    }
}

// Mass and momentum of a wall or lid node's nine populations in FP64 (its
// share of the stats), in population order; each population enters the
// momentum sums only where its velocity component is nonzero.
template <class A>
__device__ __forceinline__ void moments_fp64(const A (&g)[9], double& dr, double& jx, double& jy)
{
    using L = Lat<kD2Q9>;
    dr = 0.0;
    jx = 0.0;
    jy = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double v = double(g[i]);
        dr += v;
        if (L::vx(i) > 0) jx += v;
        if (L::vx(i) < 0) jx -= v;
        if (L::vy(i) > 0) jy += v;
        if (L::vy(i) < 0) jy -= v;
    }
}

// STREAM: the nontemporal hint, for a wave whose 64 lanes write whole
// aligned row segments; a wave that writes a segment sharing its end sectors
// with another wave's (the fused step) stores plainly, so that L2 merges the
// two halves of a sector before it goes to HBM
template <class T, bool STREAM = true>
__device__ __forceinline__ void store_limited(gptr<T> dst, long long plane, long long row, unsigned own,
                                              const SiteState<kD2Q9, typename Store<T>::A>& S,
                                              typename Store<T>::A phi, typename Store<T>::A c)
{
    using A = typename Store<T>::A;
    const A k = phi * c;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if constexpr (STREAM) Store<T>::st_stream(at_bytes(dst + (i * plane + row), own), S.gs[i] - k * S.d[i]);
        else Store<T>::st(at_bytes(dst + (i * plane + row), own), S.gs[i] - k * S.d[i]);
    }
}

// Diffusive Maxwell wall node (Sec. 4.4.2), inward normal (mx, my), wall
// velocity (uw, 0): the populations pointing into the fluid become
// gamma f*_i(1, u_wall), gamma = (mass that arrived from the fluid) / (mass of
// those f*_i), the others keep what free flight brought.  No collision.
template <class T, int QE>
__device__ __forceinline__ void diffusive_wall(gptr<T> dst, long long plane, long long row, unsigned own,
                                               const typename Store<T>::A (&g)[9], typename Store<T>::A shift,
                                               int mx, int my, typename Store<T>::A uw)
{
    using A = typename Store<T>::A;
    using L = Lat<kD2Q9>;
    A E[9];
    eq_excess<kD2Q9, QE>(uw, A(0), E);
    A sum_in = A(0), sum_arrived = A(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int d = L::vx(i) * mx + L::vy(i) * my;
        if (d > 0) sum_in += A(L::w(i)) * (A(1) + E[i]);
        if (d < 0) sum_arrived += A(L::w(i)) * shift + g[i];
    }
    const A gamma = sum_arrived / sum_in;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int d = L::vx(i) * mx + L::vy(i) * my;
        const A v = d > 0 ? gamma * (A(L::w(i)) * (A(1) + E[i])) - A(L::w(i)) * shift : g[i];
        Store<T>::st(at_bytes(dst + (i * plane + row), own), v);
    }
}

template <class T, int QE, int DS, int BC, bool ELBM = false>
__global__ void __launch_bounds__(kThreads) k_collide2d(StepArgs a)
{
    using A = typename Store<T>::A;
    using L = Lat<kD2Q9>;
    constexpr int Q = 9;
    __shared__ double red[4 * kNStat];
    // one row block per workgroup, in row-major order: the grid streams
    // through the domain a few rows at a time (DRAM pages and the rows that
    // neighbours pull from stay few), one node per thread; a block of a
    // narrow domain holds kThreads / width of its rows
    const int ridx = int(blockIdx.x);
    const RowBlock t = a.rows[ridx];
    const DomainDev& D = a.dom[t.domain];
    const int nx = D.nx, ny = D.ny;
    const long long plane = D.plane;
    const gptr<const T> src = to_global<T>(static_cast<const void*>(D.buf[a.parity]));
    const gptr<T> dst = to_global<T>(D.buf[1 - a.parity]);
    const gptr<A> dsb = to_global<A>(D.dsbuf);
    const A shift = A(D.shift), c = A(D.c);
    const bool record = a.flags & kFlagRecord;
    const bool want_ent = a.flags & kFlagEntropy;
    const bool keep_ds = D.limiter & (kLimMedian | kLimEns);
    const long long step = a.counter[a.parity];
    // the index of the next step, read by the next launch (which reads buffer 1 - parity)
    if (ridx == 0 && threadIdx.x == 0) a.counter[1 - a.parity] = step + 1;

    // The ensemble limiters and the GATE reading of the median use every
    // Delta S'.  The FLOOR median only needs the values above delta: its
    // threshold max(median, delta) and its decision are unchanged when every
    // value at or below delta is replaced by 0.  So there a wave with no node
    // above delta stores nothing, and the median pass reads its 64 columns as
    // zeros (the segment's partial records which waves stored).
    const bool every = (D.limiter & kLimEns) || D.median_mode != 0;
    AccT<A> acc;
    // the node (cl.x, y) of this thread
    auto visit = [&](const int y, const Cols<T, BC>& cl) {
        {
            A g[Q];
            gather2d<BC>(src, plane, nx, ny, cl, y, g);
            const long long row = (long long)y * nx;
            const unsigned node = unsigned(row) + unsigned(cl.x);
            const int cls = node_class<BC>(cl.x, y, nx, ny);
            if (cls == kNodeFluid) {
                SiteState<kD2Q9, A> S;
                SiteScalars sc;
                collide_site<kD2Q9, QE, DS, ELBM>(g, shift, c, S, sc, true);
                acc.moments(sc);
                acc.fluid_site(sc, S.dpost);
                if (want_ent) {
                    const double e = entropy_site<kD2Q9>(g, shift);
                    if (isfinite(e)) acc.ent += A(e);
                }
                if (cl.x == D.probe_x && y == D.probe_y) {
                    const gptr<float> p = to_global<float>(D.probe) + 2 * (step % D.probe_cap);
                    p[0] = sc.ux;
                    p[1] = sc.uy;
                }
                unsigned mask = 0;
                A phi = trim_phi(D, S.dpost, mask);
                if constexpr (DS == kExact) {
                    if (D.homothety && (mask & kMaskTrim) && !D.trim_mode && isfinite(S.dpost))
                        phi = exact_homothety<kD2Q9>(S, shift, A(D.delta_trim), S.dpost);
                }
                if (S.posrule) {
                    mask |= kMaskPos;
                    ++acc.pos;
                }
                if (D.limiter & kLimPos) {
                    const A pp = positivity_phi<kD2Q9>(S, shift);
                    if (pp < A(1)) {
                        mask |= kMaskPos;
                        ++acc.pos;
                        phi = fmin(phi, pp);
                    }
                }
                store_limited<T>(dst, plane, row, cl.own, S, phi, S.c);
                if (keep_ds) {
                    // NaN counts as above: such a wave always stores its values
                    const bool up = (D.limiter & kLimMedian) && !(S.dpost <= A(D.delta_median));
                    if (up) acc.above = 1;
                    if (every || __ballot(up) != 0) Store<A>::st(dsb + node, S.dpost);
                }
                if (mask & kMaskTrim) ++acc.trim;
                if (phi < A(1) && isfinite(S.dpost)) acc.lim += S.dpost - delta_s_scaled<kD2Q9, DS>(S, shift, S.c, phi);
                if (sc.nonpos) mask |= kMaskNonpos;
                if (record) {
                    to_global<unsigned char>(D.mask)[node] = (unsigned char)mask;
                    to_global<double>(D.dS)[node] = double(S.dpost);
                }
            } else {
                const bool corner = (cl.x == 0 || cl.x == nx - 1) && (y == 0 || y == ny - 1);
                if (D.diffusive && !corner) {
                    // diffusive Maxwell wall; the lid moves with (u0, 0)
                    const int mx = cl.x == 0 ? 1 : (cl.x == nx - 1 ? -1 : 0);
                    const int my = y == 0 ? 1 : (y == ny - 1 ? -1 : 0);
                    diffusive_wall<T, QE>(dst, plane, row, cl.own, g, shift, my != 0 ? 0 : mx, my,
                                          y == ny - 1 ? A(D.lid_ux) : A(0));
                } else if (cls == kNodeWall) {
                    // bounce-back: every population leaves reversed, no collision
#pragma unroll
                    for (int i = 0; i < Q; ++i) Store<T>::st(at_bytes(dst + (i * plane + row), cl.own), g[L::opp(i)]);
                } else {
                    // lid: f*(rho0, (u0, 0)) in shift form
                    A E[Q];
                    eq_excess<kD2Q9, QE>(A(D.lid_ux), A(0), E);
                    const A r0 = A(D.rho0);
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        Store<T>::st(at_bytes(dst + (i * plane + row), cl.own), A(L::w(i)) * ((r0 - shift) + r0 * E[i]));
                }
                SiteScalars sc;
                moments_fp64(g, sc.dr, sc.jx, sc.jy);
                acc.moments(sc);
                if (record) {
                    to_global<unsigned char>(D.mask)[node] = (unsigned char)kMaskNotFluid;
                    to_global<double>(D.dS)[node] = 0.0;
                }
            }
        }
    };
    if (t.width == kThreads) {
        // one row per block: its index is uniform, so are the row offsets
        // of every load and store (scalar bases, 32-bit lane offsets)
        const int x = t.x0 + int(threadIdx.x);
        const Cols<T, BC> cl(x, nx, x < t.x1);
        if (cl.ok) visit(t.y0, cl);
    } else {
        // a block of a narrow domain (its width a power of two: 64 or 128,
        // so that a wave never spans two rows, as the cavity gather needs)
        const int lx = int(threadIdx.x) & (t.width - 1), ly = int(threadIdx.x) >> __builtin_ctz(unsigned(t.width));
        const int y = t.y0 + ly;
        const Cols<T, BC> cl(t.x0 + lx, nx, t.x0 + lx < t.x1 && y < t.y1);
        if (cl.ok) visit(y, cl);
    }
    // one partial per row of the block (row y, strip x0 / kThreads)
    node_partial_rows(acc, a.rowpart + ((long long)D.row_first + (long long)t.y0 * D.strips + t.x0 / kThreads) * kNStat,
                      D.strips, t.width / kWave, t.y1 - t.y0, red);
}

// Second pass: median filter (Sec. 3.5; cavity stencils of Sec. 4.4) on the
// Delta S' plane written by the collision kernel, and the ensemble-dependent
// limiters.  Each thread walks down its column in chunks of kMedChunk rows:
// the loads of a whole chunk (one per row; the neighbouring columns come from
// the adjacent lanes) are issued together, then the decisions of the chunk
// are taken from registers, row by row, and last the chunk's moved nodes are
// rescaled with the loads of their stored states in flight together.  A node
// rescaled on the spot would make every row of a wave wait for its loads and
// for the acknowledgement of the previous row's stores; short chunks keep the
// window and the deferred states in few enough registers for four waves per
// SIMD.
constexpr int kMedChunk = 4;
constexpr int kPipe = 4;     // moved rows whose stored states are loaded together

// the filter's threshold and decision for a node with Delta S' = dc whose
// stencil median is med (FLOOR or GATE reading of the tolerance delta)
template <class A, class DD>
__device__ __forceinline__ bool median_decide(const DD& D, A dc, A med, A& thr)
{
    const A dmed = A(D.delta_median);
    if (D.median_mode) {
        thr = med;
        return dc > dmed && dc > med;
    }
    thr = fmax(med, dmed);
    return dc > thr;
}

// median threshold of a fluid node from its window (rows b, c, n = y-1, y, y+1;
// columns l, m, r = x-1, x, x+1); returns whether the filter hits the node
template <int BC, class A, class DD>
__device__ __forceinline__ bool median_hit(const DD& D, int x, int y, int nx, int ny, const A (&b)[3],
                                           const A (&c)[3], const A (&n)[3], A& thr)
{
    A med;
    if constexpr (BC == kPeriodic) {
        med = median9(b[0], b[1], b[2], c[0], c[1], c[2], n[0], n[1], n[2]);
    } else {
        // three nodes along a neighbouring wall; two inner axis neighbours
        // next to a corner; 3x3 elsewhere
        const bool wl = x == 1, wr = x == nx - 2, wb = y == 1, wt = y == ny - 2;
        if ((wl || wr) && (wb || wt))
            med = med3(c[1], wl ? c[2] : c[0], wb ? n[1] : b[1]);
        else if (wl || wr)
            med = med3(b[1], c[1], n[1]);
        else if (wb || wt)
            med = med3(c[0], c[1], c[2]);
        else
            med = median9(b[0], b[1], b[2], c[0], c[1], c[2], n[0], n[1], n[2]);
    }
    return median_decide(D, c[1], med, thr);
}

// A node the second pass moves further with the exact Delta S: rescale the
// limited state that the collision kernel stored at it toward its f*, rebuilt
// from the state's own moments (the limiter kept them): f* + r (f_stored - f*),
// r = pq / pt (the new factor over the applied one).  With the exact homothety
// the stored state's deviation e = pt x is scaled to the target directly, and
// a direct factor is taken relative to f' = f* + e / pt.  Returns the change of
// the limiter's entropy production (Delta S of the stored state minus Delta S
// of the new one).  A real call: its root solves would otherwise be inlined
// into every unrolled row of the median walk, and the walk's window would no
// longer fit in registers.  (The quadratic form rescales after each chunk's
// decisions, in the walk itself.)
template <class T, int QE>
__device__ __attribute__((noinline)) typename Store<T>::A rescale_stored_exact(
    gptr<T> buf, long long plane, long long rc, unsigned own, typename Store<T>::A shift, typename Store<T>::A pq,
    typename Store<T>::A pt, typename Store<T>::A tgt, typename Store<T>::A fac, typename Store<T>::A dc, bool exact)
{
    using A = typename Store<T>::A;
    constexpr int Q = 9;
    const gptr<const T> lsrc = buf;
    A gl[Q], gs[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) gl[i] = Store<T>::ld(at_bytes(lsrc + (i * plane + rc), own));
    A dr, jx, jy, rho, ux, uy;
    moments_equilibrium<kD2Q9, QE>(gl, shift, dr, jx, jy, rho, ux, uy, gs);
    A r = pq * rcp(pt);
    // deviation of the stored state
    A fs[Q], e[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        fs[i] = A(Lat<kD2Q9>::w(i)) * shift + gs[i];
        e[i] = (gl[i] - gs[i]) * rcp(fs[i]);
    }
    if (exact) {
        A ds_s = A(0), emin = A(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            ds_s += fs[i] * hkern(e[i]);
            emin = fmin(emin, e[i]);
        }
        r = A(1);
        if (ds_s > A(0)) {
            if (tgt < ds_s) r = kullback_scale<Q>(fs, e, tgt, sqrt_(tgt * rcp(ds_s)), A(0), A(1));
            if (fac < A(1)) {
                const A lmax = emin < A(0) ? A(-1) / emin : A(__builtin_huge_val());
                const A lam = pt < A(1) ? kullback_scale<Q>(fs, e, dc, sqrt_(dc * rcp(ds_s)), A(1), lmax) : A(1);
                r = fmin(r, fac * lam);
            }
        }
    }
    A lim = A(0);
    if (r < A(1)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<T>::st(at_bytes(buf + (i * plane + rc), own), gs[i] + r * (gl[i] - gs[i]));
        if (isfinite(dc)) {
            A ds_new = A(0), ds_old = A(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                ds_old += fs[i] * hkern(e[i]);
                ds_new += fs[i] * hkern(r * e[i]);
            }
            lim = ds_old - ds_new;
        }
    }
    return lim;
}

template <class T, int QE, int DS, int BC, bool ENS>
__device__ __forceinline__ void second_pass2d(const StepArgs& a)
{
    using A = typename Store<T>::A;
    constexpr int Q = 9;
    __shared__ double red[4 * kNStat];
    const int tidx = tile_of_block(a, 0);
    const Tile t = a.tiles[tidx];
    const DomainDev& D = a.dom[t.domain];
    if constexpr (!ENS) {
        // no median filter in this domain: an empty partial
        if (!(D.limiter & kLimMedian)) {
            if (threadIdx.x < kNStat) partial_slot(a, 1, tidx)[threadIdx.x] = 0.0;
            return;
        }
    }
    AccT<A, double> acc;
    const int nx = D.nx, ny = D.ny;
    const int x = t.x0 + int(threadIdx.x);
    // rows y0-1 .. y1 are read; y1 <= ny, so one wrap keeps them in range
    auto row_of = [&](int y) -> int {
        if constexpr (BC == kPeriodic)
            return y < 0 ? y + ny : (y >= ny ? y - ny : y);
        else
            return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
    };
    // FLOOR median only: the 64 columns of a collision wave in which no node
    // exceeded delta hold no Delta S' of this step and read as zeros.  Which
    // waves stored (bit w of the segment's candidate count) is staged in LDS
    // for the tile's rows and halo rows, for its own column strip and the two
    // neighbouring ones: [0] left, [1] own, [2] right.
    const bool sparse = !((D.limiter & kLimEns) || D.median_mode != 0);
    __shared__ int sflag[3][kMaxTileH + 2];
    const int strip = t.x0 / kThreads;
    int strip_l, strip_r;
    if constexpr (BC == kPeriodic) {
        strip_l = (t.x0 == 0 ? nx - 1 : t.x0 - 1) / kThreads;
        strip_r = (t.x1 == nx ? 0 : t.x1) / kThreads;
    } else {
        strip_l = (t.x0 == 0 ? 0 : t.x0 - 1) / kThreads;
        strip_r = (t.x1 == nx ? nx - 1 : t.x1) / kThreads;
    }
    // The filter's threshold is never below delta (FLOOR: max(median, delta);
    // GATE: only nodes above delta), so a tile none of whose nodes has
    // Delta S' > delta (the collision kernel counted them, in the same
    // precision) has nothing to filter and skips the medians.
    // The ensemble limiters use this step's E(Delta S') and thresholds;
    // threshold-type ones skip tiles whose largest Delta S' is at or below
    // the threshold (and that hold no infinite value), the smooth ones move
    // every node with Delta S' > 0.
    bool active = false;
    double ensv[kNEns] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (ENS) {
        if (D.limiter & kLimEns) {
#pragma unroll
            for (int k = 0; k < kNEns; ++k) ensv[k] = D.ens[k];
        }
    }
    if (D.limiter & (kLimMedian | kLimEns)) {
        const long long r0 = (long long)D.row_first + (long long)t.y0 * D.strips + t.x0 / kThreads;
        const int rows = t.y1 - t.y0;
        bool cand = false;
        if (int(threadIdx.x) < rows) {
            const double* rp = a.rowpart + (r0 + (long long)threadIdx.x * D.strips) * kNStat;
            const A mx = A(rp[kSMax]);
            const bool inf = rp[kSNonpos] > 0.0;
            if (D.limiter & kLimMedian) cand = cand || rp[kSAbove] > 0.0;
            if constexpr (ENS) {
                if (D.limiter & (kLimEnsSmooth | kLimEnsRational)) cand = cand || rp[kSFluid] > 0.0;
                if (D.limiter & kLimEnsThresh) cand = cand || inf || mx > A(ensv[kEThresh]);
                if (D.limiter & kLimEnsBudget) cand = cand || inf || mx > A(ensv[kEBudget]);
                if (D.limiter & kLimTopK) cand = cand || inf || mx > A(D.delta_trim);
            }
        }
        active = __syncthreads_or(cand || (a.flags & kFlagAllTiles));
        // staged only for a tile that has something to filter
        if (active && (D.limiter & kLimMedian) && sparse) {
            const int nr = rows + 2;
            for (int idx = int(threadIdx.x); idx < 3 * nr; idx += kThreads) {
                const int slot = idx / nr, ry = idx - slot * nr;
                const int s3 = slot == 0 ? strip_l : (slot == 1 ? strip : strip_r);
                const long long seg = (long long)D.row_first + (long long)row_of(t.y0 - 1 + ry) * D.strips + s3;
                sflag[slot][ry] = int(a.rowpart[seg * kNStat + kSAbove]);
            }
            __syncthreads();
        }
    }
    // nothing to filter in this tile: its partial is zero (no reduction)
    if (!active) {
        if (threadIdx.x < kNStat) partial_slot(a, 1, tidx)[threadIdx.x] = 0.0;
        return;
    }
    if (x < t.x1) {
        const long long plane = D.plane;
        const gptr<const A> dsb = to_global<A>(static_cast<const void*>(D.dsbuf));
        const A shift = A(D.shift);
        const bool record = a.flags & kFlagRecord;
        int xm, xp;
        if constexpr (BC == kPeriodic) {
            xm = x == 0 ? nx - 1 : x - 1;
            xp = x == nx - 1 ? 0 : x + 1;
        } else {
            // cavity: columns off the grid are never part of a fluid stencil
            xm = x > 0 ? x - 1 : x;
            xp = x < nx - 1 ? x + 1 : x;
        }
        const int sx = x / kThreads, sxm = xm / kThreads, sxp = xp / kThreads;
        const int wx = (x % kThreads) / kWave, wxm = (xm % kThreads) / kWave, wxp = (xp % kThreads) / kWave;
        const int slot_m = sxm == sx ? 1 : 0, slot_p = sxp == sx ? 1 : 2;
        // Each lane loads its own column (one aligned load per row); the
        // columns x -+ 1 come from the neighbouring lanes.  Only the first
        // lane of a wave and the lane at the right end of a wave or of the
        // tile load their outside neighbour themselves.
        const int lane = int(threadIdx.x) & (kWave - 1);
        const bool own_l = lane == 0;
        const bool own_r = lane == kWave - 1 || x == t.x1 - 1;
        auto load_raw = [&](int y, A (&r)[3]) {
            const int yy = row_of(y);
            const long long rr = (long long)yy * nx;
            r[1] = Store<A>::ld(dsb + (rr + x));
            if (own_l) r[0] = Store<A>::ld(dsb + (rr + xm));
            if (own_r) r[2] = Store<A>::ld(dsb + (rr + xp));
        };
        // zeros for the columns of waves that stored nothing (FLOOR median),
        // then the columns x -+ 1 from the neighbouring lanes
        auto complete = [&](int y, A (&r)[3]) {
            if (sparse) {
                const int ry = y - (t.y0 - 1);
                if (!((sflag[1][ry] >> wx) & 1)) r[1] = A(0);
                if (own_l && !((sflag[slot_m][ry] >> wxm) & 1)) r[0] = A(0);
                if (own_r && !((sflag[slot_p][ry] >> wxp) & 1)) r[2] = A(0);
            }
            // every active lane takes part in the shifts (no branch around them)
            const A l = lane_shift<-1>(r[1]), rr = lane_shift<+1>(r[1]);
            r[0] = own_l ? r[0] : l;
            r[2] = own_r ? r[2] : rr;
        };
        // w[k] holds row yb - 1 + k of the current chunk; the rows of the next
        // chunk are loaded into nw before the current chunk's rescale, so
        // waiting for them does not wait for that rescale's stores
        A w[kMedChunk + 2][3], nw[kMedChunk][3];
#pragma unroll
        for (int k = 0; k < kMedChunk + 2; ++k) w[k][0] = w[k][2] = A(0);
#pragma unroll
        for (int k = 0; k < kMedChunk; ++k) nw[k][0] = nw[k][1] = nw[k][2] = A(0);
        load_raw(t.y0 - 1, w[0]);
        load_raw(t.y0, w[1]);
        complete(t.y0 - 1, w[0]);
        complete(t.y0, w[1]);
#pragma unroll
        for (int k = 0; k < kMedChunk; ++k)
            if (t.y0 + k + 1 <= t.y1) load_raw(t.y0 + k + 1, nw[k]);
        for (int yb = t.y0; yb < t.y1; yb += kMedChunk) {
#pragma unroll
            for (int k = 0; k < kMedChunk; ++k)
                if (yb + k + 1 <= t.y1) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) w[k + 2][q] = nw[k][q];
                    complete(yb + k + 1, w[k + 2]);
                }
            // decisions for the rows of the chunk in order; with the exact
            // Delta S a moved node is rescaled on the spot by its lane (its
            // root solves are a real call), with the quadratic one after the
            // chunk
            unsigned mv = 0;          // rows of the chunk this lane rescales afterwards
            A rr[kMedChunk];          // their factor over the applied one
#pragma unroll
            for (int k = 0; k < kMedChunk; ++k) {
                const int y = yb + k;
                const A dc = w[k + 1][1];
                auto fluid = [&] { return y < t.y1 && node_class<BC>(x, y, nx, ny) == kNodeFluid; };
                // smallest homothety target and smallest direct factor of the
                // limiters that act on this node (relative to f')
                A tgt = A(__builtin_huge_val()), fac = A(1), thr;
                SecondHit h;
                if ((D.limiter & kLimMedian) && fluid() && median_hit<BC>(D, x, y, nx, ny, w[k], w[k + 1], w[k + 2], thr)) {
                    h.bits |= kMaskMedian;
                    tgt = thr;
                }
                if constexpr (ENS) {
                    if ((D.limiter & kLimEns) && fluid()) ens_terms(D, ensv, dc, tgt, fac, h);
                }
                if (h.bits) {
                    if (h.bits & kMaskMedian) ++acc.filt;
                    acc.ens += h.ens;
                    acc.trim += h.trim;
                    const long long rc = (long long)y * nx;
                    if (record) to_global<unsigned char>(D.mask)[unsigned(rc) + unsigned(x)] |= (unsigned char)h.bits;
                    unsigned tmask = 0;
                    // the factor the collision kernel applied (trimming)
                    const A pt = trim_phi(D, dc, tmask);
                    const A pq = fmin(fac, tgt < A(__builtin_huge_val()) ? sqrt_(tgt * rcp(dc)) : A(1));
                    bool exact = false;
                    if constexpr (DS == kExact) exact = D.homothety && isfinite(dc);
                    if constexpr (DS == kExact) {
                        if (exact || pq < pt) {
                            const gptr<T> buf = to_global<T>(D.buf[1 - a.parity]);
                            const unsigned own = unsigned(sizeof(T)) * unsigned(x);
                            acc.lim += rescale_stored_exact<T, QE>(buf, plane, rc, own, shift, pq, pt, tgt, fac, dc,
                                                                   exact);
                        }
                    } else if (pq < pt) {
                        // quadratic form: the factor is all the move needs
                        // (the limiter's entropy production follows from it),
                        // and the rescale is done after the chunk's decisions
                        mv |= 1u << k;
                        rr[k] = pq * rcp(pt);
                        if (isfinite(dc)) acc.lim += pt * pt * dc * (A(1) - rr[k] * rr[k]);
                    }
                }
            }
            {
                const int yn = yb + kMedChunk;
#pragma unroll
                for (int k = 0; k < kMedChunk; ++k)
                    if (yn < t.y1 && yn + k + 1 <= t.y1) load_raw(yn + k + 1, nw[k]);
            }
            if constexpr (DS != kExact) {
                // rescale the chunk's moved nodes kPipe rows at a time: the
                // loads of those rows are in flight together
                if (mv) {
                    const gptr<T> buf = to_global<T>(D.buf[1 - a.parity]);
                    const gptr<const T> lsrc = buf;
                    const unsigned own = unsigned(sizeof(T)) * unsigned(x);
#pragma unroll
                    for (int k0 = 0; k0 < kMedChunk; k0 += kPipe) {
                        A gl[kPipe][Q];
#pragma unroll
                        for (int u = 0; u < kPipe; ++u)
                            if ((mv >> (k0 + u)) & 1u) {
                                const long long rc = (long long)(yb + k0 + u) * nx;
#pragma unroll
                                for (int i = 0; i < Q; ++i)
                                    gl[u][i] = Store<T>::ld(at_bytes(lsrc + (i * plane + rc), own));
                            }
#pragma unroll
                        for (int u = 0; u < kPipe; ++u)
                            if ((mv >> (k0 + u)) & 1u) {
                                const long long rc = (long long)(yb + k0 + u) * nx;
                                A gs[Q], dr, jx, jy, rho, ux, uy;
                                moments_equilibrium<kD2Q9, QE>(gl[u], shift, dr, jx, jy, rho, ux, uy, gs);
                                const A r = rr[k0 + u];
#pragma unroll
                                for (int i = 0; i < Q; ++i)
                                    Store<T>::st(at_bytes(buf + (i * plane + rc), own), gs[i] + r * (gl[u][i] - gs[i]));
                            }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                w[0][q] = w[kMedChunk][q];
                w[1][q] = w[kMedChunk + 1][q];
            }
        }
    }
    store_partial(acc, partial_slot(a, 1, tidx), red);
}

// the second D2Q9 pass without and with ensemble-dependent limiters (the
// latter needs more registers)
template <class T, int QE, int DS, int BC>
__global__ void __launch_bounds__(kThreads) k_median2d(StepArgs a)
{
    second_pass2d<T, QE, DS, BC, false>(a);
}

template <class T, int QE, int DS, int BC>
__global__ void __launch_bounds__(kThreads) k_median_ens2d(StepArgs a)
{
    second_pass2d<T, QE, DS, BC, true>(a);
}

// The domain fields the fused step reads in its row loop.
struct FusedDom {
    int nx, ny, limiter, trim_mode, median_mode, homothety, diffusive, probe_x, probe_y, probe_cap;
    double delta_trim, delta_median, lid_ux, rho0;
    float* probe;
    unsigned char* mask;
    double* dS;
};

// the exact homothety as a real call (its root solve would otherwise be
// inlined twice into the fused kernel's row loop)
template <class A>
__device__ __attribute__((noinline)) A exact_homothety_call(const SiteState<kD2Q9, A>& o, A shift, A t, A dpost)
{
    return exact_homothety<kD2Q9>(o, shift, t, dpost);
}

// Fused D2Q9 step: collision, trimming, positivity and the median filter of
// Sec. 3.5 (cavity stencils of Sec. 4.4) in one pass, for domains without
// ensemble-dependent limiters.  Each wave walks down 64 adjacent columns of a
// tile, lane l on column xw - 1 + l: lanes 1..62 own the wave's columns, lanes
// 0 and 63 compute the neighbours that the owned columns' stencils read (their
// Delta S' reaches the owned lanes by DPP lane shifts), and the rows above
// and below the tile are computed for their Delta S' only.  A row is decided
// one row later, when the Delta S' of the row below it is known; meanwhile
// it keeps f* and the nonequilibrium part, so that its final state
// f* - phi c d is formed once, phi the smallest of the trimming, positivity
// and median factors (as in eq. (LimGenF) with the factors of Sec. 3).  The
// gathers of the next row are issued before the current row is computed.  No
// Delta S' plane is written; one FP64 partial per tile goes to set 1.
template <class T, int QE, int DS, int BC>
__global__ void __launch_bounds__(kThreads) k_fused2d(StepArgs a)
{
    using A = typename Store<T>::A;
    using L = Lat<kD2Q9>;
    constexpr int Q = 9;
    __shared__ double red[4 * kNStat];
    // the pending row's f* and nonequilibrium part, one column per thread
    // (each thread reads back only its own slots)
    __shared__ A pend[2 * Q][kThreads];
    const int tidx = tile_of_block(a, 0);
    const Tile t = a.tiles[tidx];
    // the fields the walk reads, copied once: held in scalar registers (read
    // through the table they would be reloaded, each time with a wait for
    // every load in flight, after each store)
    const DomainDev& Dt = a.dom[t.domain];
    const FusedDom D{Dt.nx, Dt.ny, Dt.limiter, Dt.trim_mode, Dt.median_mode, Dt.homothety, Dt.diffusive,
                     Dt.probe_x, Dt.probe_y, Dt.probe_cap, Dt.delta_trim, Dt.delta_median, Dt.lid_ux, Dt.rho0,
                     Dt.probe, Dt.mask, Dt.dS};
    const int nx = D.nx, ny = D.ny;
    const long long plane = Dt.plane;
    const gptr<const T> src = to_global<T>(static_cast<const void*>(Dt.buf[a.parity]));
    const gptr<T> dst = to_global<T>(Dt.buf[1 - a.parity]);
    const A shift = A(Dt.shift), c = A(Dt.c);
    const bool record = a.flags & kFlagRecord;
    const bool want_ent = a.flags & kFlagEntropy;
    const bool median = D.limiter & kLimMedian;
    const long long step = a.counter[a.parity];
    // the index of the next step, read by the next launch (which reads buffer 1 - parity)
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counter[1 - a.parity] = step + 1;

    const int lane = int(threadIdx.x) & (kWave - 1);
    const int xw = t.x0 + (int(threadIdx.x) >> 6) * kFusedCols;   // the wave's first owned column
    const int xw1 = xw + kFusedCols < t.x1 ? xw + kFusedCols : t.x1;
    // per-thread sums over the rows it owns: moments and limiter production
    // in FP64, the rest in the arithmetic type
    AccT<A, double> acc;
    double am = 0.0, ax = 0.0, ay = 0.0;
    if (xw < t.x1) {   // uniform per wave
        // the lane's column; lanes past the right neighbour of the last owned
        // column repeat it (their values are never used)
        const int x = xw - 1 + lane;
        const int xe = x < xw1 ? x : xw1;
        const bool owned = lane >= 1 && x < xw1;
        bool in_x = true;
        int xc = xe;
        if constexpr (BC == kPeriodic) {
            xc = xe < 0 ? xe + nx : (xe >= nx ? xe - nx : xe);
        } else {
            in_x = xe >= 0 && xe < nx;
            xc = xe < 0 ? 0 : (xe >= nx ? nx - 1 : xe);
        }
        const Cols<T, BC> cl(xc, nx, true);
        // rows y0 - 1 .. y1; off a cavity they are no nodes (clamped loads)
        auto row_of = [&](int y) -> int {
            if constexpr (BC == kPeriodic) return y < 0 ? y + ny : (y >= ny ? y - ny : y);
            else return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
        };
        // Delta S' window of the node's stencil: rows y - 2 (b), y - 1 (m)
        // and y (n) relative to the row being computed; [0] left, [1] own,
        // [2] right column
        A wb[3] = {A(0), A(0), A(0)}, wm[3] = {A(0), A(0), A(0)};
        // the pending row (the one above the row being computed): f* and d
        // in LDS, the rest here
        const int tid = int(threadIdx.x);
        A p_dpost = A(0), p_phi = A(1);
        unsigned p_mask = 0;
        bool p_fluid = false;
        // one row: collision of row y from its gathered populations g, then the
        // decision and store of row y - 1
        auto do_row = [&](int y, const A (&g)[Q]) {
            const int yr = row_of(y);
            const bool in_dom = in_x && (BC == kPeriodic || (y >= 0 && y < ny));
            const int cls = in_dom ? node_class<BC>(xc, yr, nx, ny) : int(kNodeNone);
            const bool own = owned && y >= t.y0 && y < t.y1;
            const long long row = (long long)yr * nx;
            const unsigned node = unsigned(row) + unsigned(xc);
            SiteState<kD2Q9, A> S;
            SiteScalars sc;
            A dcur = A(0);
            unsigned mask = 0;
            A phi = A(1);
            if (cls == kNodeFluid) {
                collide_site<kD2Q9, QE, DS, false>(g, shift, c, S, sc, true);
                dcur = S.dpost;
                if (own) {
                    am += sc.dr;
                    ax += sc.jx;
                    ay += sc.jy;
                    if (!(isfinite(sc.dr) && isfinite(sc.jx) && isfinite(sc.jy))) ++acc.nonfin;
                    acc.fluid_site(sc, S.dpost);
                    if (want_ent) {
                        const double e = entropy_site<kD2Q9>(g, shift);
                        if (isfinite(e)) acc.ent += A(e);
                    }
                    if (xc == D.probe_x && yr == D.probe_y) {
                        const gptr<float> pr = to_global<float>(D.probe) + 2 * (step % D.probe_cap);
                        pr[0] = sc.ux;
                        pr[1] = sc.uy;
                    }
                    phi = trim_phi(D, S.dpost, mask);
                    if constexpr (DS == kExact) {
                        if (D.homothety && (mask & kMaskTrim) && !D.trim_mode && isfinite(S.dpost))
                            phi = exact_homothety_call(S, shift, A(D.delta_trim), S.dpost);
                    }
                    if (D.limiter & kLimPos) {
                        const A pp = positivity_phi<kD2Q9>(S, shift);
                        if (pp < A(1)) {
                            mask |= kMaskPos;
                            ++acc.pos;
                            phi = fmin(phi, pp);
                        }
                    }
                    if (sc.nonpos) mask |= kMaskNonpos;
                    if (record) to_global<double>(D.dS)[node] = double(S.dpost);
                }
            } else if (own && cls != kNodeNone) {
                // walls and lid: no collision, no limiter; stored at once
                const unsigned ob = cl.own;
                const bool corner = (xc == 0 || xc == nx - 1) && (yr == 0 || yr == ny - 1);
                if (D.diffusive && !corner) {
                    const int mx = xc == 0 ? 1 : (xc == nx - 1 ? -1 : 0);
                    const int my = yr == 0 ? 1 : (yr == ny - 1 ? -1 : 0);
                    diffusive_wall<T, QE>(dst, plane, row, ob, g, shift, my != 0 ? 0 : mx, my,
                                          yr == ny - 1 ? A(D.lid_ux) : A(0));
                } else if (cls == kNodeWall) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) Store<T>::st(at_bytes(dst + (i * plane + row), ob), g[L::opp(i)]);
                } else {
                    A E[Q];
                    eq_excess<kD2Q9, QE>(A(D.lid_ux), A(0), E);
                    const A r0 = A(D.rho0);
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        Store<T>::st(at_bytes(dst + (i * plane + row), ob), A(L::w(i)) * ((r0 - shift) + r0 * E[i]));
                }
                double dr, jx, jy;
                moments_fp64(g, dr, jx, jy);
                am += dr;
                ax += jx;
                ay += jy;
                if (!(isfinite(dr) && isfinite(jx) && isfinite(jy))) ++acc.nonfin;
                if (record) {
                    to_global<unsigned char>(D.mask)[node] = (unsigned char)kMaskNotFluid;
                    to_global<double>(D.dS)[node] = 0.0;
                }
            }
            // this row's Delta S' with its neighbours' (every lane takes part)
            A wn[3];
            wn[1] = dcur;
            wn[0] = lane_shift<-1>(dcur);
            wn[2] = lane_shift<+1>(dcur);
            // decide and store the row above (row y - 1)
            const int yd = y - 1;
            if (owned && yd >= t.y0 && yd < t.y1 && p_fluid) {
                const int ydr = row_of(yd);
                const long long drow = (long long)ydr * nx;
                SiteState<kD2Q9, A> P;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    P.gs[i] = pend[i][tid];
                    P.d[i] = pend[Q + i][tid];
                }
                P.dpost = p_dpost;
                P.c = c;
                P.posrule = false;
                A thr;
                if (median && median_hit<BC>(D, xc, ydr, nx, ny, wb, wm, wn, thr)) {
                    p_mask |= kMaskMedian;
                    ++acc.filt;
                    A pm = A(1);
                    bool done = false;
                    if constexpr (DS == kExact) {
                        if (D.homothety && isfinite(p_dpost)) {
                            pm = exact_homothety_call(P, shift, thr, p_dpost);
                            done = true;
                        }
                    }
                    if (!done) pm = sqrt_(thr * rcp(p_dpost));
                    p_phi = fmin(p_phi, pm);
                }
                store_limited<T, false>(dst, plane, drow, cl.own, P, p_phi, c);
                if (p_mask & kMaskTrim) ++acc.trim;
                if (p_phi < A(1) && isfinite(p_dpost)) acc.lim += double(p_dpost - delta_s_scaled<kD2Q9, DS>(P, shift, c, p_phi));
                if (record) to_global<unsigned char>(D.mask)[unsigned(drow) + unsigned(xc)] = (unsigned char)p_mask;
            }
            // this row becomes the pending one
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                wb[k] = wm[k];
                wm[k] = wn[k];
            }
            p_fluid = own && cls == kNodeFluid;
            if (p_fluid) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    pend[i][tid] = S.gs[i];
                    pend[Q + i][tid] = S.d[i];
                }
                p_dpost = S.dpost;
                p_phi = phi;
                p_mask = mask;
            }
        };
        // rows y0 - 1 .. y1, the gathers of the next two rows in flight while a
        // row is computed (a wave walks its rows alone, so its own loads are
        // what hides the memory latency); three buffers used in turn, so no
        // register copy waits for a load.  The gathers are unconditional
        // (past the last row they repeat it and go unused): a load skipped on
        // one path would make every use wait for all loads in flight.
        auto fetch = [&](int y, A (&g)[Q]) { gather2d<BC>(src, plane, nx, ny, cl, row_of(y <= t.y1 ? y : t.y1), g); };
        A ga[Q], gb[Q], gc[Q];
        fetch(t.y0 - 1, ga);
        fetch(t.y0, gb);
        for (int y = t.y0 - 1;; y += 3) {
            fetch(y + 2, gc);
            do_row(y, ga);
            if (y + 1 > t.y1) break;
            fetch(y + 3, ga);
            do_row(y + 1, gb);
            if (y + 2 > t.y1) break;
            fetch(y + 4, gb);
            do_row(y + 2, gc);
            if (y + 3 > t.y1) break;
        }
    }
    AccT<double> tot;
    tot.mass = am;
    tot.jx = ax;
    tot.jy = ay;
    tot.dpre = double(acc.dpre);
    tot.dpost = double(acc.dpost);
    tot.maxd = double(acc.maxd);
    tot.lim = acc.lim;
    tot.ent = double(acc.ent);
    tot.trim = acc.trim;
    tot.filt = acc.filt;
    tot.nonpos = acc.nonpos;
    tot.nonfin = acc.nonfin;
    tot.fluid = acc.fluid;
    tot.pos = acc.pos;
    store_partial(tot, partial_slot(a, 1, tidx), red);
}

// D1Q3: each workgroup computes Delta S' at kThreads consecutive sites and
// updates the inner ones (3-point median, Sec. 4.3.2).
template <int BC, class T>
__device__ inline void gather1d(gptr<const T> src, long long plane, int nx, int x,
                                typename Store<T>::A (&g)[3])
{
    using L = Lat<kD1Q3>;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int xs = x - L::vx(i);
        long long off;
        if constexpr (BC == kPeriodic) {
            off = i * plane + wrapi(xs, nx);
        } else {
            off = (xs >= 0 && xs < nx) ? i * plane + xs : L::opp(i) * plane + x;
        }
        g[i] = Store<T>::ld(src + off);
    }
}

template <class T, int QE, int DS, int BC, bool ELBM = false>
__global__ void __launch_bounds__(kThreads) k_step1d(StepArgs a)
{
    using A = typename Store<T>::A;
    constexpr int LAT = kD1Q3;
    constexpr int Q = Lat<LAT>::Q;
    __shared__ A ds[kThreads];
    __shared__ double red[4 * kNStat];

    if (blockIdx.x == 0) {
        reduce_block(a, red);
        return;
    }
    const int tidx = tile_of_block(a, 1);
    const Tile t = a.tiles[tidx];
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
    const bool owned = tid >= 1 && tid <= kThreads - 2 && xr >= t.x0 && xr < t.x1;

    Acc acc;
    A g[Q];
    SiteState<LAT, A> S;
    SiteScalars sc;
    A dsv = A(0);
    if (inside) {
        gather1d<BC>(src, plane, nx, x, g);
        collide_site<LAT, QE, DS, ELBM>(g, shift, c, S, sc, owned);
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
        A tgt;
        A phi = limiter_phi(S.dpost, has_med, med, D, mask, tgt);
        if constexpr (DS == kExact) {
            if (D.homothety && phi > A(0) && tgt < A(__builtin_huge_val()) && isfinite(S.dpost))
                phi = exact_homothety<LAT>(S, shift, tgt, S.dpost);
        }
        if (S.posrule) {
            mask |= kMaskPos;
            ++acc.pos;
        }
        if (D.limiter & kLimPos) {
            const A pp = positivity_phi<LAT>(S, shift);
            if (pp < A(1)) {
                mask |= kMaskPos;
                ++acc.pos;
                phi = fmin(phi, pp);
            }
        }
        const A k = phi * S.c;
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<T>::st(dst + i * plane + x, S.gs[i] - k * S.d[i]);
        if (mask & kMaskTrim) ++acc.trim;
        if (mask & kMaskMedian) ++acc.filt;
        if (phi < A(1) && isfinite(S.dpost)) acc.lim += double(S.dpost - delta_s_scaled<LAT, DS>(S, shift, S.c, phi));
        if (sc.nonpos) mask |= kMaskNonpos;
        if (a.flags & kFlagRecord) {
            to_global<unsigned char>(D.mask)[x] = (unsigned char)mask;
            to_global<double>(D.dS)[x] = double(S.dpost);
        }
        if (D.limiter & kLimEns) {
            // for the ensemble pass: Delta S' and the factor applied here
            Store<A>::st(to_global<A>(D.dsbuf) + x, S.dpost);
            Store<A>::st(to_global<A>(D.phibuf) + x, phi);
        }
    }
    store_partial(acc, partial_slot(a, 0, tidx), red);
}

// D1Q3 ensemble pass (after the step kernel and the E(Delta S') reduction):
// a site whose ensemble factor is below the factor the step kernel applied is
// moved further toward its f*, rebuilt from the stored state's moments:
// f* + (phi_ens / phi_applied)(f_stored - f*).
template <class T, int QE, int DS, int BC>
__global__ void __launch_bounds__(kThreads) k_ens1d(StepArgs a)
{
    using A = typename Store<T>::A;
    constexpr int LAT = kD1Q3;
    constexpr int Q = Lat<LAT>::Q;
    __shared__ double red[4 * kNStat];
    const int tidx = int(blockIdx.x);
    const Tile t = a.tiles[tidx];
    const DomainDev& D = a.dom[t.domain];
    const int x = t.x0 + int(threadIdx.x);
    AccT<A> acc;
    if ((D.limiter & kLimEns) && x < t.x1) {
        double ensv[kNEns];
#pragma unroll
        for (int k = 0; k < kNEns; ++k) ensv[k] = D.ens[k];
        const A d = Store<A>::ld(to_global<A>(static_cast<const void*>(D.dsbuf)) + x);
        const A pa = Store<A>::ld(to_global<A>(static_cast<const void*>(D.phibuf)) + x);
        A tgt = A(__builtin_huge_val()), fac = A(1);
        SecondHit h;
        ens_terms(D, ensv, d, tgt, fac, h);
        if (h.bits) {
            acc.ens += h.ens;
            acc.trim += h.trim;
            if (a.flags & kFlagRecord) to_global<unsigned char>(D.mask)[x] |= (unsigned char)h.bits;
            const A pq = fmin(fac, tgt < A(__builtin_huge_val()) ? sqrt_(tgt * rcp(d)) : A(1));
            bool exact = false;
            if constexpr (DS == kExact) exact = D.homothety && isfinite(d) && pa > A(0);
            if (exact || pq < pa) {
                const long long plane = D.plane;
                const A shift = A(D.shift);
                const gptr<const T> lsrc = to_global<T>(static_cast<const void*>(D.buf[1 - a.parity]));
                const gptr<T> dst = to_global<T>(D.buf[1 - a.parity]);
                A gl[Q], gs[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) gl[i] = Store<T>::ld(lsrc + (i * plane + x));
                A dr, jx, jy, rho, ux, uy;
                moments_equilibrium<LAT, QE>(gl, shift, dr, jx, jy, rho, ux, uy, gs);
                A fs[Q], e[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    fs[i] = A(Lat<LAT>::w(i)) * shift + gs[i];
                    e[i] = (gl[i] - gs[i]) * rcp(fs[i]);
                }
                A r = pq * rcp(pa);
                if constexpr (DS == kExact) {
                    if (exact) {
                        // exact homothety from f' = f* + e / pa (Sec. 3.6)
                        A xp[Q];
#pragma unroll
                        for (int i = 0; i < Q; ++i) xp[i] = e[i] / pa;
                        A ph = fac;
                        if (tgt < d) ph = fmin(ph, kullback_scale<Q>(fs, xp, tgt, sqrt_(tgt * rcp(d)), A(0), A(1)));
                        r = ph / pa;
                    }
                }
                if (r < A(1)) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) Store<T>::st(dst + (i * plane + x), gs[i] + r * (gl[i] - gs[i]));
                    if (isfinite(d)) {
                        A ds_old, ds_new;
                        if constexpr (DS == kQuad) {
                            ds_old = pa * pa * d;
                            ds_new = r * r * pa * pa * d;
                        } else {
                            ds_old = ds_new = A(0);
#pragma unroll
                            for (int i = 0; i < Q; ++i) {
                                ds_old += fs[i] * hkern(e[i]);
                                ds_new += fs[i] * hkern(r * e[i]);
                            }
                        }
                        // the step kernel counted d - Delta S(stored)
                        acc.lim += ds_old - ds_new;
                    }
                }
            }
        }
    }
    store_partial(acc, partial_slot(a, 1, tidx), red);
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
// ELBM needs the entropic f*: kernels for qe = 1 only
#define LBM_CASE_E(KER, D_, B_, ...) \
    case 100 + D_ * 10 + B_: hipLaunchKernelGGL((KER<StT, 1, D_, B_, true>), __VA_ARGS__); break;
#define LBM_DISPATCH_ELBM(KER, B0, B1, ...)                                                            \
    do {                                                                                               \
        switch (qe * 100 + ds * 10 + bc) {                                                             \
            LBM_CASE_E(KER, 0, B0, __VA_ARGS__)                                                        \
            LBM_CASE_E(KER, 0, B1, __VA_ARGS__)                                                        \
            LBM_CASE_E(KER, 1, B0, __VA_ARGS__)                                                        \
            LBM_CASE_E(KER, 1, B1, __VA_ARGS__)                                                        \
        default: return hipErrorInvalidValue;                                                          \
        }                                                                                              \
    } while (0)

hipError_t LBM_CAT(launch_step2d, LBM_SUFFIX)(int qe, int ds, int bc, const StepArgs& a, int kernel,
                                             hipStream_t s)
{
    if (kernel == 0)
        LBM_DISPATCH(k_collide2d, 0, 1, dim3(a.nrows), dim3(kThreads), 0, s, a);
    else if (kernel == 2)
        LBM_DISPATCH_ELBM(k_collide2d, 0, 1, dim3(a.nrows), dim3(kThreads), 0, s, a);
    else if (kernel == 3)
        LBM_DISPATCH(k_fused2d, 0, 1, dim3(a.ntiles), dim3(kThreads), 0, s, a);
    else if (a.ens_pass)
        LBM_DISPATCH(k_median_ens2d, 0, 1, dim3(a.ntiles), dim3(kThreads), 0, s, a);
    else
        LBM_DISPATCH(k_median2d, 0, 1, dim3(a.ntiles), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t LBM_CAT(launch_step1d, LBM_SUFFIX)(int qe, int ds, int bc, const StepArgs& a, int kernel,
                                             hipStream_t s)
{
    if (kernel == 0)
        LBM_DISPATCH(k_step1d, 0, 2, dim3(a.ntiles + 1), dim3(kThreads), 0, s, a);
    else if (kernel == 2)
        LBM_DISPATCH_ELBM(k_step1d, 0, 2, dim3(a.ntiles + 1), dim3(kThreads), 0, s, a);
    else
        LBM_DISPATCH(k_ens1d, 0, 2, dim3(a.ntiles), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace lbm
