// Auxiliary kernels: initial equilibrium, conversion between the FP64 state
// f(x, t) and the stored pre-free-flight buffer, moments, stats finalisation,
// and the storage-type dispatch of the step kernels.
#include "lbm_device.h"

namespace lbm {

hipError_t launch_step2d_st0(int, int, int, const StepArgs&, int, hipStream_t);
hipError_t launch_step2d_st1(int, int, int, const StepArgs&, int, hipStream_t);
hipError_t launch_step2d_st2(int, int, int, const StepArgs&, int, hipStream_t);
hipError_t launch_step2d_st3(int, int, int, const StepArgs&, int, hipStream_t);
hipError_t launch_step1d_st0(int, int, int, const StepArgs&, int, hipStream_t);
hipError_t launch_step1d_st1(int, int, int, const StepArgs&, int, hipStream_t);
hipError_t launch_step1d_st2(int, int, int, const StepArgs&, int, hipStream_t);
hipError_t launch_step1d_st3(int, int, int, const StepArgs&, int, hipStream_t);

hipError_t launch_step2d(int storage, int qe, int ds, int bc, const StepArgs& a, int kernel, hipStream_t s)
{
    switch (storage) {
    case kF64: return launch_step2d_st0(qe, ds, bc, a, kernel, s);
    case kF32: return launch_step2d_st1(qe, ds, bc, a, kernel, s);
    case kF16: return launch_step2d_st2(qe, ds, bc, a, kernel, s);
    case kBF16: return launch_step2d_st3(qe, ds, bc, a, kernel, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step1d(int storage, int qe, int ds, int bc, const StepArgs& a, int kernel, hipStream_t s)
{
    switch (storage) {
    case kF64: return launch_step1d_st0(qe, ds, bc, a, kernel, s);
    case kF32: return launch_step1d_st1(qe, ds, bc, a, kernel, s);
    case kF16: return launch_step1d_st2(qe, ds, bc, a, kernel, s);
    case kBF16: return launch_step1d_st3(qe, ds, bc, a, kernel, s);
    }
    return hipErrorInvalidValue;
}

__global__ void k_finalize(StepArgs a, int parity_done, long long step)
{
    __shared__ double red[4 * kNStat];
    reduce_partials(a, parity_done, step, red);
}

// D2Q9: the set-0 partial of each group (kMaxTileH rows of one strip) is the
// sum of the collision partials of its rows (index row_first + y strips +
// strip), in row order.
__global__ void __launch_bounds__(kThreads) k_tile_rows(StepArgs a, int parity_done)
{
    __shared__ double red[4 * kNStat];
    __shared__ double rowbuf[kMaxTileH * kNStat + 8 * kNStat];
    const Tile t = a.groups[blockIdx.x];
    const DomainDev& D = a.dom[t.domain];
    const long long r0 = (long long)D.row_first + (long long)t.y0 * D.strips + t.x0 / kThreads;
    const Acc none;
    store_partial_rows(none, a.partials + ((long long)parity_done * 2 * a.pstride + blockIdx.x) * kNStat, red,
                       a.rowpart + r0 * kNStat, t.y1 - t.y0, D.strips, rowbuf);
}

// E(Delta S') of this step and the thresholds of the ensemble limiters, per
// domain (Sec. 3.3, 3.4): the collision partials (set 0; for D2Q9 summed from
// the rows beforehand) are reduced exactly as the stats are, so E equals the
// reported mean_dS bit for bit.
__global__ void __launch_bounds__(kThreads) k_ens_prepare(StepArgs a, int parity)
{
    __shared__ double red[4 * kNStat];
    StepArgs b = a;
    b.median_pass = 0;
    reduce_partials(b, parity, a.counter[parity], red);
    __syncthreads();
    for (int d = threadIdx.x; d < a.ndomains; d += blockDim.x) {
        const DomainDev& D = a.dom[d];
        if (!(D.limiter & kLimEns)) continue;
        const double nf = D.stats[kSFluid];
        const double mean = nf > 0.0 ? D.stats[kSDpost] / nf : 0.0;
        D.ens[kEMean] = mean;
        D.ens[kEThresh] = fmax(D.ens_c * mean, D.delta_ens);
        D.ens[kESmoothA] = mean > 0.0 ? D.delta_ens / pow(mean, D.ens_k) : 0.0;
        if (D.limiter & kLimEnsBudget) {
            // eq. (EntThresh): the limiter may produce delta_0 times the
            // entropy production of the LBGK step, [1 - (2 beta - 1)^2] sum Delta S
            BudgetState& b = *D.bstate;
            const double budget = D.ens_c * (1.0 - D.c * D.c) * D.stats[kSDpost];
            b.prefix = 0;
            b.budget = budget;
            b.s_above = 0.0;
            b.c_above = 0.0;
            b.level = 0;
            b.done = budget > 0.0 ? 0 : 1;
            // no budget: the threshold sits at the largest value, nothing moves
            D.ens[kEBudget] = fmax(budget > 0.0 ? 0.0 : D.stats[kSMax], D.delta_ens);
        }
        if (D.limiter & kLimTopK) {
            // top-k trimming (Sec. 3.2): the k-th largest finite Delta S' by the
            // same radix selection, counts only; -inf (every node above
            // delta) until found
            BudgetState& b = *D.bstate;
            b.prefix = 0;
            b.budget = double(D.top_k);
            b.s_above = 0.0;
            b.c_above = 0.0;
            b.level = 0;
            b.done = 0;
            D.ens[kETopk] = -__builtin_huge_val();
        }
    }
}

// Keys of the budget selection: the bit pattern of a non-negative finite
// value (0 for values <= 0), ordered as the values are.
template <class A>
struct BKey;
template <>
struct BKey<double> {
    using U = unsigned long long;
    static constexpr bool dbl = true;
    static constexpr int mbits = 52, bias = 1075;
    __device__ static U key(double d) { return d > 0.0 ? U(__double_as_longlong(d)) : U(0); }
    __device__ static double value(U k) { return __longlong_as_double((long long)k); }
};
template <>
struct BKey<float> {
    using U = unsigned int;
    static constexpr bool dbl = false;
    static constexpr int mbits = 23, bias = 150;
    __device__ static U key(float d) { return d > 0.0f ? U(__float_as_uint(d)) : U(0); }
    __device__ static double value(U k) { return double(__uint_as_float(k)); }
};

// integer significand m and exponent e of a key: value = m 2^e
template <class K>
__device__ inline unsigned long long key_significand(typename K::U k)
{
    using U = typename K::U;
    const U e = k >> K::mbits;
    return (unsigned long long)((k & ((U(1) << K::mbits) - 1)) | (e ? (U(1) << K::mbits) : U(0)));
}
template <class K>
__device__ inline int key_exponent(typename K::U k)
{
    const int e = int(k >> K::mbits);
    return (e ? e : 1) - K::bias;
}

// One level of the budget selection: per tile, a histogram of the digit
// (count and exact significand sum per bucket) of the values whose higher
// digits match the prefix, added into the domain's histogram.  Each thread
// walks one column of the tile and merges runs of equal buckets in registers
// first (at most kMaxTileH values: the significand sum stays below 2^59).
template <class A, bool CAV>
__global__ void __launch_bounds__(kThreads) k_budget_hist(StepArgs a, int level)
{
    using K = BKey<A>;
    using U = typename K::U;
    __shared__ unsigned hn[kBudgetBuckets];
    __shared__ unsigned long long hlo[kBudgetBuckets];
    __shared__ unsigned hhi[kBudgetBuckets];
    const Tile t = a.tiles[blockIdx.x];
    const DomainDev& D = a.dom[t.domain];
    if (!(D.limiter & (kLimEnsBudget | kLimTopK)) || D.bstate->done) return;
    const unsigned long long prefix = D.bstate->prefix;
    const int lo = budget_lo(K::dbl, level), hi = budget_hi(K::dbl, level);
    const U dmask = (U(1) << (hi - lo)) - 1;
    for (int k = threadIdx.x; k < kBudgetBuckets; k += kThreads) {
        hn[k] = 0;
        hlo[k] = 0;
        hhi[k] = 0;
    }
    __syncthreads();
    const int x = t.x0 + int(threadIdx.x);
    auto flush = [&](int b, unsigned cnt, unsigned long long sum) {
        atomicAdd(&hn[b], cnt);
        const unsigned long long old = atomicAdd(&hlo[b], sum);
        if (old + sum < old) atomicAdd(&hhi[b], 1u);
    };
    if (x < t.x1) {
        const A* ds = static_cast<const A*>(D.dsbuf);
        int cur = -1;
        unsigned cnt = 0;
        unsigned long long sum = 0;
        for (int y = t.y0; y < t.y1; ++y) {
            if (CAV && (x == 0 || x == D.nx - 1 || y == 0 || y == D.ny - 1)) continue;   // walls and lid
            const A d = ds[(long long)y * D.nx + x];
            if (!isfinite(d)) continue;
            const U k = K::key(d);
            if ((unsigned long long)(k >> hi) != prefix) continue;
            const int b = int((k >> lo) & dmask);
            if (b != cur) {
                if (cnt) flush(cur, cnt, sum);
                cur = b;
                cnt = 0;
                sum = 0;
            }
            ++cnt;
            sum += key_significand<K>(k);
        }
        if (cnt) flush(cur, cnt, sum);
    }
    __syncthreads();
    BudgetBucket* gh = D.bhist;
    for (int k = threadIdx.x; k < kBudgetBuckets; k += kThreads)
        if (hn[k]) {
            atomicAdd(&gh[k].n, (unsigned long long)hn[k]);
            const unsigned long long old = atomicAdd(&gh[k].lo, hlo[k]);
            const unsigned long long hiadd = (unsigned long long)hhi[k] + (old + hlo[k] < old ? 1ull : 0ull);
            if (hiadd) atomicAdd(&gh[k].hi, hiadd);
        }
}

// One level of the budget selection, one workgroup per domain.  With
// g(t) = sum over values v > t of (v - t), decreasing in t, the threshold
// solves g(Delta S_0) = budget; it lies in the highest bucket whose lower
// edge L has g(L) >= budget.  That bucket's digit extends the prefix; at the
// last level the bucket is a single value v, g is linear above it, and
// Delta S_0 = (sum of the values above v - budget) / (their count).  The
// histogram is read in a fixed order and left zero for the next level.
template <class A>
__global__ void __launch_bounds__(kThreads) k_budget_select(StepArgs a, int level)
{
    using K = BKey<A>;
    using U = typename K::U;
    constexpr int per = kBudgetBuckets / kThreads;
    __shared__ double ts[kThreads], tc[kThreads];
    __shared__ int best;
    const DomainDev& D = a.dom[blockIdx.x];
    if (!(D.limiter & kLimEnsBudget)) return;
    BudgetState* bs = D.bstate;
    if (bs->done) return;
    const int tid = int(threadIdx.x);
    const unsigned long long prefix = bs->prefix;
    const int lo = budget_lo(K::dbl, level), hi = budget_hi(K::dbl, level);
    const int w = hi - lo;
    auto edge_of = [&](int b) { return U(((prefix << w) | (unsigned long long)b) << lo); };
    double s[per], c[per];
    double my_s = 0.0, my_c = 0.0;
#pragma unroll
    for (int i = per - 1; i >= 0; --i) {
        const int b = tid * per + i;
        BudgetBucket& gb = D.bhist[b];
        const unsigned long long n = gb.n, l = gb.lo, h = gb.hi;
        gb.n = 0;
        gb.lo = 0;
        gb.hi = 0;
        c[i] = double(n);
        s[i] = n ? ldexp(double(h) * 18446744073709551616.0 + double(l), key_exponent<K>(edge_of(b))) : 0.0;
        my_s += s[i];
        my_c += c[i];
    }
    ts[tid] = my_s;
    tc[tid] = my_c;
    if (tid == 0) best = -1;
    __syncthreads();
    if (tid == 0) {
        // sums above each thread's buckets, from the top down
        double rs = bs->s_above, rc = bs->c_above;
        for (int k = kThreads - 1; k >= 0; --k) {
            const double vs = ts[k], vc = tc[k];
            ts[k] = rs;
            tc[k] = rc;
            rs += vs;
            rc += vc;
        }
    }
    __syncthreads();
    const double budget = bs->budget;
    const int nb = 1 << w;   // buckets of this digit (the rest stay empty)
    double S = ts[tid], C = tc[tid];
    double sa = 0.0, ca = 0.0, sa0 = 0.0, ca0 = 0.0;
    int mine = -1;
#pragma unroll
    for (int i = per - 1; i >= 0; --i) {
        const int b = tid * per + i;
        const double L = b < nb ? K::value(edge_of(b)) : 0.0;
        if (i == 0) {
            sa0 = S;
            ca0 = C;
        }
        const double S1 = S + s[i], C1 = C + c[i];
        if (mine < 0 && b < nb && S1 - L * C1 >= budget) {
            mine = b;
            sa = S;
            ca = C;
        }
        S = S1;
        C = C1;
    }
    if (mine >= 0) atomicMax(&best, mine);
    __syncthreads();
    int j = best;
    if (j < 0 && level == 0) {
        // the budget exceeds g(0) = sum Delta S: every node goes to f*
        if (tid == 0) {
            D.ens[kEBudget] = fmax(0.0, D.delta_ens);
            bs->done = 1;
        }
        return;
    }
    if (j < 0) {
        // the lower edge of the parent bucket met the condition; rounding in
        // the regrouped sums may put it just below here: keep its lowest bucket
        j = 0;
        mine = tid == 0 ? 0 : -1;
        sa = sa0;
        ca = ca0;
    }
    if (mine != j) return;
    bs->prefix = (prefix << w) | (unsigned long long)j;
    bs->s_above = sa;
    bs->c_above = ca;
    bs->level = level + 1;
    if (level + 1 == budget_levels(K::dbl)) {
        const double v = K::value(edge_of(j));
        const double t0 = ca > 0.0 ? (sa - budget) / ca : v;
        D.ens[kEBudget] = fmax(fmax(t0, 0.0), D.delta_ens);
        bs->done = 1;
    }
}

// One level of the top-k selection, one workgroup per domain: the bucket
// holding the k-th largest value is the highest one where the count of the
// values at or above its lower edge reaches k.  At the last level the bucket
// is a single value, the k-th largest; trimming acts at and above it (ties
// included).  Fewer than k finite values: every node above delta.
template <class A>
__global__ void __launch_bounds__(kThreads) k_topk_select(StepArgs a, int level)
{
    using K = BKey<A>;
    using U = typename K::U;
    constexpr int per = kBudgetBuckets / kThreads;
    __shared__ double tc[kThreads];
    __shared__ int best;
    const DomainDev& D = a.dom[blockIdx.x];
    if (!(D.limiter & kLimTopK)) return;
    BudgetState* bs = D.bstate;
    if (bs->done) return;
    const int tid = int(threadIdx.x);
    const unsigned long long prefix = bs->prefix;
    const int lo = budget_lo(K::dbl, level), hi = budget_hi(K::dbl, level);
    const int w = hi - lo;
    const int nb = 1 << w;
    double c[per];
    double my_c = 0.0;
#pragma unroll
    for (int i = per - 1; i >= 0; --i) {
        BudgetBucket& gb = D.bhist[tid * per + i];
        c[i] = double(gb.n);
        gb.n = 0;
        gb.lo = 0;
        gb.hi = 0;
        my_c += c[i];
    }
    tc[tid] = my_c;
    if (tid == 0) best = -1;
    __syncthreads();
    if (tid == 0) {
        double rc = bs->c_above;
        for (int k = kThreads - 1; k >= 0; --k) {
            const double v = tc[k];
            tc[k] = rc;
            rc += v;
        }
    }
    __syncthreads();
    const double kk = bs->budget;
    double C = tc[tid], ca = 0.0, ca0 = 0.0;
    int mine = -1;
#pragma unroll
    for (int i = per - 1; i >= 0; --i) {
        const int b = tid * per + i;
        if (i == 0) ca0 = C;
        const double C1 = C + c[i];
        if (mine < 0 && b < nb && C1 >= kk) {
            mine = b;
            ca = C;
        }
        C = C1;
    }
    if (mine >= 0) atomicMax(&best, mine);
    __syncthreads();
    int j = best;
    if (j < 0 && level == 0) {
        if (tid == 0) bs->done = 1;      // fewer than k values: no limit
        return;
    }
    if (j < 0) {
        j = 0;
        mine = tid == 0 ? 0 : -1;
        ca = ca0;
    }
    if (mine != j) return;
    const U edge = U(((prefix << w) | (unsigned long long)j) << lo);
    bs->prefix = (prefix << w) | (unsigned long long)j;
    bs->c_above = ca;
    bs->level = level + 1;
    if (level + 1 == budget_levels(K::dbl)) {
        D.ens[kETopk] = K::value(edge);
        bs->done = 1;
    }
}

hipError_t launch_budget(int storage, int bc, const StepArgs& a, hipStream_t s)
{
    const bool dbl = storage == kF64;
    for (int level = 0; level < budget_levels(dbl); ++level) {
        if (dbl) {
            if (bc == kCavity)
                hipLaunchKernelGGL((k_budget_hist<double, true>), dim3(a.ntiles), dim3(kThreads), 0, s, a, level);
            else
                hipLaunchKernelGGL((k_budget_hist<double, false>), dim3(a.ntiles), dim3(kThreads), 0, s, a, level);
            hipLaunchKernelGGL(k_budget_select<double>, dim3(a.ndomains), dim3(kThreads), 0, s, a, level);
            hipLaunchKernelGGL(k_topk_select<double>, dim3(a.ndomains), dim3(kThreads), 0, s, a, level);
        } else {
            if (bc == kCavity)
                hipLaunchKernelGGL((k_budget_hist<float, true>), dim3(a.ntiles), dim3(kThreads), 0, s, a, level);
            else
                hipLaunchKernelGGL((k_budget_hist<float, false>), dim3(a.ntiles), dim3(kThreads), 0, s, a, level);
            hipLaunchKernelGGL(k_budget_select<float>, dim3(a.ndomains), dim3(kThreads), 0, s, a, level);
            hipLaunchKernelGGL(k_topk_select<float>, dim3(a.ndomains), dim3(kThreads), 0, s, a, level);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_ens_prepare(const StepArgs& a, hipStream_t s)
{
    if (a.nrows > 0) {
        hipLaunchKernelGGL(k_tile_rows, dim3(a.ngroups), dim3(kThreads), 0, s, a, a.parity);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_ens_prepare, dim3(1), dim3(kThreads), 0, s, a, a.parity);
    return hipGetLastError();
}

hipError_t launch_finalize(const StepArgs& a, int parity_done, long long steps_done, hipStream_t s)
{
    if (a.nrows > 0 && !a.fused) {
        hipLaunchKernelGGL(k_tile_rows, dim3(a.ngroups), dim3(kThreads), 0, s, a, parity_done);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, a, parity_done, steps_done);
    return hipGetLastError();
}

// The number of nodes the median filter moved in the step that read buffer
// parity_done: the sum of the second-pass partials (set 1) of every tile,
// which the two kernels and the fused step both write.  One workgroup, a
// fixed order of the sums.
__global__ void __launch_bounds__(kThreads) k_filtered_count(StepArgs a, int parity_done, double* out)
{
    __shared__ double red[kThreads];
    const double* part = a.partials + ((long long)parity_done * 2 + 1) * a.pstride * kNStat;
    double s = 0.0;
    for (int t = int(threadIdx.x); t < a.ntiles; t += kThreads) s += part[(long long)t * kNStat + kSFilt];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w /= 2) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_filtered_count(const StepArgs& a, int parity_done, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_filtered_count, dim3(1), dim3(kThreads), 0, s, a, parity_done, out);
    return hipGetLastError();
}

// f = f*(rho, u) at every node, FP64 (Sec. 4.1 quasiequilibria)
template <int LAT, int QE>
__global__ void k_init_f(const double* __restrict__ rho, const double* __restrict__ u, double* __restrict__ f,
                         int n)
{
    using L = Lat<LAT>;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double r = rho[s];
    const double ux = u[s];
    const double uy = LAT == kD2Q9 ? u[n + s] : 0.0;
    double E[L::Q];
    eq_excess<LAT, QE>(ux, uy, E);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) f[(long long)i * n + s] = r * L::w(i) * (1.0 + E[i]);
}

hipError_t launch_init_f(int lattice, int qe, const double* rho, const double* u, double* f, int nx, int ny,
                         hipStream_t s)
{
    const int n = nx * ny;
    const dim3 grid((n + 255) / 256), block(256);
    if (lattice == kD2Q9) {
        if (qe == kPoly) hipLaunchKernelGGL((k_init_f<kD2Q9, kPoly>), grid, block, 0, s, rho, u, f, n);
        else hipLaunchKernelGGL((k_init_f<kD2Q9, kEntropic>), grid, block, 0, s, rho, u, f, n);
    } else {
        if (qe == kPoly) hipLaunchKernelGGL((k_init_f<kD1Q3, kPoly>), grid, block, 0, s, rho, u, f, n);
        else hipLaunchKernelGGL((k_init_f<kD1Q3, kEntropic>), grid, block, 0, s, rho, u, f, n);
    }
    return hipGetLastError();
}

// The buffer holds the values o_i(x) about to leave x; the state is
// f_i(x) = o_i(x - v_i) (or o_opp(i)(x) off a non-periodic edge).  Scatter
// inverts that map: o_i(x) = f_i(x + v_i), or f_opp(i)(x) when x + v_i is off
// the grid.
template <int LAT, class T>
__global__ void k_scatter(const double* __restrict__ f, T* buf_, long long plane, int nx, int ny,
                          int periodic, double shift)
{
    using L = Lat<LAT>;
    const gptr<T> buf = to_global<T>(static_cast<void*>(buf_));
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = nx * ny;
    if (s >= n) return;
    const int x = s % nx, y = s / nx;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int tx = x + L::vx(i), ty = y + L::vy(i);
        double v;
        if (periodic) {
            tx = wrapi(tx, nx);
            ty = wrapi(ty, ny);
            v = f[(long long)i * n + ty * nx + tx];
        } else if (tx >= 0 && tx < nx && ty >= 0 && ty < ny) {
            v = f[(long long)i * n + ty * nx + tx];
        } else {
            v = f[(long long)L::opp(i) * n + s];
        }
        Store<T>::st(buf + i * plane + s, typename Store<T>::A(v - L::w(i) * shift));
    }
}

// Gather: f_i(x) from the buffer as FP64; optionally rho and u (eq. macro_dis)
template <int LAT, class T>
__global__ void k_gather(const T* buf_, long long plane, double* __restrict__ f, int nx, int ny,
                         int periodic, double shift, int want_f, double* __restrict__ rho, double* __restrict__ u)
{
    using L = Lat<LAT>;
    const gptr<const T> buf = to_global<T>(static_cast<const void*>(buf_));
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = nx * ny;
    if (s >= n) return;
    const int x = s % nx, y = s / nx;
    double r = 0, jx = 0, jy = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int sx = x - L::vx(i), sy = y - L::vy(i);
        long long off;
        if (periodic) {
            off = i * plane + wrapi(sy, ny) * nx + wrapi(sx, nx);
        } else if (sx >= 0 && sx < nx && sy >= 0 && sy < ny) {
            off = i * plane + sy * nx + sx;
        } else {
            off = L::opp(i) * plane + s;
        }
        const double v = double(Store<T>::ld(buf + off)) + L::w(i) * shift;
        if (want_f) f[(long long)i * n + s] = v;
        r += v;
        jx += L::vx(i) * v;
        jy += L::vy(i) * v;
    }
    if (rho) rho[s] = r;
    if (u) {
        u[s] = jx / r;
        if (LAT == kD2Q9) u[n + s] = jy / r;
    }
}

template <class T>
static hipError_t scatter_t(int lattice, int periodic, const double* f, void* buf, long long plane, int nx, int ny,
                            double shift, hipStream_t s)
{
    const int n = nx * ny;
    const dim3 grid((n + 255) / 256), block(256);
    if (lattice == kD2Q9)
        hipLaunchKernelGGL((k_scatter<kD2Q9, T>), grid, block, 0, s, f, (T*)buf, plane, nx, ny, periodic, shift);
    else
        hipLaunchKernelGGL((k_scatter<kD1Q3, T>), grid, block, 0, s, f, (T*)buf, plane, nx, ny, periodic, shift);
    return hipGetLastError();
}

template <class T>
static hipError_t gather_t(int lattice, int periodic, const void* buf, long long plane, double* f, int nx, int ny,
                           double shift, int want_f, double* rho, double* u, hipStream_t s)
{
    const int n = nx * ny;
    const dim3 grid((n + 255) / 256), block(256);
    if (lattice == kD2Q9)
        hipLaunchKernelGGL((k_gather<kD2Q9, T>), grid, block, 0, s, (const T*)buf, plane, f, nx, ny, periodic, shift,
                           want_f, rho, u);
    else
        hipLaunchKernelGGL((k_gather<kD1Q3, T>), grid, block, 0, s, (const T*)buf, plane, f, nx, ny, periodic, shift,
                           want_f, rho, u);
    return hipGetLastError();
}

hipError_t launch_scatter(int storage, int lattice, int bc, const double* f, void* buf, long long plane, int nx,
                          int ny, double shift, hipStream_t s)
{
    const int periodic = bc == kPeriodic;
    switch (storage) {
    case kF64: return scatter_t<double>(lattice, periodic, f, buf, plane, nx, ny, shift, s);
    case kF32: return scatter_t<float>(lattice, periodic, f, buf, plane, nx, ny, shift, s);
    case kF16: return scatter_t<_Float16>(lattice, periodic, f, buf, plane, nx, ny, shift, s);
    case kBF16: return scatter_t<__bf16>(lattice, periodic, f, buf, plane, nx, ny, shift, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gather(int storage, int lattice, int bc, const void* buf, long long plane, double* f, int nx, int ny,
                         double shift, int want_f, double* rho, double* u, hipStream_t s)
{
    const int periodic = bc == kPeriodic;
    switch (storage) {
    case kF64: return gather_t<double>(lattice, periodic, buf, plane, f, nx, ny, shift, want_f, rho, u, s);
    case kF32: return gather_t<float>(lattice, periodic, buf, plane, f, nx, ny, shift, want_f, rho, u, s);
    case kF16: return gather_t<_Float16>(lattice, periodic, buf, plane, f, nx, ny, shift, want_f, rho, u, s);
    case kBF16: return gather_t<__bf16>(lattice, periodic, buf, plane, f, nx, ny, shift, want_f, rho, u, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
