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

// D2Q9: the partial of each tile is the sum of the collision partials of its
// rows (row table index row_first + y strips + strip), in row order.
__global__ void __launch_bounds__(kThreads) k_tile_rows(StepArgs a, int parity_done)
{
    __shared__ double red[4 * kNStat];
    __shared__ double rowbuf[kMaxTileH * kNStat + 8 * kNStat];
    const Tile t = a.tiles[blockIdx.x];
    const DomainDev& D = a.dom[t.domain];
    const long long r0 = (long long)D.row_first + (long long)t.y0 * D.strips + t.x0 / kThreads;
    const Acc none;
    store_partial_rows(none, a.partials + ((long long)parity_done * 2 * a.ntiles + blockIdx.x) * kNStat, red,
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
    }
}

hipError_t launch_ens_prepare(const StepArgs& a, hipStream_t s)
{
    if (a.nrows > 0) {
        hipLaunchKernelGGL(k_tile_rows, dim3(a.ntiles), dim3(kThreads), 0, s, a, a.parity);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_ens_prepare, dim3(1), dim3(kThreads), 0, s, a, a.parity);
    return hipGetLastError();
}

hipError_t launch_finalize(const StepArgs& a, int parity_done, long long steps_done, hipStream_t s)
{
    if (a.nrows > 0) {
        hipLaunchKernelGGL(k_tile_rows, dim3(a.ntiles), dim3(kThreads), 0, s, a, parity_done);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, a, parity_done, steps_done);
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
