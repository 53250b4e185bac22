// Device memory of the allocation-free entry point lbm_step_static: one
// file-scope array per GPU that holds every array a step needs besides the
// caller's two population buffers (domain view, work tables, partials,
// Delta S' plane, counters, stats), and the kernels that prepare it
// and copy the stats out.  Nothing here allocates.
//
// The array's host-side name is only a stand-in for the device symbol: host
// code uses the address hipGetSymbolAddress returns for the current device,
// looked up once per device and kept.
#include <algorithm>
#include <mutex>

#include "lbm_common.h"

namespace lbm {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(int device, char** ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        // the caller made `device` current: its own copy of the array
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<char*>(p);
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

// Fills the domain view, the work tables (entries computed as the host
// builds them for a context) and clears what a run must start from: the
// step counters, the stats and the selection histogram.
__global__ void __launch_bounds__(kThreads) k_static_setup(DomainDev dd, int lattice, DomainDev* dom, Tile* tiles,
                                                           int ntiles, RowBlock* rows, int nrows, long long* counter)
{
    const int width = seg_width(dd.nx, 1);
    const int nb = dd.bhist ? kBudgetBuckets : 0;
    const int n = max(max(ntiles, nrows), max(nb, kNStat + 1));
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (i == 0) {
            *dom = dd;
            counter[0] = 0;
            counter[1] = 0;
        }
        if (i <= kNStat) dd.stats[i] = 0.0;
        if (i < ntiles)
            tiles[i] = lattice == kD2Q9 ? tile_entry2d(0, dd.nx, dd.ny, kMaxTileH, i) : tile_entry1d(0, dd.nx, i);
        if (i < nrows) rows[i] = block_entry2d(0, dd.nx, dd.ny, width, i);
        if (i < nb) dd.bhist[i] = BudgetBucket{0, 0, 0};
    }
}

// The finalised sums of the last step in the order of lbm_step_static's
// stats array: mass (the storage shift added back), momentum, sums of
// Delta S before and after collision, largest Delta S', limiter entropy
// production, then the counts.
__global__ void k_static_stats(const DomainDev* dom, double shift_mass, double* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double* s = dom->stats;
    out[0] = s[kSMass] + shift_mass;
    out[1] = s[kSJx];
    out[2] = s[kSJy];
    out[3] = s[kSDpre];
    out[4] = s[kSDpost];
    out[5] = s[kSMax];
    out[6] = s[kSLim];
    out[7] = s[kSTrim];
    out[8] = s[kSFilt];
    out[9] = s[kSNonpos];
    out[10] = s[kSNonfin];
    out[11] = s[kSFluid];
    out[12] = s[kSEns];
    out[13] = s[kSPos];
}

hipError_t launch_static_setup(const DomainDev& dd, int lattice, DomainDev* dom, Tile* tiles, int ntiles,
                               RowBlock* rows, int nrows, long long* counter, hipStream_t s)
{
    const int n = std::max(std::max(ntiles, nrows), std::max(kBudgetBuckets, kNStat + 1));
    const int blocks = std::min((n + kThreads - 1) / kThreads, 1024);
    hipLaunchKernelGGL(k_static_setup, dim3(blocks), dim3(kThreads), 0, s, dd, lattice, dom, tiles, ntiles, rows,
                       nrows, counter);
    return hipGetLastError();
}

hipError_t launch_static_stats(const DomainDev* dom, double shift_mass, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_static_stats, dim3(1), dim3(64), 0, s, dom, shift_mass, out);
    return hipGetLastError();
}

}  // namespace lbm
