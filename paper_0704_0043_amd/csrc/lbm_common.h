// Structures shared by the host runtime (lbm.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

enum { kD1Q3 = 1, kD2Q9 = 2 };
enum { kPoly = 0, kEntropic = 1 };
enum { kExact = 0, kQuad = 1 };
enum { kPeriodic = 0, kCavity = 1, kTube = 2 };
enum { kLimTrim = 1, kLimMedian = 2, kLimEnsThresh = 4, kLimEnsSmooth = 8, kLimEnsRational = 16,
       kLimEnsBudget = 32, kLimPos = 64,
       // internal: trimming limited to the top_k largest Delta S' (a second-pass
       // limiter; the domain's kLimTrim bit is cleared on the device)
       kLimTopK = 128, kLimEns = 4 | 8 | 16 | 32 | 128 };
enum { kLBGK = 0, kELBM = 1 };
enum { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

enum : unsigned { kMaskTrim = 1, kMaskMedian = 2, kMaskNonpos = 4, kMaskNotFluid = 8, kMaskEns = 16, kMaskPos = 32 };
// kFlagAllTiles makes the second pass walk every tile, as if each had a
// candidate; only the tuner sets it, to time that pass's full work.
enum : unsigned { kFlagRecord = 1, kFlagEntropy = 2, kFlagAllTiles = 4 };

constexpr int kThreads = 256;      // workgroup size of the step kernels (= D2Q9 tile width)
constexpr int kWave = 64;          // wavefront size (CDNA)
constexpr int kMaxTileH = 64;      // rows per D2Q9 tile
constexpr int kNStat = 16;         // FP64 values per tile partial

// partial / stats slot layout (FP64 each)
enum {
    kSMass = 0,   // sum of rho - shift (the shift is added back on the host)
    kSJx, kSJy,
    kSDpre, kSDpost, kSMax, kSLim, kSEnt,
    kSTrim, kSFilt, kSNonpos, kSNonfin, kSFluid,
    kSAbove,      // median candidates (Delta S' > delta_median); in a collision partial: bit w set
                  // when wave w of the segment holds one (that wave stored its Delta S')
    kSEns,        // nodes an ensemble-dependent limiter moved
    kSPos         // nodes the positivity rule moved (limiter, or ELBM without a root)
};

// per-domain ensemble values of the current step (device array of kNEns doubles)
enum { kEMean = 0, kEThresh, kESmoothA, kEBudget, kETopk, kNEns };

// Entropy-budget threshold (eq. EntThresh) by radix selection over the bit
// patterns of the non-negative Delta S' values, most significant digit
// first.  Each level histograms one digit of the values whose higher digits
// equal the prefix chosen so far.  A bucket holds values of one binary
// exponent, so its sum is kept exactly as the integer sum of the
// significands: the histogram does not depend on the order of the additions,
// and neither does the threshold.
constexpr int kBudgetBuckets = 2048;
struct BudgetState {
    unsigned long long prefix;   // digits chosen so far
    double budget;               // delta_0 [1 - (2 beta - 1)^2] sum Delta S'
    double s_above, c_above;     // sum and count of the values above the chosen bucket
    int level, done;
};
struct BudgetBucket {
    unsigned long long n, lo, hi;   // count; significand sum = hi 2^64 + lo
};
// key digits: FP64 keys 11 bits (the exponent), 11, 11, 10, 10, 10; FP32 keys
// 11 bits (the exponent and 3 significand bits), 10, 10
__host__ __device__ constexpr int budget_levels(bool dbl) { return dbl ? 6 : 3; }
__host__ __device__ constexpr int budget_lo(bool dbl, int level)
{
    return dbl ? (level == 0 ? 52 : level == 1 ? 41 : level == 2 ? 30 : level == 3 ? 20 : level == 4 ? 10 : 0)
               : (level == 0 ? 20 : level == 1 ? 10 : 0);
}
__host__ __device__ constexpr int budget_hi(bool dbl, int level)   // one past the digit's top bit
{
    return level == 0 ? (dbl ? 63 : 31) : budget_lo(dbl, level - 1);
}

// Per-domain parameters, device visible.  Pointers are device pointers.
struct DomainDev {
    void* buf[2];           // population planes (storage type), A and B
    long long plane;        // elements per population plane
    int nx, ny;
    double c;               // 2 beta - 1
    double shift;           // rho0 for shifted storage, 0 for FP64
    double delta_trim, delta_median;
    double rho0, lid_ux;
    int limiter, trim_mode, median_mode;
    int diffusive;          // cavity walls: 0 on-node bounce-back + equilibrium lid, 1 diffusive Maxwell
    int collision;          // kLBGK or kELBM
    int homothety;          // 1: homothety targets reached exactly with the exact Delta S
    long long top_k;        // kLimTopK: trimming at the top_k largest finite Delta S' only
    int probe_x, probe_y, probe_cap;
    float* probe;           // [probe_cap][2]
    unsigned char* mask;    // [ny*nx] when recording
    double* dS;             // [ny*nx] when recording
    int tile_first, tile_count;   // this domain's range in the tile table
    double ens_c, ens_k, delta_ens;   // ensemble limiter parameters
    double* ens;                  // [kNEns]: E(Delta S') and the thresholds of this step
    void* phibuf;                 // D1Q3 with ensemble limiters: phi applied by the first pass
    int strips;                   // D2Q9: column strips of kThreads columns
    int row_first, row_count;     // D2Q9: this domain's range of row partials (one per row and strip)
    int group_first, group_count; // this domain's range of collision-partial groups (kMaxTileH rows)
    BudgetState* bstate;          // budget threshold: search state (budget limiter only)
    BudgetBucket* bhist;          // [kBudgetBuckets], left zero between levels
    double* stats;          // [kNStat + 1]: last finalised sums, then the step index
    void* dsbuf;            // [ny*nx] Delta S' of the last collision (arithmetic type), median only
};

constexpr int kXcds = 8;   // MI355X: 8 accelerator dies, each with its own L2

// Workgroup b is dispatched to XCD b % 8.  Tiles are numbered in spatial
// order (domain, row chunk, column strip); XCD x takes one contiguous range
// of that order so neighbouring tiles share an L2.  This maps a block id to
// its spatial tile index (a bijection on [0, T)).
__host__ __device__ inline int xcd_spatial(int b, int T)
{
    const int x = b % kXcds, j = b / kXcds;
    const int q = T / kXcds, r = T % kXcds;
    return x * q + (x < r ? x : r) + j;
}

// One work item (one workgroup) over columns [x0, x1) of one domain.  The
// median kernel takes the consecutive rows [y0, y1); the collision kernel the
// rows ys, ys + ystep, ..., (yn of them).  With ystep = the number of row
// chunks, the collision tiles that run together all work on one narrow band
// of rows at a time, which keeps the DRAM pages they touch few and the rows
// their neighbours pull from in L2.
struct Tile {
    int domain, x0, x1, y0, y1, ys, ystep, yn;
};

constexpr int k1DWidth = kThreads - 2;   // output sites of one D1Q3 workgroup

// One D2Q9 collision workgroup: rows [y0, y1) by columns [x0, x1) of one
// domain, `width` (64, 128 or 256) columns per row, kThreads / width rows.
struct RowBlock {
    int domain, x0, x1, y0, y1, width;
};

// Columns of a domain's row blocks: with `narrow`, the narrowest of 64, 128
// and 256 that spans a row of a narrow domain (several of its rows then share
// a workgroup and fewer lanes idle), else 256.
__host__ __device__ inline int seg_width(int nx, int narrow)
{
    return (narrow && nx <= 64) ? 64 : ((narrow && nx <= 128) ? 128 : kThreads);
}

// Entry i of a domain's work tables (host and device build them alike):
// D2Q9 tiles of kThreads columns by th rows in spatial order (row chunk, then
// column strip); D2Q9 row blocks in row-major order; D1Q3 tiles of k1DWidth
// sites.
__host__ __device__ inline Tile tile_entry2d(int domain, int nx, int ny, int th, int i)
{
    const int strips = (nx + kThreads - 1) / kThreads;
    const int chunks = (ny + th - 1) / th;
    const int r = i / strips, x0 = (i - r * strips) * kThreads;
    return Tile{domain, x0, x0 + kThreads < nx ? x0 + kThreads : nx, r * th, r * th + th < ny ? r * th + th : ny,
                r, chunks, (ny - r + chunks - 1) / chunks};
}
__host__ __device__ inline int blocks_of(int nx, int ny, int width)
{
    const int rows = kThreads / width;
    return ((nx + width - 1) / width) * ((ny + rows - 1) / rows);
}
__host__ __device__ inline RowBlock block_entry2d(int domain, int nx, int ny, int width, int i)
{
    const int cols = (nx + width - 1) / width, rows = kThreads / width;
    const int r = i / cols, x0 = (i - r * cols) * width, y0 = r * rows;
    return RowBlock{domain, x0, x0 + width < nx ? x0 + width : nx, y0, y0 + rows < ny ? y0 + rows : ny, width};
}
__host__ __device__ inline Tile tile_entry1d(int domain, int nx, int i)
{
    const int x0 = i * k1DWidth;
    return Tile{domain, x0, x0 + k1DWidth < nx ? x0 + k1DWidth : nx, 0, 1, 0, 1, 1};
}
__host__ __device__ inline int tiles_of(int lattice, int nx, int ny, int th)
{
    return lattice == kD2Q9 ? ((nx + kThreads - 1) / kThreads) * ((ny + th - 1) / th) : (nx + k1DWidth - 1) / k1DWidth;
}

// The fused D2Q9 step (collision and median filter in one pass): each wave
// computes 64 adjacent columns and keeps the 62 inner ones (the two outer
// lanes supply the stencil's neighbours), so a workgroup of four waves owns
// kFusedWidth columns of a tile of th rows (plus one halo row above and
// below, computed for their Delta S' only).
constexpr int kFusedCols = kWave - 2;
constexpr int kFusedWidth = (kThreads / kWave) * kFusedCols;
__host__ __device__ inline int fused_tiles_of(int nx, int ny, int th)
{
    return ((nx + kFusedWidth - 1) / kFusedWidth) * ((ny + th - 1) / th);
}
__host__ __device__ inline Tile fused_tile_entry(int domain, int nx, int ny, int th, int i)
{
    const int strips = (nx + kFusedWidth - 1) / kFusedWidth;
    const int chunks = (ny + th - 1) / th;
    const int r = i / strips, x0 = (i - r * strips) * kFusedWidth;
    return Tile{domain, x0, x0 + kFusedWidth < nx ? x0 + kFusedWidth : nx, r * th, r * th + th < ny ? r * th + th : ny,
                r, chunks, 1};
}

struct StepArgs {
    const DomainDev* dom;
    const Tile* tiles;      // spatial order (domain, row chunk, column strip)
    int ntiles;             // the D2Q9 median pass (and D1Q3) has one workgroup per tile
    int ndomains;
    int parity;             // read buf[parity], write buf[1 - parity]
    unsigned flags;
    double* partials;       // [2 parities][2 sets][pstride][kNStat]: FP64 stats, set 0 (collision)
                            // per group of kMaxTileH rows, set 1 (second pass) per tile
    const Tile* groups;     // the collision-partial groups: tiles of kMaxTileH rows, fixed, so
                            // that the set-0 sums (and E(Delta S')) do not depend on the tile
                            // height; D1Q3: the tiles
    int ngroups;
    int pstride;            // slots per set in `partials` (>= ntiles, ngroups)
    int median_pass;        // 1 if a second pass (median and/or ensemble limiters) writes set 1
    int fused = 0;          // 1: the fused step kernel runs alone over `tiles` (fused tiles)
                            // and writes every partial to set 1
    int ens_pass;           // 1 if some domain has an ensemble-dependent limiter
    int budget;             // 1 if some domain has the budget threshold
    const RowBlock* rows;   // D2Q9 row blocks in row-major order, one per collision workgroup
    int nrows;              // the D2Q9 collision grid has nrows blocks
    double* rowpart;        // [rows x strips][kNStat]: collision partials of the last step, one
                            // per domain row and 256-column strip
    long long* counter;     // [2] step index by parity
};

// Allocation-free stepping (lbm_step_static): bytes of the per-GPU static
// device array that holds everything but the caller's population buffers.
constexpr size_t kStaticScratchBytes = LBM_STATIC_SCRATCH_BYTES;
// its address on `device` (looked up once per device; `device` must be current)
hipError_t static_scratch(int device, char** ptr);
hipError_t launch_static_setup(const DomainDev& dd, int lattice, DomainDev* dom, Tile* tiles, int ntiles,
                               RowBlock* rows, int nrows, long long* counter, hipStream_t s);
hipError_t launch_static_stats(const DomainDev* dom, double shift_mass, double* out, hipStream_t s);

// Launchers (one per storage type / lattice), defined in the .hip files.
// kernel 0: collision kernel (LBGK); kernel 2: the same with the ELBM collision;
// kernel 1: the second pass (median filter, ensemble factors; after kernel 0 or 2);
// kernel 3: the fused step (LBGK, trimming, positivity and median filter)
hipError_t launch_step2d(int storage, int qe, int ds, int bc, const StepArgs& a, int kernel, hipStream_t s);
// kernel 0: D1Q3 step (LBGK); kernel 2: the same with ELBM; kernel 1: D1Q3 ensemble pass
hipError_t launch_step1d(int storage, int qe, int ds, int bc, const StepArgs& a, int kernel, hipStream_t s);
// E(Delta S') and ensemble thresholds of the step just run (before the second pass)
hipError_t launch_ens_prepare(const StepArgs& a, hipStream_t s);
// the budget threshold of the step just run (after launch_ens_prepare)
hipError_t launch_budget(int storage, int bc, const StepArgs& a, hipStream_t s);
hipError_t launch_finalize(const StepArgs& a, int parity_done, long long steps_done, hipStream_t s);
// nodes moved by the median filter in the step that read buffer parity_done -> out[0]
hipError_t launch_filtered_count(const StepArgs& a, int parity_done, double* out, hipStream_t s);
hipError_t launch_init_f(int lattice, int qe, const double* rho, const double* u, double* f, int nx, int ny,
                         hipStream_t s);
hipError_t launch_scatter(int storage, int lattice, int bc, const double* f, void* buf, long long plane, int nx,
                          int ny, double shift, hipStream_t s);
hipError_t launch_gather(int storage, int lattice, int bc, const void* buf, long long plane, double* f, int nx,
                         int ny, double shift, int want_f, double* rho, double* u, hipStream_t s);

}  // namespace lbm
