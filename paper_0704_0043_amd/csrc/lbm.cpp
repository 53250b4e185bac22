// Host runtime and C ABI of the limited lattice Boltzmann step (see lbm.h).
//
// Owns the device memory of a context (or carves a caller workspace), builds
// the tile table of the step kernels (XCD-aware order), tunes the tile shape,
// captures chunks of steps into hipGraphs, and reads back state and stats.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_common.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

constexpr size_t kAlign = 256;
constexpr int kMinTuneH = 16;   // smallest median-tile height the tuner tries
constexpr int kMinFusedH = 4;   // smallest fused-tile height the tuner tries
constexpr int kMaxFusedH = 128; // tallest fused tile

// D2Q9 tiles: kThreads consecutive columns
int strips_of(int nx) { return (nx + kThreads - 1) / kThreads; }

bool is_cavity(int bc) { return bc == LBM_BC_CAVITY || bc == LBM_BC_CAVITY_DIFFUSIVE; }

// trimming limited to the top_k largest Delta S' (a second-pass limiter)
bool is_topk(const lbm_domain_desc& d) { return (d.limiter & LBM_LIM_TRIM) && d.top_k > 0; }
// limiters that need the whole domain's Delta S' before any node is limited
bool deferred(const lbm_domain_desc& d) { return (d.limiter & kLimEns) || is_topk(d); }

// the fused step applies: D2Q9 LBGK domains, the median filter in some, no
// ensemble-dependent limiter (nor top-k trimming) in any
bool fusable(const lbm_domain_desc* doms, int32_t nd)
{
    if (doms[0].lattice != LBM_D2Q9 || doms[0].collision == LBM_COLL_ELBM) return false;
    bool median = false;
    for (int k = 0; k < nd; ++k) {
        if (deferred(doms[k])) return false;
        median = median || (doms[k].limiter & LBM_LIM_MEDIAN);
    }
    return median;
}

// both forms of the step are kept and chosen between while the run goes
bool adaptive_run(const lbm_domain_desc* doms, int32_t nd, const lbm_run_desc* run)
{
    return (run->flags & LBM_RUN_ADAPTIVE) && run->tile_x != kFusedWidth && fusable(doms, nd);
}
// the device limiter mask: top-k trimming moves to the second pass
int device_limiter(const lbm_domain_desc& d)
{
    return is_topk(d) ? ((d.limiter & ~kLimTrim) | kLimTopK) : d.limiter;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int q_of(int lattice) { return lattice == LBM_D2Q9 ? 9 : 3; }

size_t elem_size(int storage)
{
    switch (storage) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    default: return 2;
    }
}

struct DomainHost {
    lbm_domain_desc d;     // copy without host pointers
    int q = 0;
    long long plane = 0;
    size_t n = 0;
    size_t off_buf[2] = {0, 0}, off_mask = 0, off_ds = 0, off_probe = 0, off_stats = 0, off_dsbuf = 0;
    size_t off_ens = 0, off_phibuf = 0, off_bstate = 0, off_bhist = 0;
    bool dsbuf = false, phibuf = false;
    double shift = 0;
    int tile_first = 0, tile_count = 0;
    int row_first = 0, row_count = 0;
    int group_first = 0, group_count = 0;
};

struct Layout {
    size_t off_dom = 0, off_tiles = 0, off_partials = 0, off_counter = 0, off_stage = 0, total = 0;
    size_t off_dom_alt = 0, off_tiles_alt = 0, off_adapt = 0;   // LBM_RUN_ADAPTIVE only
    size_t off_rows = 0, off_rowpart = 0, off_groups = 0;
    int max_tiles = 0, nrows = 0, ngroups = 0;
    size_t max_n = 0;
};

}  // namespace

struct lbm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int storage = LBM_F32, lattice = LBM_D2Q9, qe = 0, ds = 0, bc = 0;
    unsigned flags = 0;
    int stats_every = 0, probe_cap = 4096, graph_chunk = 64;
    std::vector<DomainHost> dom;
    Layout lay;
    char* ws = nullptr;
    bool own_ws = false;
    bool median_pass = false;   // D2Q9 with the median filter in some domain
    bool ens_pass = false;      // an ensemble-dependent limiter in some domain
    bool fuse_ok = false;       // the fused step applies (D2Q9 LBGK, median filter, no ensemble limiter)
    bool budget = false;        // the budget threshold in some domain
    bool elbm = false;          // ELBM collisions (all domains)
    long long steps_done = 0, finalized_for = -1;
    // captured step sequences, for each starting parity: graph_chunk steps
    // and every power of two below it, longest first
    struct StepGraph {
        int64_t len;
        hipGraphExec_t exec;
    };
    // One form of the step: the work tables it reads (tiles, and the domain
    // views that hold each domain's tile range), in workspace regions of its
    // own, and the graphs captured with them.  `act` runs the steps; with
    // LBM_RUN_ADAPTIVE, `alt` holds the other form (the fused step or the two
    // kernels) and the two trade places between chunks of steps.
    struct Slot {
        size_t off_dom = 0, off_tiles = 0;
        int th = 16;                    // rows per D2Q9 tile
        int ntiles = 0;
        bool fused = false;             // the fused step (tiles are fused tiles)
        std::vector<Tile> tiles_host;   // host copies kept alive for async uploads
        std::vector<DomainDev> dom_host;
        std::vector<StepGraph> graphs[2];
    };
    Slot act, alt;
    // LBM_RUN_ADAPTIVE: at every multiple of graph_chunk steps the filtered
    // count of the step just run goes to pinned host memory (no wait), and
    // the form of the next chunk is chosen from the count read back at the
    // previous such point
    bool adaptive = false;
    double fluid_total = 0;             // fluid nodes of all domains
    double* adapt_host = nullptr;       // [2] pinned
    hipEvent_t adapt_ev[2] = {nullptr, nullptr};
    bool adapt_pending[2] = {false, false};
    long long adapt_points = 0, next_check = 0;
    std::string err;
    std::vector<RowBlock> rows_host;
    std::vector<Tile> groups_host;
    int narrow = 1;             // row blocks of 64 / 128 columns for narrow domains
    int tuned = 0;              // 1 when the tile shape was chosen by timing

    DomainDev* d_dom() const { return reinterpret_cast<DomainDev*>(ws + act.off_dom); }
    Tile* d_tiles() const { return reinterpret_cast<Tile*>(ws + act.off_tiles); }
    double* d_adapt() const { return reinterpret_cast<double*>(ws + lay.off_adapt); }
    RowBlock* d_rows() const { return reinterpret_cast<RowBlock*>(ws + lay.off_rows); }
    Tile* d_groups() const { return reinterpret_cast<Tile*>(ws + lay.off_groups); }
    double* d_rowpart() const { return reinterpret_cast<double*>(ws + lay.off_rowpart); }
    double* d_partials() const { return reinterpret_cast<double*>(ws + lay.off_partials); }
    long long* d_counter() const { return reinterpret_cast<long long*>(ws + lay.off_counter); }
    double* d_stage() const { return reinterpret_cast<double*>(ws + lay.off_stage); }
};

namespace {

int fail(lbm_ctx* ctx, int code, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    g_err = msg;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool finite(double v) { return std::isfinite(v); }

int validate(const lbm_domain_desc* doms, int32_t nd, const lbm_run_desc* run)
{
    if (!doms || nd < 1 || !run) return fail(nullptr, LBM_EINVAL, "domains/run must be non-NULL, n_domains >= 1");
    if (run->struct_size < sizeof(lbm_run_desc)) return fail(nullptr, LBM_EINVAL, "lbm_run_desc.struct_size too small");
    if (run->storage < LBM_F64 || run->storage > LBM_BF16_SHIFT) return fail(nullptr, LBM_EINVAL, "bad storage");
    if (run->tile_x != 0 && run->tile_x != kWave && run->tile_x != kThreads && run->tile_x != kFusedWidth)
        return fail(nullptr, LBM_EINVAL, "tile_x must be 0 (tuned), 64 (narrow row blocks), 256 or 248 (fused step)");
    if (run->tile_y != 0 && run->tile_y != 1) return fail(nullptr, LBM_EINVAL, "tile_y must be 0 or 1");
    if (run->tile_h < 0 || run->tile_h > (run->tile_x == kFusedWidth ? kMaxFusedH : kMaxTileH))
        return fail(nullptr, LBM_EINVAL, "tile_h out of range [0, 64] (fused step: [0, 128])");
    if (run->graph_chunk < 0 || run->graph_chunk > 4096)
        return fail(nullptr, LBM_EINVAL, "graph_chunk out of range [0, 4096]");
    if (run->probe_capacity < 0) return fail(nullptr, LBM_EINVAL, "probe_capacity < 0");
    const lbm_domain_desc& d0 = doms[0];
    for (int k = 0; k < nd; ++k) {
        const lbm_domain_desc& d = doms[k];
        const std::string where = "domain " + std::to_string(k) + ": ";
        if (d.struct_size < sizeof(lbm_domain_desc)) return fail(nullptr, LBM_EINVAL, where + "struct_size too small");
        if (d.lattice != LBM_D1Q3 && d.lattice != LBM_D2Q9) return fail(nullptr, LBM_EINVAL, where + "bad lattice");
        if (d.lattice != d0.lattice || d.qe != d0.qe || d.ds_form != d0.ds_form || d.bc != d0.bc ||
            d.collision != d0.collision)
            return fail(nullptr, LBM_EINVAL, where + "lattice, qe, ds_form, bc and collision must match across domains");
        if (d.collision != LBM_COLL_LBGK && d.collision != LBM_COLL_ELBM)
            return fail(nullptr, LBM_EINVAL, where + "bad collision");
        if (d.collision == LBM_COLL_ELBM && d.qe != LBM_QE_ENTROPIC)
            return fail(nullptr, LBM_EINVAL, where + "ELBM needs the entropic f*");
        if (d.homothety != 0 && d.homothety != 1) return fail(nullptr, LBM_EINVAL, where + "bad homothety");
        if (d.top_k < 0) return fail(nullptr, LBM_EINVAL, where + "top_k must be >= 0");
        if (d.top_k > 0 && (d.limiter & LBM_LIM_ENS_BUDGET))
            return fail(nullptr, LBM_EINVAL, where + "top_k trimming and the budget threshold cannot share a domain");
        if (d.qe != LBM_QE_POLYNOMIAL && d.qe != LBM_QE_ENTROPIC) return fail(nullptr, LBM_EINVAL, where + "bad qe");
        if (d.ds_form != LBM_DS_EXACT && d.ds_form != LBM_DS_QUADRATIC) return fail(nullptr, LBM_EINVAL, where + "bad ds_form");
        if (d.limiter < 0 || d.limiter > 127) return fail(nullptr, LBM_EINVAL, where + "bad limiter mask");
        // a second pass rebuilds the applied factor from Delta S' alone, which
        // the positivity factor is not; with the exact Delta S a node it acts
        // on has Delta S' = +inf, and every second-pass limiter sends it to f*
        if (d.lattice == LBM_D2Q9 && (d.limiter & LBM_LIM_POSITIVITY) &&
            (d.limiter & (LBM_LIM_MEDIAN | kLimEns)) && d.ds_form != LBM_DS_EXACT)
            return fail(nullptr, LBM_EINVAL,
                        where + "the positivity rule with the median or ensemble limiters needs the exact Delta S");
        if (d.limiter & kLimEns) {
            if (!(d.ens_c >= 0.0) || !finite(d.ens_c) || !(d.ens_k > 0.0) || !finite(d.ens_k) ||
                !(d.delta_ens >= 0.0) || !finite(d.delta_ens))
                return fail(nullptr, LBM_EINVAL, where + "ensemble limiter needs finite ens_c >= 0, ens_k > 0, delta_ens >= 0");
            if ((d.limiter & LBM_LIM_ENS_RATIONAL) && !(d.ens_c > 0.0 && d.ens_k >= 0.5))
                return fail(nullptr, LBM_EINVAL, where + "rational limiter needs ens_c > 0 and ens_k >= 1/2");
        }
        if (d.trim_mode != 0 && d.trim_mode != 1) return fail(nullptr, LBM_EINVAL, where + "bad trim_mode");
        if (d.median_mode != 0 && d.median_mode != 1) return fail(nullptr, LBM_EINVAL, where + "bad median_mode");
        if (d.nx < 1 || d.ny < 1) return fail(nullptr, LBM_EINVAL, where + "nx, ny must be >= 1");
        if ((long long)d.nx * d.ny * q_of(d.lattice) >= (1LL << 31))
            return fail(nullptr, LBM_EINVAL, where + "grid too large (Q*nx*ny must be < 2^31)");
        if (d.lattice == LBM_D1Q3) {
            if (d.ny != 1) return fail(nullptr, LBM_EINVAL, where + "D1Q3 needs ny = 1");
            if (d.bc != LBM_BC_PERIODIC && d.bc != LBM_BC_TUBE_ENDS)
                return fail(nullptr, LBM_EINVAL, where + "D1Q3 supports periodic or tube ends");
            if (d.bc == LBM_BC_TUBE_ENDS && d.nx < 2) return fail(nullptr, LBM_EINVAL, where + "tube needs nx >= 2");
        } else {
            if (d.bc != LBM_BC_PERIODIC && !is_cavity(d.bc))
                return fail(nullptr, LBM_EINVAL, where + "D2Q9 supports periodic or cavity");
            if (is_cavity(d.bc) && (d.nx < 4 || d.ny < 4))
                return fail(nullptr, LBM_EINVAL, where + "cavity needs nx, ny >= 4");
        }
        if (!(d.beta >= 0.0 && d.beta <= 1.0)) return fail(nullptr, LBM_EINVAL, where + "beta must be in [0, 1]");
        if (!(d.delta_trim >= 0.0) || !finite(d.delta_trim) || !(d.delta_median >= 0.0) || !finite(d.delta_median))
            return fail(nullptr, LBM_EINVAL, where + "delta must be finite and >= 0");
        if (!(d.rho0 > 0.0) || !finite(d.rho0)) return fail(nullptr, LBM_EINVAL, where + "rho0 must be finite and > 0");
        if (!finite(d.lid_ux)) return fail(nullptr, LBM_EINVAL, where + "lid_ux not finite");
        if (d.qe == LBM_QE_ENTROPIC && is_cavity(d.bc) && std::fabs(d.lid_ux) >= 1.0)
            return fail(nullptr, LBM_EINVAL, where + "entropic f* needs |lid_ux| < 1");
        if (d.probe_x >= 0 || d.probe_y >= 0) {
            const bool in = d.probe_x >= 0 && d.probe_x < d.nx && d.probe_y >= 0 && d.probe_y < d.ny;
            const bool fluid = !is_cavity(d.bc) ||
                               (d.probe_x >= 1 && d.probe_x <= d.nx - 2 && d.probe_y >= 1 && d.probe_y <= d.ny - 2);
            if (!in || !fluid) return fail(nullptr, LBM_EINVAL, where + "probe must be a fluid node of the grid");
        }
        const size_t n = size_t(d.nx) * d.ny;
        const int dim = d.lattice == LBM_D2Q9 ? 2 : 1;
        if (d.f_init) {
            for (size_t s = 0; s < n * q_of(d.lattice); ++s)
                if (!finite(d.f_init[s])) return fail(nullptr, LBM_EINVAL, where + "f_init has non-finite values");
        } else {
            if (d.rho_init)
                for (size_t s = 0; s < n; ++s)
                    if (!(d.rho_init[s] > 0.0) || !finite(d.rho_init[s]))
                        return fail(nullptr, LBM_EINVAL, where + "rho_init must be finite and > 0");
            if (d.u_init)
                for (size_t s = 0; s < n * dim; ++s) {
                    if (!finite(d.u_init[s])) return fail(nullptr, LBM_EINVAL, where + "u_init not finite");
                    if (d.qe == LBM_QE_ENTROPIC && std::fabs(d.u_init[s]) >= 1.0)
                        return fail(nullptr, LBM_EINVAL, where + "entropic f* needs |u| < 1");
                }
        }
    }
    if ((run->flags & LBM_RUN_ADAPTIVE) && (run->tile_x == kFusedWidth || !fusable(doms, nd)))
        return fail(nullptr, LBM_EINVAL,
                    "LBM_RUN_ADAPTIVE needs D2Q9 LBGK domains with the median filter and no "
                    "ensemble-dependent limiter, and tile_x other than 248");
    return LBM_OK;
}

// Per-domain arrays besides the populations, the record planes and the
// probe ring, placed from `off`: stats, the Delta S' plane (median filter or
// a limiter that needs the whole domain), the applied factor (D1Q3 ensemble
// pass), the ensemble values, the selection state.
size_t plan_extras(DomainHost& h, int storage, size_t off)
{
    h.off_stats = off;
    off = align_up(off + (kNStat + 1) * sizeof(double), kAlign);
    const bool ens = deferred(h.d);
    h.dsbuf = (h.d.lattice == LBM_D2Q9 && (h.d.limiter & LBM_LIM_MEDIAN)) || ens;
    if (h.dsbuf) {
        h.off_dsbuf = off;
        off = align_up(off + h.n * (storage == LBM_F64 ? 8 : 4), kAlign);
    }
    h.phibuf = ens && h.d.lattice == LBM_D1Q3;
    if (h.phibuf) {
        h.off_phibuf = off;
        off = align_up(off + h.n * (storage == LBM_F64 ? 8 : 4), kAlign);
    }
    h.off_ens = off;
    off = align_up(off + kNEns * sizeof(double), kAlign);
    if ((h.d.limiter & kLimEnsBudget) || is_topk(h.d)) {
        h.off_bstate = off;
        off = align_up(off + sizeof(BudgetState), kAlign);
        h.off_bhist = off;
        off = align_up(off + kBudgetBuckets * sizeof(BudgetBucket), kAlign);
    }
    return off;
}

// Device layout for the given descriptors.  The tile arrays are sized for the
// smallest tile shape so any autotuned shape fits.
void plan(std::vector<DomainHost>& dh, const lbm_domain_desc* doms, int32_t nd, const lbm_run_desc* run, Layout& L)
{
    const int storage = run->storage;
    const size_t es = elem_size(storage);
    const unsigned flags = run->flags;
    const int cap = run->probe_capacity > 0 ? run->probe_capacity : 4096;
    const bool adaptive = adaptive_run(doms, nd, run);
    size_t off = 0;
    L.max_tiles = 0;
    L.nrows = 0;
    L.ngroups = 0;
    L.max_n = 0;
    dh.resize(nd);
    for (int k = 0; k < nd; ++k) {
        DomainHost& h = dh[k];
        h.d = doms[k];
        h.d.rho_init = h.d.u_init = h.d.f_init = nullptr;
        h.q = q_of(h.d.lattice);
        h.n = size_t(h.d.nx) * h.d.ny;
        h.plane = (long long)align_up(h.n, 64);
        h.shift = storage == LBM_F64 ? 0.0 : h.d.rho0;
        for (int b = 0; b < 2; ++b) {
            h.off_buf[b] = off;
            off = align_up(off + size_t(h.q) * h.plane * es, kAlign);
        }
        if (flags & LBM_RUN_RECORD) {
            h.off_mask = off;
            off = align_up(off + h.n, kAlign);
            h.off_ds = off;
            off = align_up(off + h.n * 8, kAlign);
        }
        if (h.d.probe_x >= 0) {
            h.off_probe = off;
            off = align_up(off + size_t(cap) * 2 * sizeof(float), kAlign);
        }
        off = plan_extras(h, storage, off);
        // the tile table is sized for the smallest height the tuner may pick
        const int min_h = run->tile_h > 0 ? run->tile_h : kMinTuneH;
        int tiles = tiles_of(h.d.lattice, h.d.nx, h.d.ny, min_h);
        if (h.d.lattice == LBM_D2Q9 && run->tile_x == kFusedWidth)
            tiles = std::max(tiles, fused_tiles_of(h.d.nx, h.d.ny, run->tile_h > 0 ? run->tile_h : kMinFusedH));
        // adaptive: the fused tiles (any tuned height) share the partial slots
        if (h.d.lattice == LBM_D2Q9 && adaptive) tiles = std::max(tiles, fused_tiles_of(h.d.nx, h.d.ny, kMinFusedH));
        L.max_tiles += tiles;
        L.ngroups += tiles_of(h.d.lattice, h.d.nx, h.d.ny, kMaxTileH);
        if (h.d.lattice == LBM_D2Q9) L.nrows += strips_of(h.d.nx) * h.d.ny;
        L.max_n = std::max(L.max_n, h.n);
    }
    L.off_dom = off;
    off = align_up(off + nd * sizeof(DomainDev), kAlign);
    L.off_tiles = off;
    off = align_up(off + L.max_tiles * sizeof(Tile), kAlign);
    if (adaptive) {
        L.off_dom_alt = off;
        off = align_up(off + nd * sizeof(DomainDev), kAlign);
        L.off_tiles_alt = off;
        off = align_up(off + L.max_tiles * sizeof(Tile), kAlign);
        L.off_adapt = off;
        off = align_up(off + sizeof(double), kAlign);
    }
    L.off_groups = off;
    off = align_up(off + L.ngroups * sizeof(Tile), kAlign);
    L.off_partials = off;
    off = align_up(off + size_t(4) * L.max_tiles * kNStat * sizeof(double), kAlign);
    L.off_rows = off;
    off = align_up(off + size_t(L.nrows) * sizeof(RowBlock), kAlign);
    L.off_rowpart = off;
    off = align_up(off + size_t(L.nrows) * kNStat * sizeof(double), kAlign);
    L.off_counter = off;
    off = align_up(off + 2 * sizeof(long long), kAlign);
    L.off_stage = off;
    off = align_up(off + size_t(q_of(doms[0].lattice) + 3) * L.max_n * sizeof(double), kAlign);
    L.total = off;
}

// Tiles in spatial order: domain, row block, column block.  A D2Q9 tile is
// kThreads consecutive columns by `th` rows (one thread per column walking
// the rows).  The kernels map workgroups to runs of this order XCD by XCD
// (xcd_spatial), so vertically adjacent tiles, which share halo rows, run
// on the same L2, and per-domain partial ranges stay contiguous.
std::vector<Tile> build_tiles(lbm_ctx* ctx, int th, bool fused)
{
    std::vector<Tile> spatial;
    for (size_t k = 0; k < ctx->dom.size(); ++k) {
        DomainHost& h = ctx->dom[k];
        h.tile_first = int(spatial.size());
        const int nx = h.d.nx, ny = h.d.ny;
        const int count = fused ? fused_tiles_of(nx, ny, th) : tiles_of(ctx->lattice, nx, ny, th);
        for (int i = 0; i < count; ++i)
            spatial.push_back(fused ? fused_tile_entry(int(k), nx, ny, th, i)
                                    : (ctx->lattice == LBM_D2Q9 ? tile_entry2d(int(k), nx, ny, th, i)
                                                                : tile_entry1d(int(k), nx, i)));
        h.tile_count = count;
    }
    return spatial;
}

// D2Q9 row blocks, row-major within each domain: the collision kernel runs
// one workgroup per block in this order.  Every domain row has one collision
// partial per 256-column strip (row_first + y strips + strip), whatever the
// blocks; `narrow` gives narrow domains blocks of several rows.
void build_rows(lbm_ctx* ctx, int narrow)
{
    ctx->rows_host.clear();
    ctx->narrow = narrow;
    if (ctx->lattice != LBM_D2Q9) return;
    int part = 0;
    for (size_t k = 0; k < ctx->dom.size(); ++k) {
        DomainHost& h = ctx->dom[k];
        h.row_first = part;
        h.row_count = strips_of(h.d.nx) * h.d.ny;
        part += h.row_count;
        const int width = seg_width(h.d.nx, narrow);
        const int nb = blocks_of(h.d.nx, h.d.ny, width);
        for (int i = 0; i < nb; ++i) ctx->rows_host.push_back(block_entry2d(int(k), h.d.nx, h.d.ny, width, i));
    }
}

// The groups of kMaxTileH rows whose collision partials are summed together
// for the stats and E(Delta S'), fixed so that those sums do not depend on
// the tile height in use (D1Q3: its tiles).
void build_groups(lbm_ctx* ctx)
{
    ctx->groups_host.clear();
    for (size_t k = 0; k < ctx->dom.size(); ++k) {
        DomainHost& h = ctx->dom[k];
        h.group_first = int(ctx->groups_host.size());
        const int nx = h.d.nx, ny = h.d.ny;
        const int count = tiles_of(ctx->lattice, nx, ny, kMaxTileH);
        for (int i = 0; i < count; ++i)
            ctx->groups_host.push_back(ctx->lattice == LBM_D2Q9 ? tile_entry2d(int(k), nx, ny, kMaxTileH, i)
                                                                : tile_entry1d(int(k), nx, i));
        h.group_count = count;
    }
}

int upload_rows(lbm_ctx* ctx)
{
    if (ctx->rows_host.empty()) return LBM_OK;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_rows(), ctx->rows_host.data(), ctx->rows_host.size() * sizeof(RowBlock),
                                hipMemcpyHostToDevice, ctx->stream));
    return LBM_OK;
}

// Device view of one domain: device pointers into `base` at the host
// layout's offsets; the population buffers are b0 and b1.
DomainDev make_dev(const DomainHost& h, char* base, void* b0, void* b1, int probe_cap, unsigned flags)
{
    DomainDev d{};
    d.buf[0] = b0;
    d.buf[1] = b1;
    d.plane = h.plane;
    d.nx = h.d.nx;
    d.ny = h.d.ny;
    d.c = 2.0 * h.d.beta - 1.0;
    d.shift = h.shift;
    d.delta_trim = h.d.delta_trim;
    d.delta_median = h.d.delta_median;
    d.rho0 = h.d.rho0;
    d.lid_ux = h.d.lid_ux;
    d.trim_mode = h.d.trim_mode;
    d.median_mode = h.d.median_mode;
    d.probe_x = h.d.probe_x >= 0 ? h.d.probe_x : -1;
    d.probe_y = h.d.probe_x >= 0 ? h.d.probe_y : -1;
    d.probe_cap = probe_cap;
    d.probe = h.d.probe_x >= 0 ? reinterpret_cast<float*>(base + h.off_probe) : nullptr;
    d.mask = (flags & LBM_RUN_RECORD) ? reinterpret_cast<unsigned char*>(base + h.off_mask) : nullptr;
    d.dS = (flags & LBM_RUN_RECORD) ? reinterpret_cast<double*>(base + h.off_ds) : nullptr;
    d.tile_first = h.tile_first;
    d.tile_count = h.tile_count;
    d.strips = strips_of(h.d.nx);
    d.row_first = h.row_first;
    d.row_count = h.row_count;
    d.group_first = h.group_first;
    d.group_count = h.group_count;
    d.stats = reinterpret_cast<double*>(base + h.off_stats);
    d.dsbuf = h.dsbuf ? base + h.off_dsbuf : nullptr;
    d.phibuf = h.phibuf ? base + h.off_phibuf : nullptr;
    d.ens = reinterpret_cast<double*>(base + h.off_ens);
    d.ens_c = h.d.ens_c;
    d.ens_k = h.d.ens_k;
    d.delta_ens = h.d.delta_ens;
    d.diffusive = h.d.bc == LBM_BC_CAVITY_DIFFUSIVE ? 1 : 0;
    d.collision = h.d.collision;
    d.homothety = h.d.homothety;
    d.top_k = h.d.top_k;
    d.limiter = device_limiter(h.d);
    const bool budget = (h.d.limiter & kLimEnsBudget) || is_topk(h.d);
    d.bstate = budget ? reinterpret_cast<BudgetState*>(base + h.off_bstate) : nullptr;
    d.bhist = budget ? reinterpret_cast<BudgetBucket*>(base + h.off_bhist) : nullptr;
    return d;
}

int upload_domains(lbm_ctx* ctx)
{
    std::vector<DomainDev>& dd = ctx->act.dom_host;
    dd.assign(ctx->dom.size(), DomainDev{});
    for (size_t k = 0; k < ctx->dom.size(); ++k) {
        const DomainHost& h = ctx->dom[k];
        dd[k] = make_dev(h, ctx->ws, ctx->ws + h.off_buf[0], ctx->ws + h.off_buf[1], ctx->probe_cap, ctx->flags);
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_dom(), dd.data(), dd.size() * sizeof(DomainDev), hipMemcpyHostToDevice,
                                ctx->stream));
    return LBM_OK;
}

int set_tiles(lbm_ctx* ctx, int th, bool fused = false)
{
    lbm_ctx::Slot& sl = ctx->act;
    sl.tiles_host = build_tiles(ctx, th, fused);
    sl.fused = fused;
    if (int(sl.tiles_host.size()) > ctx->lay.max_tiles) return fail(ctx, LBM_EINVAL, "tile table overflow");
    sl.ntiles = int(sl.tiles_host.size());
    sl.th = th;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_tiles(), sl.tiles_host.data(), sl.tiles_host.size() * sizeof(Tile),
                                hipMemcpyHostToDevice, ctx->stream));
    int rc = upload_domains(ctx);
    if (rc) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

StepArgs step_args(const lbm_ctx* ctx, int parity)
{
    StepArgs a;
    a.dom = ctx->d_dom();
    a.tiles = ctx->d_tiles();
    a.ntiles = ctx->act.ntiles;
    a.ndomains = int(ctx->dom.size());
    a.median_pass = (ctx->median_pass || ctx->ens_pass) ? 1 : 0;
    a.ens_pass = ctx->ens_pass ? 1 : 0;
    a.budget = ctx->budget ? 1 : 0;
    a.fused = ctx->act.fused ? 1 : 0;
    a.rows = ctx->d_rows();
    a.nrows = int(ctx->rows_host.size());
    a.groups = ctx->d_groups();
    a.ngroups = ctx->lay.ngroups;
    a.pstride = ctx->lay.max_tiles;
    a.rowpart = ctx->d_rowpart();
    a.parity = parity;
    a.flags = ctx->flags & (LBM_RUN_RECORD | LBM_RUN_ENTROPY);
    a.partials = ctx->d_partials();
    a.counter = ctx->d_counter();
    return a;
}

// The kernels one step launches (what a context or a static call runs).
struct StepKind {
    int storage, lattice, qe, ds, bc;
    bool elbm, median_pass, ens_pass, budget, fused = false;
};

// One step of every domain of `a`.  With `ev` (three events) the launches
// are bracketed for per-kernel timing: ev[0] | collision | ev[1] | rest | ev[2].
hipError_t launch_step(const StepKind& k, const StepArgs& a, hipStream_t s, hipEvent_t* ev = nullptr)
{
    hipError_t e = hipSuccess;
    if (ev) e = hipEventRecord(ev[0], s);
    if (k.fused) {
        // one kernel: collision and median filter together
        if (e == hipSuccess) e = launch_step2d(k.storage, k.qe, k.ds, k.bc, a, 3, s);
        if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
        return e;
    }
    if (e == hipSuccess) {
        if (k.lattice == LBM_D2Q9)
            e = launch_step2d(k.storage, k.qe, k.ds, k.bc, a, k.elbm ? 2 : 0, s);
        else
            e = launch_step1d(k.storage, k.qe, k.ds, k.bc, a, k.elbm ? 2 : 0, s);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
    // ensemble limiters: E(Delta S') of this step first (Sec. 3.3, 3.4)
    if (e == hipSuccess && k.ens_pass) e = launch_ens_prepare(a, s);
    if (e == hipSuccess && k.budget) e = launch_budget(k.storage, k.bc, a, s);
    if (e == hipSuccess && (k.median_pass || k.ens_pass)) {
        if (k.lattice == LBM_D2Q9)
            e = launch_step2d(k.storage, k.qe, k.ds, k.bc, a, 1, s);
        else
            e = launch_step1d(k.storage, k.qe, k.ds, k.bc, a, 1, s);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
    return e;
}

StepKind step_kind(const lbm_ctx* ctx)
{
    return StepKind{ctx->storage, ctx->lattice, ctx->qe, ctx->ds, ctx->bc, ctx->elbm, ctx->median_pass,
                    ctx->ens_pass, ctx->budget, ctx->act.fused};
}

int launch_one(lbm_ctx* ctx, int parity, hipEvent_t* ev = nullptr, unsigned extra_flags = 0)
{
    StepArgs a = step_args(ctx, parity);
    a.flags |= extra_flags;
    const hipError_t e = launch_step(step_kind(ctx), a, ctx->stream, ev);
    if (e != hipSuccess) return fail(ctx, LBM_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    return LBM_OK;
}

// counter[p] holds the index of the next step when that step reads buffer p
int reset_counters(lbm_ctx* ctx)
{
    long long c[2];
    c[ctx->steps_done % 2] = ctx->steps_done;
    c[1 - ctx->steps_done % 2] = 0;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_counter(), c, sizeof(c), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

void drop_graphs(lbm_ctx* ctx)
{
    for (lbm_ctx::Slot* sl : {&ctx->act, &ctx->alt})
        for (auto& gs : sl->graphs) {
            for (auto& g : gs)
                if (g.exec) (void)hipGraphExecDestroy(g.exec);
            gs.clear();
        }
}

// ---- autotuner ---------------------------------------------------------------
// Three shape choices change the speed of a D2Q9 step: the row blocks of the
// collision kernel (256 columns per row, or several rows of a narrow domain
// per workgroup), the height of the tiles the second pass walks, and, for
// domains with the median filter and no ensemble-dependent limiter, the fused
// step (collision and median filter in one pass over tiles of kFusedWidth
// columns) in place of the two kernels, taken when the run asks for it
// (tile_x = kFusedWidth; the tuner then picks its tile height).  The fused
// step costs the same whatever the filter does; the two kernels cost less
// while few nodes move and more when many do (each moved node's stored state
// is read and written again), which the steps timed at creation, from a
// state where nothing has moved yet, cannot show.  Row blocks and tile heights change
// nothing the step computes (the stats partials are grouped by fixed 64-row
// groups, so E(Delta S') and every field come out the same; only the FP64
// sums that the second pass adds to may differ in the last bits).  The fused
// step forms a moved node's state f* - phi c d once, with phi the smallest
// factor, where the two kernels rescale the stored trimmed state: the masks
// and every decision are the same, a moved node's populations agree to
// rounding.  lbm_create times the candidate shapes on the live state with HIP
// events and keeps the fastest; a process-wide cache keyed by the descriptors
// gives the same choice to every later context of the same problem.

struct Shape {
    int narrow, th;
    bool fused;
};

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tune_cache;   // key -> chosen shape

// the problem and the shapes the run allows (a run that fixes tile_x or
// tile_h has its own entry)
std::string tune_key(const lbm_ctx* ctx, const lbm_run_desc* run)
{
    std::string k = std::to_string(run->tile_x) + "/" + std::to_string(run->tile_h) + "/" +
                    std::to_string(ctx->device) + "/" + std::to_string(ctx->storage) + "/" + std::to_string(ctx->qe) +
                    "/" + std::to_string(ctx->ds) + "/" + std::to_string(ctx->bc) + "/" + std::to_string(ctx->elbm) +
                    "/" + std::to_string(ctx->flags & (LBM_RUN_RECORD | LBM_RUN_ENTROPY));
    for (const auto& h : ctx->dom)
        k += ";" + std::to_string(h.d.nx) + "x" + std::to_string(h.d.ny) + ":" + std::to_string(h.d.limiter) + ":" +
             std::to_string(h.d.median_mode) + ":" + std::to_string(h.d.homothety) + ":" +
             std::to_string(h.d.top_k > 0) + ":" + std::to_string(h.d.bc);
    return k;
}

int apply_shape(lbm_ctx* ctx, const Shape& sh)
{
    build_rows(ctx, sh.narrow);
    int rc = upload_rows(ctx);
    return rc ? rc : set_tiles(ctx, sh.th, sh.fused);
}

// average milliseconds of `n` steps that all read buffer 0 (the initial state
// stays intact; buffer 1 and the scratch arrays are overwritten)
int time_shape(lbm_ctx* ctx, int n, double& ms, unsigned extra_flags = 0)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = LBM_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(ctx, LBM_EDEVICE, "event");
    if (!rc) rc = launch_one(ctx, 0, nullptr, extra_flags);   // untimed: first launch of this shape
    if (!rc && hipEventRecord(e0, ctx->stream) != hipSuccess) rc = fail(ctx, LBM_EDEVICE, "event record");
    for (int k = 0; k < n && !rc; ++k) rc = launch_one(ctx, 0, nullptr, extra_flags);
    float t = 0;
    if (!rc && (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = fail(ctx, LBM_EDEVICE, "event timing");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ms = double(t) / n;
    return rc;
}

// fused_alt: the fused form of an adaptive run (its tile height only; the
// row blocks of the two-kernel form stay as tuned)
int autotune(lbm_ctx* ctx, const lbm_run_desc* run, bool fused_alt = false)
{
    bool any_narrow = false;
    for (const auto& h : ctx->dom) any_narrow = any_narrow || seg_width(h.d.nx, 1) < kThreads;
    std::vector<int> widths;
    if (run->tile_x == kThreads || !any_narrow) widths = {0};
    else if (run->tile_x == kWave) widths = {1};
    else widths = {1, 0};
    const bool second = ctx->median_pass || ctx->ens_pass;
    std::vector<int> heights;
    if (run->tile_h > 0) heights = {run->tile_h};
    else if (second) heights = {16, 32, 64};
    else heights = {kMaxTileH};
    std::vector<Shape> cand;
    if (fused_alt) {
        for (int th : {kMinFusedH, 8, 16, 32, 64}) cand.push_back({ctx->narrow, th, true});
        if (ctx->flags & LBM_RUN_NO_TUNE) return apply_shape(ctx, {ctx->narrow, 8, true});
    } else if (run->tile_x != kFusedWidth)
        for (int w : widths)
            for (int th : heights) cand.push_back({w, th, false});
    // the fused step only when asked for: at creation no node has moved yet,
    // and the tuner cannot see how much of the flow the filter will move
    if (!fused_alt && ctx->fuse_ok && run->tile_x == kFusedWidth) {
        const std::vector<int> fh = run->tile_h > 0 ? std::vector<int>{run->tile_h}
                                                    : std::vector<int>{kMinFusedH, 8, 16, 32, 64};
        for (int th : fh) cand.push_back({widths[0], th, true});
    }
    ctx->tuned = 0;
    if (cand.size() == 1) return apply_shape(ctx, cand[0]);
    if (ctx->flags & LBM_RUN_NO_TUNE) {
        // narrow row blocks where a domain allows them, tile_h or 64 rows
        // for the second pass; the fused step only when asked for
        if (run->tile_x == kFusedWidth) return apply_shape(ctx, {widths[0], run->tile_h > 0 ? run->tile_h : 64, true});
        return apply_shape(ctx, {widths[0], heights.back(), false});
    }
    const std::string key = tune_key(ctx, run) + (fused_alt ? "/fused form" : "");
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            ctx->tuned = 1;
            return apply_shape(ctx, it->second);
        }
    }
    // Warm the part up on the first candidate, then time every candidate in
    // two rounds (the second in reverse order) and keep each one's best.  How
    // much of the second pass has work depends on the flow (at the start
    // often no tile has a candidate); a candidate is scored by the sum of a
    // step as it stands and a step whose second pass walks every tile (the
    // fused step does its median work on every node either way).
    int rc = apply_shape(ctx, cand[0]);
    double ms = 0;
    if (!rc) rc = time_shape(ctx, 8, ms);
    std::vector<double> best(cand.size(), 1e30), best_all(cand.size(), second ? 1e30 : 0.0);
    for (int round = 0; round < 2 && !rc; ++round)
        for (size_t j = 0; j < cand.size() && !rc; ++j) {
            const size_t c = round ? cand.size() - 1 - j : j;
            rc = apply_shape(ctx, cand[c]);
            if (!rc) rc = time_shape(ctx, 3, ms);
            if (!rc) best[c] = std::min(best[c], ms);
            if (!rc && second) rc = time_shape(ctx, 3, ms, kFlagAllTiles);
            if (!rc && second) best_all[c] = std::min(best_all[c], ms);
        }
    if (rc) return rc;
    size_t pick = 0;
    for (size_t c = 1; c < cand.size(); ++c)
        if (best[c] + best_all[c] < best[pick] + best_all[pick]) pick = c;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = cand[pick];
    }
    ctx->tuned = 1;
    return apply_shape(ctx, cand[pick]);
}

// Capture `len` steps starting at `parity` into one executable graph.
int capture(lbm_ctx* ctx, int parity, int64_t len)
{
    hipGraph_t g = nullptr;
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int rc = LBM_OK;
    for (int64_t k = 0; k < len && rc == LBM_OK; ++k) rc = launch_one(ctx, int((parity + k) % 2));
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(ctx, LBM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(ctx, LBM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    ctx->act.graphs[parity].push_back({len, x});
    return LBM_OK;
}

// Every step of lbm_step runs inside a graph: for each starting parity, one
// graph of graph_chunk steps and one of each power of two below it, so that
// any count is a few replays (e.g. 20 = 16 + 4).  Captured once, at creation,
// so that no capture happens inside a caller's timed loop.
int capture_all(lbm_ctx* ctx)
{
    std::vector<int64_t> lens{ctx->graph_chunk};
    for (int64_t l = 1; l < ctx->graph_chunk; l *= 2) lens.push_back(l);
    std::sort(lens.begin(), lens.end(), std::greater<int64_t>());
    for (int parity = 0; parity < 2; ++parity)
        for (int64_t l : lens) {
            int rc = capture(ctx, parity, l);
            if (rc) return rc;
        }
    return LBM_OK;
}

// Adaptive runs: the filtered fraction (nodes the median filter moved over
// the fluid nodes of all domains) above which the fused step takes over, and
// below which the two kernels come back.  The two kernels cost less while
// few nodes move; once the filter moves a few per mille their second pass
// reads and rewrites most sectors of the population planes again.
constexpr double kAdaptOn = 5e-3;
constexpr double kAdaptOff = 1e-3;

// At a multiple of graph_chunk steps (or the first call past one): queue the
// filtered count of the step just run for reading back without a wait, then
// choose the form of the next chunk from the count queued at the previous
// such point (which the stream has long passed).  The choice depends on the
// states at those steps only, not on how the steps were split into calls.
int adapt(lbm_ctx* ctx)
{
    if (ctx->steps_done < ctx->next_check) return LBM_OK;
    const int slot = int(ctx->adapt_points % 2);
    if (ctx->steps_done > 0) {
        const StepArgs a = step_args(ctx, 0);
        hipError_t e = launch_filtered_count(a, int((ctx->steps_done - 1) % 2), ctx->d_adapt(), ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->adapt_host + slot, ctx->d_adapt(), sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(ctx->adapt_ev[slot], ctx->stream);
        if (e != hipSuccess) return fail(ctx, LBM_EDEVICE, std::string("filtered count: ") + hipGetErrorString(e));
        ctx->adapt_pending[slot] = true;
    }
    if (ctx->adapt_pending[1 - slot]) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->adapt_ev[1 - slot]));
        ctx->adapt_pending[1 - slot] = false;
        const double frac = ctx->adapt_host[1 - slot] / std::max(ctx->fluid_total, 1.0);
        if (ctx->act.fused ? frac < kAdaptOff : frac > kAdaptOn) std::swap(ctx->act, ctx->alt);
    }
    ++ctx->adapt_points;
    const long long p = ctx->graph_chunk;
    ctx->next_check = (ctx->steps_done / p + 1) * p;
    return LBM_OK;
}

int check_domain(lbm_ctx* ctx, int32_t d)
{
    if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL context");
    if (d < 0 || d >= int(ctx->dom.size())) return fail(ctx, LBM_ERANGE, "domain index out of range");
    return LBM_OK;
}

int finalize_stats(lbm_ctx* ctx)
{
    if (ctx->steps_done == 0 || ctx->finalized_for == ctx->steps_done) return LBM_OK;
    const StepArgs a = step_args(ctx, 0);
    hipError_t e = launch_finalize(a, int((ctx->steps_done - 1) % 2), ctx->steps_done, ctx->stream);
    if (e != hipSuccess) return fail(ctx, LBM_EDEVICE, std::string("finalize: ") + hipGetErrorString(e));
    ctx->finalized_for = ctx->steps_done;
    return LBM_OK;
}

int read_stats(lbm_ctx* ctx, int32_t d, lbm_entropy_stats_t* out)
{
    int rc = finalize_stats(ctx);
    if (rc) return rc;
    const DomainHost& h = ctx->dom[d];
    double raw[kNStat + 1];
    std::memset(raw, 0, sizeof(raw));
    if (ctx->steps_done > 0) {
        HIP_TRY(ctx, hipMemcpyAsync(raw, ctx->ws + h.off_stats, sizeof(raw), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    lbm_entropy_stats_t s;
    std::memset(&s, 0, sizeof(s));
    s.struct_size = sizeof(s);
    s.step = ctx->steps_done;
    const double c = 2.0 * h.d.beta - 1.0;
    s.mass = raw[kSMass] + (ctx->steps_done > 0 ? h.shift * double(h.n) : 0.0);
    s.mom_x = raw[kSJx];
    s.mom_y = raw[kSJy];
    s.sum_dS_pre = raw[kSDpre];
    s.sum_dS_post = raw[kSDpost];
    s.max_dS = raw[kSMax];
    s.n_fluid = (int64_t)raw[kSFluid];
    s.mean_dS = s.n_fluid > 0 ? s.sum_dS_post / double(s.n_fluid) : 0.0;
    s.lbgk_production = (1.0 - c * c) * s.sum_dS_pre;
    s.limiter_production = raw[kSLim];
    s.total_entropy = (ctx->flags & LBM_RUN_ENTROPY) ? raw[kSEnt] : NAN;
    s.n_trimmed = (int64_t)raw[kSTrim];
    s.n_filtered = (int64_t)raw[kSFilt];
    s.n_nonpositive = (int64_t)raw[kSNonpos];
    s.n_nonfinite = (int64_t)raw[kSNonfin];
    s.n_ensemble = (int64_t)raw[kSEns];
    s.n_positivity = (int64_t)raw[kSPos];
    if (h.d.limiter & (LBM_LIM_ENS_THRESHOLD | LBM_LIM_ENS_BUDGET)) {
        double ev[kNEns] = {0, 0, 0, 0};
        if (ctx->steps_done > 0) {
            HIP_TRY(ctx, hipMemcpyAsync(ev, ctx->ws + h.off_ens, sizeof(ev), hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        }
        s.ens_threshold = (h.d.limiter & LBM_LIM_ENS_BUDGET) ? ev[kEBudget] : ev[kEThresh];
    }
    if (out) {
        const uint32_t keep = out->struct_size ? std::min<uint32_t>(out->struct_size, sizeof(s)) : sizeof(s);
        std::memcpy(out, &s, keep);
    }
    if (s.n_nonfinite > 0) return fail(ctx, LBM_EUNSTABLE, "non-finite moments in the last step");
    // with the exact Delta S a non-positive population leaves the entropy
    // undefined (Delta S = +inf); trimming and the positivity rule send such
    // a node to f* (or back to the positive side) in the same step, without
    // them the state stays outside the domain of the entropy
    if (s.n_nonpositive > 0 && h.d.ds_form == LBM_DS_EXACT && !(h.d.limiter & (LBM_LIM_TRIM | LBM_LIM_POSITIVITY)))
        return fail(ctx, LBM_EUNSTABLE, "non-positive populations with the exact Delta S and no limiter that resolves them");
    return LBM_OK;
}

// Layout of lbm_step_static's arrays in the static scratch array: one
// domain, tight planes (plane = nx ny), no record planes, no probe.
struct StaticLayout {
    size_t off_dom = 0, off_tiles = 0, off_rows = 0, off_partials = 0, off_rowpart = 0, off_counter = 0, total = 0;
    int ntiles = 0, nblocks = 0, nparts = 0;
};

void plan_static(const lbm_domain_desc& d, int storage, DomainHost& h, StaticLayout& L)
{
    h.d = d;
    h.d.rho_init = h.d.u_init = h.d.f_init = nullptr;
    h.q = q_of(d.lattice);
    h.n = size_t(d.nx) * d.ny;
    h.plane = (long long)h.n;
    h.shift = storage == LBM_F64 ? 0.0 : d.rho0;
    // tiles of kMaxTileH rows, which are also the stats groups; narrow row blocks
    L.ntiles = tiles_of(d.lattice, d.nx, d.ny, kMaxTileH);
    L.nblocks = d.lattice == LBM_D2Q9 ? blocks_of(d.nx, d.ny, seg_width(d.nx, 1)) : 0;
    L.nparts = d.lattice == LBM_D2Q9 ? strips_of(d.nx) * d.ny : 0;
    h.tile_first = 0;
    h.tile_count = L.ntiles;
    h.group_first = 0;
    h.group_count = L.ntiles;
    h.row_first = 0;
    h.row_count = L.nparts;
    size_t off = 0;
    L.off_dom = off;
    off = align_up(off + sizeof(DomainDev), kAlign);
    L.off_tiles = off;
    off = align_up(off + size_t(L.ntiles) * sizeof(Tile), kAlign);
    L.off_rows = off;
    off = align_up(off + size_t(L.nblocks) * sizeof(RowBlock), kAlign);
    L.off_partials = off;
    off = align_up(off + size_t(4) * L.ntiles * kNStat * sizeof(double), kAlign);
    L.off_rowpart = off;
    off = align_up(off + size_t(L.nparts) * kNStat * sizeof(double), kAlign);
    L.off_counter = off;
    off = align_up(off + 2 * sizeof(long long), kAlign);
    L.total = plan_extras(h, storage, off);
}

void release(lbm_ctx* ctx)
{
    if (!ctx) return;
    drop_graphs(ctx);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t& e : ctx->adapt_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->adapt_host) (void)hipHostFree(ctx->adapt_host);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // namespace

extern "C" {

int lbm_abi_version(void) { return LBM_ABI_VERSION; }

double lbm_beta_from_nu(double nu) { return 1.0 / (6.0 * nu + 1.0); }

const char* lbm_strerror(int code)
{
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of device memory or workspace too small";
    case LBM_EDEVICE: return "HIP device error";
    case LBM_EUNSTABLE: return "non-finite moments, or unresolved non-positive populations (unstable run)";
    case LBM_ERANGE: return "domain index out of range";
    }
    return "unknown error";
}

const char* lbm_last_error(const lbm_ctx* ctx)
{
    if (ctx && !ctx->err.empty()) return ctx->err.c_str();
    return g_err.c_str();
}

int lbm_workspace_bytes(const lbm_domain_desc* domains, int32_t n_domains, const lbm_run_desc* run, size_t* bytes)
{
    int rc = validate(domains, n_domains, run);
    if (rc) return rc;
    if (!bytes) return fail(nullptr, LBM_EINVAL, "bytes is NULL");
    std::vector<DomainHost> dh;
    Layout L;
    plan(dh, domains, n_domains, run, L);
    *bytes = L.total;
    return LBM_OK;
}

int lbm_create(const lbm_domain_desc* domains, int32_t n_domains, const lbm_run_desc* run, lbm_ctx** out)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(domains, n_domains, run);
    if (rc) return rc;
    lbm_ctx* ctx = new lbm_ctx();
    ctx->device = run->device;
    ctx->storage = run->storage;
    ctx->lattice = domains[0].lattice;
    ctx->qe = domains[0].qe;
    ctx->ds = domains[0].ds_form;
    // both cavity kinds run the cavity kernels; the wall rule is per domain
    ctx->bc = is_cavity(domains[0].bc) ? kCavity : domains[0].bc;
    ctx->elbm = domains[0].collision == LBM_COLL_ELBM;
    ctx->flags = run->flags;
    ctx->stats_every = run->stats_every;
    ctx->probe_cap = run->probe_capacity > 0 ? run->probe_capacity : 4096;
    ctx->graph_chunk = run->graph_chunk > 0 ? run->graph_chunk : 64;
    plan(ctx->dom, domains, n_domains, run, ctx->lay);
    for (const auto& h : ctx->dom) {
        ctx->median_pass = ctx->median_pass || (h.d.lattice == LBM_D2Q9 && (h.d.limiter & LBM_LIM_MEDIAN));
        ctx->ens_pass = ctx->ens_pass || deferred(h.d);
        ctx->budget = ctx->budget || (h.d.limiter & kLimEnsBudget) || is_topk(h.d);
    }
    ctx->fuse_ok = ctx->lattice == LBM_D2Q9 && !ctx->elbm && ctx->median_pass && !ctx->ens_pass;

    auto bail = [&](int code) {
        release(ctx);
        return code;
    };
    if (run->tile_x == kFusedWidth && !ctx->fuse_ok)
        return bail(fail(nullptr, LBM_EINVAL,
                         "tile_x = 248 (fused step) needs D2Q9 LBGK domains with the median filter and no "
                         "ensemble-dependent limiter"));
    ctx->adaptive = adaptive_run(domains, n_domains, run);
    ctx->act.off_dom = ctx->lay.off_dom;
    ctx->act.off_tiles = ctx->lay.off_tiles;
    ctx->alt.off_dom = ctx->lay.off_dom_alt;
    ctx->alt.off_tiles = ctx->lay.off_tiles_alt;
    for (const auto& h : ctx->dom)
        ctx->fluid_total += is_cavity(h.d.bc) ? double(h.d.nx - 2) * double(h.d.ny - 2) : double(h.n);
    hipError_t e = hipSetDevice(run->device);
    if (e != hipSuccess) return bail(fail(nullptr, LBM_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e)));
    if (run->stream) {
        ctx->stream = static_cast<hipStream_t>(run->stream);
    } else {
        e = hipStreamCreate(&ctx->stream);
        if (e != hipSuccess)
            return bail(fail(nullptr, LBM_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e)));
        ctx->own_stream = true;
    }
    if (run->workspace) {
        if (run->workspace_bytes < ctx->lay.total)
            return bail(fail(nullptr, LBM_ENOMEM, "workspace smaller than lbm_workspace_bytes()"));
        if (reinterpret_cast<uintptr_t>(run->workspace) % kAlign)
            return bail(fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned"));
        ctx->ws = static_cast<char*>(run->workspace);
    } else {
        e = hipMalloc(reinterpret_cast<void**>(&ctx->ws), ctx->lay.total);
        if (e != hipSuccess) {
            ctx->ws = nullptr;
            return bail(fail(nullptr, LBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)));
        }
        ctx->own_ws = true;
    }

    // budget histograms start zero; every selection level leaves them zero
    for (const auto& h : ctx->dom)
        if ((h.d.limiter & kLimEnsBudget) || is_topk(h.d)) {
            e = hipMemsetAsync(ctx->ws + h.off_bhist, 0, kBudgetBuckets * sizeof(BudgetBucket), ctx->stream);
            if (e != hipSuccess)
                return bail(fail(nullptr, LBM_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e)));
        }

    // initial state f(x, 0) in FP64, converted into buffer 0
    double* stage = ctx->d_stage();
    for (int k = 0; k < n_domains; ++k) {
        DomainHost& h = ctx->dom[k];
        const lbm_domain_desc& d = domains[k];
        const size_t n = h.n;
        const int dim = d.lattice == LBM_D2Q9 ? 2 : 1;
        double* f = stage;
        if (d.f_init) {
            e = hipMemcpyAsync(f, d.f_init, n * h.q * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
        } else {
            double* rho = stage + size_t(h.q) * ctx->lay.max_n;
            double* u = rho + ctx->lay.max_n;
            std::vector<double> r(n, d.rho0), uu(n * dim, 0.0);
            if (d.rho_init) std::memcpy(r.data(), d.rho_init, n * sizeof(double));
            if (d.u_init) std::memcpy(uu.data(), d.u_init, n * dim * sizeof(double));
            e = hipMemcpyAsync(rho, r.data(), n * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(u, uu.data(), n * dim * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess) e = launch_init_f(d.lattice, d.qe, rho, u, f, d.nx, d.ny, ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        }
        if (e == hipSuccess)
            e = launch_scatter(ctx->storage, d.lattice, d.bc, f, ctx->ws + h.off_buf[0], h.plane, d.nx, d.ny, h.shift,
                               ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return bail(fail(nullptr, LBM_EDEVICE, std::string("init: ") + hipGetErrorString(e)));
    }
    build_groups(ctx);
    if (int(ctx->groups_host.size()) != ctx->lay.ngroups)
        return bail(fail(nullptr, LBM_EINVAL, "group table size mismatch"));
    e = hipMemcpyAsync(ctx->d_groups(), ctx->groups_host.data(), ctx->groups_host.size() * sizeof(Tile),
                       hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return bail(fail(nullptr, LBM_EDEVICE, std::string("groups: ") + hipGetErrorString(e)));
    // the tuner runs steps: the step counters must hold valid indices first
    rc = reset_counters(ctx);
    if (!rc) rc = ctx->lattice == LBM_D2Q9 ? autotune(ctx, run) : apply_shape(ctx, Shape{0, 1, false});
    if (!rc && ctx->adaptive) {
        // the fused form in the second set of tables; the two kernels run first
        std::swap(ctx->act, ctx->alt);
        rc = autotune(ctx, run, true);
        std::swap(ctx->act, ctx->alt);
        if (!rc && hipHostMalloc(reinterpret_cast<void**>(&ctx->adapt_host), 2 * sizeof(double)) != hipSuccess) {
            ctx->adapt_host = nullptr;
            rc = fail(ctx, LBM_ENOMEM, "hipHostMalloc");
        }
        for (hipEvent_t& ev : ctx->adapt_ev)
            if (!rc && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                ev = nullptr;
                rc = fail(ctx, LBM_EDEVICE, "hipEventCreate");
            }
    }
    if (rc) {
        g_err = ctx->err;
        return bail(rc);
    }
    // clean counters and stats after tuning launches
    rc = reset_counters(ctx);
    for (auto& h : ctx->dom)
        if (!rc && hipMemsetAsync(ctx->ws + h.off_stats, 0, (kNStat + 1) * sizeof(double), ctx->stream) != hipSuccess)
            rc = fail(ctx, LBM_EDEVICE, "hipMemsetAsync stats");
    if (!rc && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = fail(ctx, LBM_EDEVICE, "sync after create");
    if (!rc && !(ctx->flags & LBM_RUN_NO_GRAPH)) rc = capture_all(ctx);
    if (!rc && ctx->adaptive && !(ctx->flags & LBM_RUN_NO_GRAPH)) {
        std::swap(ctx->act, ctx->alt);
        rc = capture_all(ctx);
        std::swap(ctx->act, ctx->alt);
    }
    if (rc) {
        g_err = ctx->err;
        return bail(rc);
    }
    *out = ctx;
    return LBM_OK;
}

int lbm_step(lbm_ctx* ctx, int64_t n_steps)
{
    if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL context");
    if (n_steps < 0) return fail(ctx, LBM_EINVAL, "n_steps < 0");
    int64_t since_check = 0;
    while (n_steps > 0) {
        int rc;
        if (ctx->adaptive && (rc = adapt(ctx))) return rc;
        int64_t done = 0;
        const int parity = int(ctx->steps_done % 2);
        // the longest captured sequence that fits before the next stats point
        // (and, adaptive, before the next choice of the form)
        int64_t limit = n_steps;
        if (ctx->stats_every > 0) limit = std::min<int64_t>(limit, ctx->stats_every - since_check);
        if (ctx->adaptive) limit = std::min<int64_t>(limit, ctx->next_check - ctx->steps_done);
        for (const auto& g : ctx->act.graphs[parity])
            if (g.len <= limit) {
                HIP_TRY(ctx, hipGraphLaunch(g.exec, ctx->stream));
                done = g.len;
                break;
            }
        if (done == 0) {
            if ((rc = launch_one(ctx, parity))) return rc;
            done = 1;
        }
        ctx->steps_done += done;
        n_steps -= done;
        since_check += done;
        if (ctx->stats_every > 0 && (since_check >= ctx->stats_every || n_steps == 0)) {
            since_check = 0;
            for (size_t d = 0; d < ctx->dom.size(); ++d) {
                lbm_entropy_stats_t s;
                s.struct_size = sizeof(s);
                if ((rc = read_stats(ctx, int32_t(d), &s))) return rc;
            }
        }
    }
    return LBM_OK;
}

int lbm_synchronize(lbm_ctx* ctx)
{
    if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL context");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

int lbm_entropy_stats(lbm_ctx* ctx, int32_t domain, lbm_entropy_stats_t* out)
{
    int rc = check_domain(ctx, domain);
    if (rc) return rc;
    if (!out) return fail(ctx, LBM_EINVAL, "out is NULL");
    return read_stats(ctx, domain, out);
}

static int gather_state(lbm_ctx* ctx, int32_t d, double* f, double* rho, double* u)
{
    const DomainHost& h = ctx->dom[d];
    const size_t n = h.n;
    const int dim = h.d.lattice == LBM_D2Q9 ? 2 : 1;
    double* sf = ctx->d_stage();
    double* sr = sf + size_t(h.q) * ctx->lay.max_n;
    double* su = sr + ctx->lay.max_n;
    const int parity = int(ctx->steps_done % 2);
    hipError_t e = launch_gather(ctx->storage, h.d.lattice, h.d.bc, ctx->ws + h.off_buf[parity], h.plane, sf, h.d.nx,
                                 h.d.ny, h.shift, f != nullptr, rho ? sr : nullptr, u ? su : nullptr, ctx->stream);
    if (e != hipSuccess) return fail(ctx, LBM_EDEVICE, std::string("gather: ") + hipGetErrorString(e));
    if (f) HIP_TRY(ctx, hipMemcpyAsync(f, sf, n * h.q * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (rho) HIP_TRY(ctx, hipMemcpyAsync(rho, sr, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (u) HIP_TRY(ctx, hipMemcpyAsync(u, su, n * dim * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

int lbm_moments(lbm_ctx* ctx, int32_t domain, double* rho, double* u)
{
    int rc = check_domain(ctx, domain);
    if (rc) return rc;
    if (!rho && !u) return LBM_OK;
    return gather_state(ctx, domain, nullptr, rho, u);
}

int lbm_get_populations(lbm_ctx* ctx, int32_t domain, double* f)
{
    int rc = check_domain(ctx, domain);
    if (rc) return rc;
    if (!f) return fail(ctx, LBM_EINVAL, "f is NULL");
    return gather_state(ctx, domain, f, nullptr, nullptr);
}

int lbm_set_populations(lbm_ctx* ctx, int32_t domain, const double* f)
{
    int rc = check_domain(ctx, domain);
    if (rc) return rc;
    if (!f) return fail(ctx, LBM_EINVAL, "f is NULL");
    const DomainHost& h = ctx->dom[domain];
    for (size_t s = 0; s < h.n * h.q; ++s)
        if (!std::isfinite(f[s])) return fail(ctx, LBM_EINVAL, "f has non-finite values");
    double* sf = ctx->d_stage();
    const int parity = int(ctx->steps_done % 2);
    HIP_TRY(ctx, hipMemcpyAsync(sf, f, h.n * h.q * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    hipError_t e = launch_scatter(ctx->storage, h.d.lattice, h.d.bc, sf, ctx->ws + h.off_buf[parity], h.plane, h.d.nx,
                                  h.d.ny, h.shift, ctx->stream);
    if (e != hipSuccess) return fail(ctx, LBM_EDEVICE, std::string("scatter: ") + hipGetErrorString(e));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

int lbm_limiter_mask(lbm_ctx* ctx, int32_t domain, uint8_t* mask, double* dS)
{
    int rc = check_domain(ctx, domain);
    if (rc) return rc;
    if (!(ctx->flags & LBM_RUN_RECORD)) return fail(ctx, LBM_EINVAL, "context was created without LBM_RUN_RECORD");
    const DomainHost& h = ctx->dom[domain];
    if (mask) HIP_TRY(ctx, hipMemcpyAsync(mask, ctx->ws + h.off_mask, h.n, hipMemcpyDeviceToHost, ctx->stream));
    if (dS) HIP_TRY(ctx, hipMemcpyAsync(dS, ctx->ws + h.off_ds, h.n * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

int lbm_probe_trace(lbm_ctx* ctx, int32_t domain, float* uv, int64_t max_samples, int64_t* n_written)
{
    int rc = check_domain(ctx, domain);
    if (rc) return rc;
    if (!n_written || (max_samples > 0 && !uv) || max_samples < 0) return fail(ctx, LBM_EINVAL, "bad probe buffers");
    *n_written = 0;
    const DomainHost& h = ctx->dom[domain];
    if (h.d.probe_x < 0) return fail(ctx, LBM_EINVAL, "domain has no probe");
    const int64_t cap = ctx->probe_cap;
    const int64_t avail = std::min<int64_t>(ctx->steps_done, cap);
    const int64_t take = std::min<int64_t>(avail, max_samples);
    if (take == 0) return LBM_OK;
    std::vector<float> ring(size_t(cap) * 2);
    HIP_TRY(ctx, hipMemcpyAsync(ring.data(), ctx->ws + h.off_probe, ring.size() * sizeof(float), hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t first = ctx->steps_done - take;
    for (int64_t k = 0; k < take; ++k) {
        const int64_t slot = (first + k) % cap;
        uv[2 * k] = ring[2 * slot];
        uv[2 * k + 1] = ring[2 * slot + 1];
    }
    *n_written = take;
    return LBM_OK;
}

int lbm_tile_config(const lbm_ctx* ctx, int32_t* tile_x, int32_t* tile_y, int32_t* tile_h)
{
    if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL context");
    const bool d2 = ctx->lattice == LBM_D2Q9;
    // D2Q9: columns of the first domain's row blocks (256, or 64 / 128 for a
    // narrow domain), their rows per workgroup, and the second pass's tile
    // height; D1Q3: sites per workgroup, 1, 1
    // height; the fused step reports kFusedWidth, 1 and its tile height
    const bool fused = ctx->act.fused;
    const int width = fused ? kFusedWidth : (d2 ? seg_width(ctx->dom[0].d.nx, ctx->narrow) : k1DWidth);
    if (tile_x) *tile_x = width;
    if (tile_y) *tile_y = (d2 && !fused) ? kThreads / width : 1;
    if (tile_h) *tile_h = d2 ? ctx->act.th : 1;
    return LBM_OK;
}

int lbm_kernel_times(lbm_ctx* ctx, int64_t n_steps, double* ms)
{
    if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL context");
    if (!ms || n_steps < 1 || n_steps > 4096) return fail(ctx, LBM_EINVAL, "need 1 <= n_steps <= 4096 and ms");
    std::vector<hipEvent_t> ev(size_t(3 * n_steps), nullptr);
    int rc = LBM_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            rc = fail(ctx, LBM_EDEVICE, "hipEventCreate failed");
            break;
        }
    for (int64_t k = 0; k < n_steps && rc == LBM_OK; ++k) {
        rc = launch_one(ctx, int(ctx->steps_done % 2), &ev[size_t(3 * k)]);
        if (rc == LBM_OK) ++ctx->steps_done;
    }
    double t[2] = {0, 0};
    if (rc == LBM_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = fail(ctx, LBM_EDEVICE, "sync failed");
    for (int64_t k = 0; k < n_steps && rc == LBM_OK; ++k)
        for (int j = 0; j < 2; ++j) {
            float x = 0;
            if (hipEventElapsedTime(&x, ev[size_t(3 * k + j)], ev[size_t(3 * k + j + 1)]) != hipSuccess) {
                rc = fail(ctx, LBM_EDEVICE, "hipEventElapsedTime failed");
                break;
            }
            t[j] += x;
        }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    ms[0] = t[0] / double(n_steps);
    ms[1] = ((ctx->median_pass || ctx->ens_pass) && !ctx->act.fused) ? t[1] / double(n_steps) : 0.0;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) { release(ctx); }

int lbm_step_static(const lbm_domain_desc* domain, int32_t storage, void* stream, void* f0, void* f1,
                    int64_t n_steps, double* stats)
{
    if (!domain) return fail(nullptr, LBM_EINVAL, "domain is NULL");
    lbm_run_desc run;
    std::memset(&run, 0, sizeof(run));
    run.struct_size = sizeof(run);
    run.storage = storage;
    int rc = validate(domain, 1, &run);
    if (rc) return rc;
    if (!f0 || !f1 || f0 == f1) return fail(nullptr, LBM_EINVAL, "f0 and f1 must be two distinct device buffers");
    if (n_steps < 0) return fail(nullptr, LBM_EINVAL, "n_steps < 0");
    if (domain->f_init || domain->rho_init || domain->u_init)
        return fail(nullptr, LBM_EINVAL, "f_init, rho_init and u_init must be NULL: the state is in f0");
    if (domain->probe_x >= 0 || domain->probe_y >= 0)
        return fail(nullptr, LBM_EINVAL, "no probe trace without a context (probe_x, probe_y must be -1)");
    DomainHost h;
    StaticLayout L;
    plan_static(*domain, storage, h, L);
    if (L.total > kStaticScratchBytes)
        return fail(nullptr, LBM_ENOMEM,
                    "lbm_step_static: the domain needs " + std::to_string(L.total) +
                        " bytes of static scratch, more than the " + std::to_string(kStaticScratchBytes) +
                        " the library holds per GPU (use lbm_create / lbm_step)");
    if (n_steps == 0) return LBM_OK;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    char* base = nullptr;
    if (e == hipSuccess) e = static_scratch(device, &base);
    if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, std::string("static scratch: ") + hipGetErrorString(e));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const DomainDev dd = make_dev(h, base, f0, f1, 1, 0);
    DomainDev* dom = reinterpret_cast<DomainDev*>(base + L.off_dom);
    Tile* tiles = reinterpret_cast<Tile*>(base + L.off_tiles);
    RowBlock* rows = reinterpret_cast<RowBlock*>(base + L.off_rows);
    long long* counter = reinterpret_cast<long long*>(base + L.off_counter);
    e = launch_static_setup(dd, domain->lattice, dom, tiles, L.ntiles, rows, L.nblocks, counter, s);
    if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, std::string("static setup: ") + hipGetErrorString(e));
    StepKind k;
    k.storage = storage;
    k.lattice = domain->lattice;
    k.qe = domain->qe;
    k.ds = domain->ds_form;
    k.bc = is_cavity(domain->bc) ? kCavity : domain->bc;
    k.elbm = domain->collision == LBM_COLL_ELBM;
    k.median_pass = domain->lattice == LBM_D2Q9 && (domain->limiter & LBM_LIM_MEDIAN);
    k.ens_pass = deferred(*domain);
    k.budget = (domain->limiter & kLimEnsBudget) || is_topk(*domain);
    StepArgs a;
    a.dom = dom;
    a.tiles = tiles;
    a.ntiles = L.ntiles;
    a.ndomains = 1;
    a.parity = 0;
    a.flags = 0;
    a.partials = reinterpret_cast<double*>(base + L.off_partials);
    a.median_pass = (k.median_pass || k.ens_pass) ? 1 : 0;
    a.ens_pass = k.ens_pass ? 1 : 0;
    a.budget = k.budget ? 1 : 0;
    a.rows = rows;
    a.nrows = L.nblocks;
    a.groups = tiles;
    a.ngroups = L.ntiles;
    a.pstride = L.ntiles;
    a.rowpart = reinterpret_cast<double*>(base + L.off_rowpart);
    a.counter = counter;
    for (int64_t t = 0; t < n_steps && e == hipSuccess; ++t) {
        a.parity = int(t % 2);
        e = launch_step(k, a, s);
    }
    if (e == hipSuccess && stats) {
        e = launch_finalize(a, int((n_steps - 1) % 2), n_steps, s);
        if (e == hipSuccess) e = launch_static_stats(dom, h.shift * double(h.n), stats, s);
    }
    if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, std::string("lbm_step_static: ") + hipGetErrorString(e));
    return LBM_OK;
}

}  // extern "C"
