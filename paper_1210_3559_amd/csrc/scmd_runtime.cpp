// Host runtime of the Sutton-Chen cluster-MD library: the C ABI declared in
// include/scmd.h.  It validates arguments, owns device memory, plans the
// split of the all-pairs sweeps into work items, enqueues the per-step kernel
// sequence on the context stream and replays it from captured HIP graphs.
#include "../../include/scmd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cell_list.h"
#include "scmd_internal.h"

using namespace scmd;

namespace {

thread_local std::string g_create_error;

// Fixed device memory of scmd_rdf_noalloc (the reference-atom list of the
// pair-distance histogram and its count): kScratchRefs 32-bit indices plus
// one 256-byte block for the count.  Every context on a device shares that
// device's copy.  Host code never passes the array itself to a kernel: each
// device's address comes from hipGetSymbolAddress (g_scratch).
constexpr int kScratchRefs = 1 << 20;
constexpr size_t kScratchBytes = (size_t)kScratchRefs * sizeof(int32_t) + 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch[kMaxDevices] = {};

// Address of the scratch array on `device` (which must be current), looked up
// once per device.
hipError_t scratch_address(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

constexpr int kGraphSteps = 32;  // steps per captured graph

struct EvPair {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;
};

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t ensure(size_t count) {
        if (count <= n && p) return hipSuccess;
        release();
        if (count == 0) return hipSuccess;
        hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        n = count;
        return hipSuccess;
    }
};

}  // namespace

struct scmd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    std::string err;

    // configuration
    bool have_clusters = false, have_pot = false, have_integ = false;
    int nclusters = 0;
    int natoms = 0;
    double mass = 0.0;
    std::vector<int64_t> offsets;
    std::vector<ClusterDesc> cdesc;
    scmd_sc_params params{};
    PotConst pc{};
    double dt = 0.0;
    int precision = SCMD_FP64;
    int neighbour = SCMD_ALLPAIRS;
    scmd_tuning tuning{};

    // device state
    DevBuf<double4> rp, v, f;
    DevBuf<double2> dpv;  // drift inputs of the fused row path (3 per atom)
    // sampled observables (ring buffer of sample_cap slots x nclusters x 5)
    int64_t sample_every = 0;
    int sample_cap = 0;
    int64_t sample_total = 0;
    DevBuf<double> d_samples;
    DevBuf<double> rho;
    DevBuf<int32_t> atom_cluster;
    DevBuf<ClusterDesc> d_cdesc;
    DevBuf<ClusterState> d_state;
    DevBuf<int> d_flag;
    DevBuf<int32_t> rdf_refs;
    DevBuf<int> rdf_nref;
    DevBuf<unsigned long long> rdf_counts;
    // frame stores of the diffusion coefficient (one per cluster that has one)
    struct FrameStore {
        int cluster = 0;
        int cap = 0;
        int64_t recorded = 0;
        DevBuf<double4> buf;
    };
    std::vector<FrameStore> frames;
    void *scratch = nullptr;  // this device's fixed scratch array (scmd_rdf_noalloc)
    DevBuf<double> diff_seg;  // per-segment coefficients, then the mean
    DevBuf<int> diff_ncentral;
    int *h_flag = nullptr;  // pinned

    // all-pairs plan
    bool plan_ok = false;
    int ipt = 1, wi = 4, wj = 1, tile = 256;
    int nitems = 0, ntiles = 0;
    DevBuf<SweepItem> d_items;
    DevBuf<int32_t> d_order;
    DevBuf<ITile> d_tiles;
    DevBuf<double> d_part;
    DevBuf<double> d_tile_sums;
    DevBuf<double4> xp;
    bool has_split = false;  // some tile's partner range spans several items

    // symmetric all-pairs plan
    bool row = false;       // row sweeps (small clusters, no partial slots)
    int row_waves = 16;
    int row_uni_off = 0, row_uni_n = 0, row_uni_ni = 0;  // single-cluster row plan (ni = 0: tables)
    int row_nmax = 0;
    bool sym = false;
    int sym_ipt = 4, sym_nitems = 0, sym_ntiles = 0;
    DevBuf<SymItem> d_sitems;
    DevBuf<int32_t> d_sorder;
    DevBuf<SymTile> d_stiles;
    DevBuf<double> d_ipart, d_jpart;

    // cell-list plan (cutoff variant)
    CellList *cells = nullptr;
    double cell_skin = 0.4;          // list margin of the cell list, A
    DevBuf<double4> restore_scratch;  // checkpoint restore of the cell lists

    // progress
    bool have_forces = false;
    int64_t step = 0;

    // graphs
    // slot 0: kGraphSteps steps; slot 1: the remainder of the last run
    // length that was not a multiple of kGraphSteps
    struct GraphSlot {
        hipGraphExec_t exec = nullptr;
        int64_t len = 0;
        int profiled = 0;
        std::vector<int> ev;  // profiling events captured in the graph
        bool unread = false;  // replayed since its events were last read
    };
    GraphSlot graphs[2];
    std::vector<int> *ev_capture = nullptr;  // event list of the graph being captured

    // profiling
    int profiling = 0;
    bool capture_sample = false;  // the step being captured carries event nodes
    bool graph_events_ok = true;
    std::vector<EvPair> evs;
    std::vector<int> ev_free, ev_pending;
    double prof_ms[SCMD_KERNEL_COUNT] = {0, 0};
    int64_t prof_n[SCMD_KERNEL_COUNT] = {0, 0};
};

namespace {

int fail(scmd_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                                  \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return fail((ctx), e_ == hipErrorOutOfMemory ? SCMD_ENOMEM : SCMD_EDEVICE,                      \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                                 \
    } while (0)

#define SCMD_GUARD(...)                                          \
    try {                                                        \
        __VA_ARGS__                                              \
    } catch (const std::bad_alloc &) {                           \
        return fail(ctx, SCMD_ENOMEM, "host allocation failed"); \
    } catch (...) {                                              \
        return fail(ctx, SCMD_EDEVICE, "internal error");        \
    }

// Batches of staged clusters (all <= kRowStageMax atoms) up to this many
// unordered pairs per step run on the row sweeps by default.
constexpr double kRowBatchPairs = 2.5e7;
constexpr int kRdfMaxBins = 32768;  // LDS histogram of 128 KiB

int64_t ndof_of(int64_t n) {
    if (n >= 3) return 3 * n - 6;
    if (n == 2) return 1;
    return 0;
}

// Thermal degrees of freedom: the Langevin bath exchanges momentum and
// angular momentum with the cluster, so all 3N are thermal under it.
int64_t ndof_for(int kind, int64_t n) { return kind == SCMD_LANGEVIN ? 3 * n : ndof_of(n); }

PotConst make_pot(const scmd_sc_params &p) {
    PotConst pc{};
    pc.n = p.n;
    pc.m = p.m;
    pc.am = std::pow(p.a, (double)p.m);
    const double an = std::pow(p.a, (double)p.n);
    pc.A = p.eps * (double)p.n * an;
    pc.Pscale = p.eps * p.c * (double)p.m * 0.5 * pc.am;
    pc.half_eps_an = 0.5 * p.eps * an;
    pc.eps_c = p.eps * p.c;
    pc.cut = p.rc > 0.0 ? 1 : 0;
    pc.rc2 = p.rc * p.rc;
    pc.inv_rc_m = p.rc > 0.0 ? std::pow(p.rc, -(double)p.m) : 0.0;
    pc.inv_rc_n = p.rc > 0.0 ? std::pow(p.rc, -(double)p.n) : 0.0;
    pc.generic = (p.n == 9 && p.m == 6) ? 0 : 1;
    pc.A8 = pc.A * 0.125;
    pc.inv_rc_n512 = pc.inv_rc_n * 512.0;
    return pc;
}

void drop_graph_slot(scmd_ctx *c, int slot) {
    scmd_ctx::GraphSlot &g = c->graphs[slot];
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.len = 0;
    for (int i : g.ev) c->ev_free.push_back(i);
    g.ev.clear();
    g.unread = false;
}

void drop_graph(scmd_ctx *c) {
    drop_graph_slot(c, 0);
    drop_graph_slot(c, 1);
}

bool ready(scmd_ctx *c) { return c->have_clusters && c->have_pot && c->have_integ; }

// -------------------------------------------------------------------------
// Profiling events
// -------------------------------------------------------------------------
int take_event(scmd_ctx *c, int kind) {
    int idx;
    if (!c->ev_free.empty()) {
        idx = c->ev_free.back();
        c->ev_free.pop_back();
    } else {
        EvPair e;
        if (hipEventCreate(&e.a) != hipSuccess) return -1;
        if (hipEventCreate(&e.b) != hipSuccess) {
            (void)hipEventDestroy(e.a);
            return -1;
        }
        c->evs.push_back(e);
        idx = (int)c->evs.size() - 1;
    }
    c->evs[idx].kind = kind;
    return idx;
}

void harvest_events(scmd_ctx *c) {
    auto read = [&](int idx) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->evs[idx].a, c->evs[idx].b) == hipSuccess) {
            c->prof_ms[c->evs[idx].kind] += ms;
            c->prof_n[c->evs[idx].kind] += 1;
        }
    };
    for (int idx : c->ev_pending) {
        read(idx);
        c->ev_free.push_back(idx);
    }
    c->ev_pending.clear();
    for (auto &g : c->graphs) {
        if (g.unread) {
            for (int idx : g.ev) read(idx);
            g.unread = false;
        }
    }
}

// -------------------------------------------------------------------------
// Plan: atom tiles and sweep items
// -------------------------------------------------------------------------
// Library default launch shape for the all-pairs sweeps: many short
// partner loops for small clusters (latency-bound), wide i tiles for large
// ones (throughput-bound).
void default_shape(const scmd_ctx *c, int *ipt, int *wi, int *wj, int *target) {
    int64_t nmax = 0;
    for (int k = 0; k < c->nclusters; ++k) nmax = std::max<int64_t>(nmax, c->offsets[k + 1] - c->offsets[k]);
    if (nmax <= 4096) {  // small clusters: latency-bound, many short partner loops
        *ipt = 1;
        *wi = 1;
        *wj = 8;
        *target = 8192;
    } else {
        *ipt = 2;
        *wi = 1;
        *wj = 8;
        *target = 2048;
    }
}

bool shape_supported(int ipt, int wi, int wj) {
#define SCMD_SHAPE_OK(I, WI_, WJ_) \
    if (ipt == I && wi == WI_ && wj == WJ_) return true;
    SCMD_SWEEP_SHAPES(SCMD_SHAPE_OK)
#undef SCMD_SHAPE_OK
    return false;
}

// Symmetric plan: 64-atom tiles, groups of IPT tiles, one diagonal item per
// group and the group's later tiles cut into chunks of about equal work.
// Derived per-cluster constants (degrees of freedom, bath factor for the
// current dt), then the table to the device.
hipError_t upload_cdesc(scmd_ctx *c) {
    for (ClusterDesc &d : c->cdesc) {
        d.ndof = ndof_for(d.kind, d.n);
        d.bath_c1 = d.kind == SCMD_LANGEVIN ? std::exp(-d.gamma * 1e-3 * c->dt) : 1.0;
    }
    if (c->cdesc.empty() || !c->d_cdesc.p) return hipSuccess;
    return hipMemcpy(c->d_cdesc.p, c->cdesc.data(), c->cdesc.size() * sizeof(ClusterDesc), hipMemcpyHostToDevice);
}

int build_sym_plan(scmd_ctx *c, int target) {
    const int ipt = c->sym_ipt;
    std::vector<SymTile> tiles;
    std::vector<SymItem> items;
    double offdiag = 0.0;
    for (int k = 0; k < c->nclusters; ++k) {
        const int64_t n = c->offsets[k + 1] - c->offsets[k];
        const int64_t nt = (n + 63) / 64;
        for (int64_t g = 0; g * ipt < nt; ++g) offdiag += (double)std::max<int64_t>(0, nt - (g + 1) * ipt);
    }
    const int chunk = std::max(1, (int)std::ceil(offdiag / std::max(1, target)));
    int jbase = 0;
    for (int k = 0; k < c->nclusters; ++k) {
        ClusterDesc &d = c->cdesc[k];
        const int off = (int)c->offsets[k];
        const int n = (int)(c->offsets[k + 1] - c->offsets[k]);
        const int nt = (n + 63) / 64;
        d.off = off;
        d.n = n;
        d.tile0 = (int)tiles.size();
        d.ntiles = nt;
        d.ndof = ndof_for(d.kind, n);
        for (int t = 0; t < nt; ++t) {
            SymTile T{};
            T.c = k;
            T.i0 = off + 64 * t;
            T.ni = std::min(64, n - 64 * t);
            T.nj = t / ipt;
            T.jbase = jbase;
            T.p = t % ipt;
            jbase += T.nj;
            tiles.push_back(T);
        }
        for (int g = 0; g * ipt < nt; ++g) {
            const int first = (int)items.size();
            SymItem it{};
            it.c = k;
            it.g = g;
            it.t0 = d.tile0 + g * ipt;
            it.ng = std::min(ipt, nt - g * ipt);
            it.b0 = it.b1 = 0;
            it.slot = first;
            items.push_back(it);
            for (int b = (g + 1) * ipt; b < nt; b += chunk) {
                SymItem o = it;
                o.b0 = d.tile0 + b;
                o.b1 = d.tile0 + std::min(nt, b + chunk);
                o.slot = (int)items.size();
                items.push_back(o);
            }
            for (int t = g * ipt; t < g * ipt + it.ng; ++t) {
                tiles[d.tile0 + t].item0 = first;
                tiles[d.tile0 + t].nitems = (int)items.size() - first;
            }
        }
    }
    std::vector<int32_t> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    auto work = [&](const SymItem &it) -> int64_t {
        return it.b1 > it.b0 ? (int64_t)(it.b1 - it.b0) * 64 * 64 * it.ng : (int64_t)64 * 64 * it.ng * it.ng / 2;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return work(items[x]) > work(items[y]); });
    c->sym_nitems = (int)items.size();
    c->sym_ntiles = (int)tiles.size();
    c->ntiles = (int)tiles.size();
    HIP_TRY(c, c->d_sitems.ensure(std::max<size_t>(items.size(), 1)));
    HIP_TRY(c, c->d_sorder.ensure(std::max<size_t>(order.size(), 1)));
    HIP_TRY(c, c->d_stiles.ensure(std::max<size_t>(tiles.size(), 1)));
    HIP_TRY(c, c->d_ipart.ensure(std::max<size_t>(items.size() * 4 * 64 * (size_t)ipt, 1)));
    HIP_TRY(c, c->d_jpart.ensure(std::max<size_t>((size_t)jbase * 3 * 64, 1)));
    HIP_TRY(c, c->d_tile_sums.ensure(std::max<size_t>((size_t)tiles.size() * kTileSums, 1)));
    HIP_TRY(c, c->d_cdesc.ensure(std::max<size_t>(c->cdesc.size(), 1)));
    HIP_TRY(c, c->xp.ensure(std::max<size_t>(c->natoms, 1)));
    HIP_TRY(c, hipMemset(c->d_tile_sums.p, 0, c->d_tile_sums.n * sizeof(double)));
    if (!items.empty()) {
        HIP_TRY(c, hipMemcpy(c->d_sitems.p, items.data(), items.size() * sizeof(SymItem), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_sorder.p, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (!tiles.empty())
        HIP_TRY(c, hipMemcpy(c->d_stiles.p, tiles.data(), tiles.size() * sizeof(SymTile), hipMemcpyHostToDevice));
    HIP_TRY(c, upload_cdesc(c));
    c->plan_ok = true;
    return SCMD_OK;
}

// Row plan: tiles of ni <= 8 * waves atoms, one workgroup each, sized so
// that the sweep has about `target` workgroups of about equal work (ni n_c).
int build_row_plan(scmd_ctx *c, int target, std::vector<ITile> *tiles_out) {
    double total = 0.0;
    int nmax = 0;
    for (int k = 0; k < c->nclusters; ++k) {
        const double n = (double)(c->offsets[k + 1] - c->offsets[k]);
        total += n * n;
        nmax = std::max(nmax, (int)(c->offsets[k + 1] - c->offsets[k]));
    }
    c->row_nmax = nmax;
    const double ni_cap = std::min(64, 8 * c->row_waves);
    const double wstar = std::max(1.0, total / std::max(1, target));
    std::vector<ITile> tiles;
    int tmax = 1;
    for (int k = 0; k < c->nclusters; ++k) {
        ClusterDesc &d = c->cdesc[k];
        const int off = (int)c->offsets[k];
        const int n = (int)(c->offsets[k + 1] - c->offsets[k]);
        int ni = n > 0 ? (int)std::min<double>(ni_cap, std::max(1.0, std::ceil(wstar / n))) : 1;
        // each atom of a tile gets floor(groups / ni) of the 8-lane groups;
        // when that leaves more than a tenth of the groups idle, take the
        // largest power of two <= ni instead (it divides the group count)
        const int groups = 8 * c->row_waves;
        if (ni * (groups / ni) < groups - groups / 10) {
            int p2 = 1;
            while (2 * p2 <= ni) p2 *= 2;
            ni = p2;
        }
        d.off = off;
        d.n = n;
        d.tile0 = (int)tiles.size();
        d.ntiles = (n + ni - 1) / ni;
        d.ndof = ndof_for(d.kind, n);
        for (int t = 0; t < d.ntiles; ++t) {
            ITile T{};
            T.c = k;
            T.i0 = off + t * ni;
            T.ni = std::min(ni, n - t * ni);
            T.first = 0;
            T.nsplit = 1;
            tiles.push_back(T);
        }
        tmax = std::max(tmax, ni);
    }
    std::vector<int32_t> order(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        const int64_t wx = (int64_t)tiles[x].ni * c->cdesc[tiles[x].c].n;
        const int64_t wy = (int64_t)tiles[y].ni * c->cdesc[tiles[y].c].n;
        return wx > wy;
    });
    c->tile = tmax;
    c->nitems = 0;
    c->ntiles = (int)tiles.size();
    c->row_uni_ni = 0;
    if (c->nclusters == 1 && !tiles.empty()) {
        c->row_uni_off = c->cdesc[0].off;
        c->row_uni_n = c->cdesc[0].n;
        c->row_uni_ni = tiles[0].ni;
    }
    c->has_split = false;
    HIP_TRY(c, c->d_items.ensure(1));
    HIP_TRY(c, c->d_order.ensure(std::max<size_t>(order.size(), 1)));
    HIP_TRY(c, c->d_tiles.ensure(std::max<size_t>(tiles.size(), 1)));
    HIP_TRY(c, c->d_part.ensure(1));
    HIP_TRY(c, c->d_tile_sums.ensure(std::max<size_t>((size_t)tiles.size() * kTileSums, 1)));
    HIP_TRY(c, c->d_cdesc.ensure(std::max<size_t>(c->cdesc.size(), 1)));
    HIP_TRY(c, c->xp.ensure(std::max<size_t>(c->natoms, 1)));
    HIP_TRY(c, hipMemset(c->d_tile_sums.p, 0, c->d_tile_sums.n * sizeof(double)));
    if (!tiles.empty()) {
        HIP_TRY(c, hipMemcpy(c->d_order.p, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_tiles.p, tiles.data(), tiles.size() * sizeof(ITile), hipMemcpyHostToDevice));
    }
    HIP_TRY(c, upload_cdesc(c));
    if (tiles_out) *tiles_out = tiles;
    c->plan_ok = true;
    return SCMD_OK;
}

int build_plan(scmd_ctx *c, std::vector<ITile> *tiles_out) {
    c->plan_ok = false;
    c->row = false;
    {
        int64_t nmax = 0;
        for (int k = 0; k < c->nclusters; ++k) nmax = std::max<int64_t>(nmax, c->offsets[k + 1] - c->offsets[k]);
        // Library choice (from the autotuner on MI355X, its table committed
        // with the Python package): symmetric sweeps for batches and for
        // clusters above 4096 atoms; eight tiles per wavefront (fewest moves
        // per pair) and fine splitting for large batches and very large
        // clusters, two tiles in between.
        const bool allowed = c->neighbour == SCMD_ALLPAIRS && !c->pc.generic;
        const bool batch = c->nclusters > 1;
        // row sweeps: single clusters up to 4096 atoms, unless a one-sided
        // launch shape was given
        const bool shape_given = c->tuning.ipt > 0 || c->tuning.waves_i > 0 || c->tuning.waves_j > 0;
        double upairs = 0.0;  // unordered pairs per step
        for (int k = 0; k < c->nclusters; ++k) {
            const double n = (double)(c->offsets[k + 1] - c->offsets[k]);
            upairs += 0.5 * n * (n - 1.0);
        }
        // row sweeps evaluate every ordered pair but finish a step in two
        // launches; the symmetric sweeps need enough work to fill the chip
        const bool row_default = nmax <= 4096 && !shape_given && (!batch || upairs <= kRowBatchPairs);
        if (c->neighbour == SCMD_ALLPAIRS && (c->tuning.pairs == 3 || (c->tuning.pairs == 0 && row_default))) {
            c->sym = false;
            c->row = true;
            c->row_waves = c->tuning.waves_j > 0 ? c->tuning.waves_j : 8;
            return build_row_plan(c, c->tuning.target_items > 0 ? c->tuning.target_items : 256, tiles_out);
        }
        c->sym = allowed && (c->tuning.pairs == 2 || (c->tuning.pairs == 0 && (batch || nmax > 4096)));
        if (c->sym) {
            int ipt = nmax > 32768 ? 8 : 2;
            int target = nmax > 32768 ? 8192 : 2048;
            if (batch) {
                // about 32k pairs per work item, 512 to 8192 items
                ipt = upairs >= 2e8 ? 8 : 2;
                target = 512;
                while (target < 8192 && target * 32768.0 * 1.5 < upairs) target *= 2;
            }
            if (c->tuning.ipt == 2 || c->tuning.ipt == 4 || c->tuning.ipt == 8) ipt = c->tuning.ipt;
            if (c->tuning.target_items > 0) target = c->tuning.target_items;
            c->sym_ipt = ipt;
            return build_sym_plan(c, target);
        }
    }
    int target = 2048;
    default_shape(c, &c->ipt, &c->wi, &c->wj, &target);
    if (c->tuning.ipt > 0) {
        c->ipt = c->tuning.ipt;
        c->wi = c->tuning.waves_i;
        c->wj = c->tuning.waves_j;
    }
    if (c->tuning.target_items > 0) target = c->tuning.target_items;
    if (c->pc.generic) {  // the generic-exponent kernels exist in one shape
        c->ipt = 1;
        c->wi = 4;
        c->wj = 1;
    }
    c->tile = 64 * c->ipt * c->wi;
    const int tile = c->tile;
    const bool cells = c->neighbour == SCMD_CELLLIST;
    std::vector<ITile> tiles;
    std::vector<SweepItem> items;
    double total = 0.0;
    for (int k = 0; k < c->nclusters; ++k) {
        const int64_t n = c->offsets[k + 1] - c->offsets[k];
        const int64_t nt = (n + tile - 1) / tile;
        total += (double)nt * tile * (double)n;
    }
    const double wstar = std::max(total / target, (double)tile * 16.0 * c->wj);
    for (int k = 0; k < c->nclusters; ++k) {
        ClusterDesc &d = c->cdesc[k];
        const int off = (int)c->offsets[k];
        const int n = (int)(c->offsets[k + 1] - c->offsets[k]);
        d.off = off;
        d.n = n;
        d.tile0 = (int)tiles.size();
        d.ntiles = (n + tile - 1) / tile;
        d.ndof = ndof_for(d.kind, n);
        // split the partner range so that each wavefront keeps >= 16 partners
        int nsplit = (int)std::ceil((double)tile * (double)n / wstar);
        nsplit = std::max(1, std::min(nsplit, std::max(1, n / (16 * c->wj))));
        if (cells) nsplit = 1;  // cell sweeps produce complete sums
        for (int t = 0; t < d.ntiles; ++t) {
            ITile T{};
            T.c = k;
            T.i0 = off + t * tile;
            T.ni = std::min(tile, n - t * tile);
            T.first = (int)items.size();
            T.nsplit = nsplit;
            for (int s = 0; s < nsplit; ++s) {
                SweepItem it{};
                it.c = k;
                it.i0 = T.i0;
                it.ni = T.ni;
                it.j0 = off + (int)((int64_t)n * s / nsplit);
                it.j1 = off + (int)((int64_t)n * (s + 1) / nsplit);
                it.slot = (int)items.size();
                it.tile = (int)tiles.size();
                items.push_back(it);
            }
            tiles.push_back(T);
        }
    }
    std::vector<int32_t> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        const int64_t wx = (int64_t)items[x].ni * (items[x].j1 - items[x].j0);
        const int64_t wy = (int64_t)items[y].ni * (items[y].j1 - items[y].j0);
        return wx > wy;
    });
    c->nitems = (int)items.size();
    c->ntiles = (int)tiles.size();
    c->has_split = false;
    for (const ITile &T : tiles) c->has_split = c->has_split || T.nsplit > 1;
    const size_t part_items = cells ? 0 : items.size();  // cell sweeps finish their own atoms
    HIP_TRY(c, c->d_items.ensure(std::max<size_t>(items.size(), 1)));
    HIP_TRY(c, c->d_order.ensure(std::max<size_t>(order.size(), 1)));
    HIP_TRY(c, c->d_tiles.ensure(std::max<size_t>(tiles.size(), 1)));
    HIP_TRY(c, c->d_part.ensure(std::max<size_t>(part_items * 4 * (size_t)tile, 1)));
    HIP_TRY(c, c->d_tile_sums.ensure(std::max<size_t>((size_t)tiles.size() * kTileSums, 1)));
    HIP_TRY(c, c->d_cdesc.ensure(std::max<size_t>(c->cdesc.size(), 1)));
    HIP_TRY(c, c->xp.ensure(std::max<size_t>(c->natoms, 1)));
    HIP_TRY(c, hipMemset(c->d_tile_sums.p, 0, c->d_tile_sums.n * sizeof(double)));
    if (!items.empty()) {
        HIP_TRY(c, hipMemcpy(c->d_items.p, items.data(), items.size() * sizeof(SweepItem), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_order.p, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (!tiles.empty())
        HIP_TRY(c, hipMemcpy(c->d_tiles.p, tiles.data(), tiles.size() * sizeof(ITile), hipMemcpyHostToDevice));
    HIP_TRY(c, upload_cdesc(c));
    if (tiles_out) *tiles_out = tiles;
    c->plan_ok = true;
    return SCMD_OK;
}

int ensure_plan(scmd_ctx *c) {
    if (c->plan_ok) return SCMD_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    std::vector<ITile> tiles;
    int rc = build_plan(c, &tiles);
    if (rc != SCMD_OK) return rc;
    if (c->neighbour == SCMD_CELLLIST) {
        if (!c->cells) c->cells = cell_list_create();
        if (!c->cells) return fail(c, SCMD_ENOMEM, "cell list allocation failed");
        hipError_t e = cell_list_plan(c->cells, c->nclusters, c->offsets.data(), c->params.rc, c->cell_skin, c->rp.p);
        if (e != hipSuccess) return fail(c, SCMD_EDEVICE, std::string("cell list plan: ") + hipGetErrorString(e));
        // the cell sweeps finish their atoms and store per-cell sums: a
        // cluster's totals add its cells' slots
        for (int k = 0; k < c->nclusters; ++k)
            cell_list_sum_slots(c->cells, k, &c->cdesc[k].tile0, &c->cdesc[k].ntiles);
        HIP_TRY(c, c->d_tile_sums.ensure(std::max<size_t>((size_t)cell_list_total_slots(c->cells) * kTileSums, 1)));
        HIP_TRY(c, hipMemset(c->d_tile_sums.p, 0, c->d_tile_sums.n * sizeof(double)));
        HIP_TRY(c, upload_cdesc(c));
    }
    return SCMD_OK;
}

// -------------------------------------------------------------------------
// Enqueue
// -------------------------------------------------------------------------
// Record event ev on stream s.  During stream capture an event record issued
// on the stream does not become a graph node on this runtime, so the node is
// added explicitly after the current capture dependencies.
hipError_t record(hipEvent_t ev, hipStream_t s, bool capturing) {
    if (!capturing) return hipEventRecord(ev, s);
    hipStreamCaptureStatus st;
    hipGraph_t g = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t ndeps = 0;
    hipError_t e = hipStreamGetCaptureInfo_v2(s, &st, nullptr, &g, &deps, &ndeps);
    if (e != hipSuccess) return e;
    if (st != hipStreamCaptureStatusActive || !g) return hipErrorIllegalState;
    hipGraphNode_t node;
    e = hipGraphAddEventRecordNode(&node, g, deps, ndeps, ev);
    if (e != hipSuccess) return e;
    return hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
}

double half_kick(const scmd_ctx *c) { return 0.5 * c->dt / (c->mass * kEvPerUA2Fs2); }

StepArgs step_args(scmd_ctx *c, int advance, int energy = 1) {
    return StepArgs{c->d_cdesc.p, c->d_state.p, c->d_flag.p, c->mass, c->dt, half_kick(c), advance, energy};
}

SweepBuffers buffers(scmd_ctx *c) {
    return SweepBuffers{c->rp.p, c->xp.p, c->f.p, c->v.p, c->rho.p, c->d_part.p, c->d_tile_sums.p, c->dpv.p};
}

// One pair sweep (with its profiling events).  energy = 0 lets the force
// sweep skip the pair energy (steps whose energies nobody reads).  Row
// sweeps of staged clusters take the drift (drift_mode, local: RowDrift)
// and the fused force epilogue.
hipError_t sweep(scmd_ctx *c, bool force, hipStream_t s, bool capturing, int advance, int energy = 1,
                 int drift_mode = 0, int local = 0, int fused = 0) {
    int ev = -1;
    if (c->profiling && (!capturing || (c->graph_events_ok && c->capture_sample))) {
        ev = take_event(c, force ? SCMD_KERNEL_FORCE : SCMD_KERNEL_DENSITY);
        if (ev >= 0) {
            hipError_t e = record(c->evs[ev].a, s, capturing);
            if (e != hipSuccess) return e;
        }
    }
    const SweepBuffers B = buffers(c);
    const StepArgs A = step_args(c, advance, energy);
    hipError_t e;
    if (c->sym) {
        const SymLaunch L{c->d_sitems.p, c->d_sorder.p, c->d_stiles.p, c->sym_nitems, c->sym_ntiles, c->sym_ipt,
                          c->d_ipart.p, c->d_jpart.p};
        e = force ? launch_sym_force(L, B, A, c->pc, c->precision, 0, s)
                  : launch_sym_density(L, B, c->pc, c->precision, 0, s);
    } else if (c->row) {
        const RowLaunch R{c->d_tiles.p, c->d_order.p, c->d_cdesc.p, c->ntiles, c->row_waves, c->row_nmax,
                          c->row_uni_off, c->row_uni_n, c->row_uni_ni};
        // which clusters are in a Langevin bath (fixed while a graph exists:
        // thermostat changes drop it)
        int nb = 0;
        for (const ClusterDesc &d : c->cdesc) nb += d.kind == SCMD_LANGEVIN;
        const int bath = nb == 0 ? 0 : (nb == c->nclusters ? 1 : 2);
        e = force ? launch_row_force(R, B, A, fused, local, bath, c->pc, c->precision, s)
                  : launch_row_density(R, B, A, RowDrift{drift_mode, local, bath}, c->pc, c->precision, s);
    } else if (c->neighbour == SCMD_CELLLIST) {
        e = force ? cell_list_force(c->cells, B, A, c->pc, c->precision, s)
                  : cell_list_density(c->cells, B, c->pc, c->precision, s);
    } else {
        SweepLaunch L{c->d_items.p, c->d_order.p, c->d_tiles.p, c->nitems, c->ipt, c->wi, c->wj};
        e = force ? launch_force(L, B, A, c->pc, c->precision, s) : launch_density(L, B, c->pc, c->precision, s);
    }
    if (e != hipSuccess) return e;
    if (ev >= 0) {
        e = record(c->evs[ev].b, s, capturing);
        if (e != hipSuccess) return e;
        (capturing ? *c->ev_capture : c->ev_pending).push_back(ev);
    }
    return hipSuccess;
}

// rho, F, energies at the current positions; advance = 1 also kicks and
// runs the thermostat (second half of a step).
// Sweeps and tile finishes of one force evaluation (everything but the
// per-cluster finalize).
// checked: this step's drift ran the cell list's check (single cluster).
hipError_t enqueue_sweeps(scmd_ctx *c, hipStream_t s, bool capturing, int advance, int energy = 1,
                          bool checked = false) {
    hipError_t e;
    const SweepBuffers B = buffers(c);
    const StepArgs A = step_args(c, advance, energy);
    if (c->sym) {
        const SymLaunch L{c->d_sitems.p, c->d_sorder.p, c->d_stiles.p, c->sym_nitems, c->sym_ntiles, c->sym_ipt,
                          c->d_ipart.p, c->d_jpart.p};
        if ((e = sweep(c, false, s, capturing, advance)) != hipSuccess) return e;
        if ((e = launch_sym_density(L, B, c->pc, c->precision, 1, s)) != hipSuccess) return e;
        if ((e = sweep(c, true, s, capturing, advance, energy)) != hipSuccess) return e;
        return launch_sym_force(L, B, A, c->pc, c->precision, 1, s);
    }
    if (c->neighbour == SCMD_CELLLIST) {
        if ((e = cell_list_build(c->cells, c->rp.p, checked, s)) != hipSuccess) return e;
    }
    if ((e = sweep(c, false, s, capturing, advance)) != hipSuccess) return e;
    if (c->has_split && (e = launch_density_reduce(c->d_tiles.p, c->ntiles, c->tile, B, c->pc, 2, s)) != hipSuccess)
        return e;
    if ((e = sweep(c, true, s, capturing, advance, energy)) != hipSuccess) return e;
    if (c->has_split && (e = launch_force_reduce(c->d_tiles.p, c->ntiles, c->tile, B, A, c->pc, 2, s)) != hipSuccess)
        return e;
    return hipSuccess;
}

// rho, F, energies at the current positions; advance = 1 also kicks and
// runs the thermostat (second half of a step).
hipError_t enqueue_forces(scmd_ctx *c, hipStream_t s, bool capturing, int advance) {
    hipError_t e = enqueue_sweeps(c, s, capturing, advance);
    if (e != hipSuccess) return e;
    return launch_finalize(step_args(c, advance), c->d_tile_sums.p, c->nclusters, advance, s);
}

// A run of nsteps velocity-Verlet steps.  Only the last step of a run
// accumulates the pair energy: the state is read (getters, samples) only
// after a run.  The step before it carries the sampled profiling events of
// a captured run (a step without the energy term, like all but one).  A single cluster finishes each step
// inside the next step's drift (k_drift_fin) and the run's last step with the
// per-cluster finalize, which also stores the step counter; a batch runs the
// finalize after every step.
hipError_t enqueue_run(scmd_ctx *c, hipStream_t s, bool capturing, int64_t nsteps) {
    hipError_t e;
    const StepArgs A = step_args(c, 1);
    if (c->row && c->row_nmax <= kRowStageMax && c->natoms > 0) {
        // two launches per step: the density sweep drifts each staged
        // cluster (after finishing the previous step's thermostat factor),
        // the force sweep's epilogue kicks and stores the positions.  For a
        // cluster in a Langevin bath the force epilogue also runs the next
        // step's bath moves and stores the drifted positions (a per-atom
        // kernel does so before the first step of the run).
        bool bath = false;
        for (const ClusterDesc &d : c->cdesc) bath = bath || d.kind == SCMD_LANGEVIN;
        for (int64_t k = 0; k < nsteps; ++k) {
            // the sampled step is the last one without the pair energy
            if (capturing) c->capture_sample = (k == std::max<int64_t>(0, nsteps - 2));
            const int en = k == nsteps - 1;
            if (bath && k == 0 &&
                (e = launch_bath_prep(A, c->atom_cluster.p, c->rp.p, c->v.p, c->f.p, c->dpv.p, c->natoms, s)) !=
                    hipSuccess)
                return e;
            if ((e = sweep(c, false, s, capturing, 1, 1, k == 0 ? 1 : 2, (int)k)) != hipSuccess) return e;
            if ((e = sweep(c, true, s, capturing, 1, en, 0, (int)k, 1)) != hipSuccess) return e;
        }
        c->capture_sample = false;
        if (nsteps > 0) return launch_finalize(A, c->d_tile_sums.p, c->nclusters, (int)nsteps, s);
        return hipSuccess;
    }
    const bool fuse = c->nclusters == 1;
    const bool cells = c->neighbour == SCMD_CELLLIST;
    CellCheck cc{};
    if (fuse && cells) cc = cell_list_check(c->cells);
    for (int64_t k = 0; k < nsteps; ++k) {
        // a batch stores the step counters after every step (local = 0)
        const bool fin = fuse && k > 0;
        if (fin)
            e = launch_drift_fin(A, c->d_tile_sums.p, (int)k, c->rp.p, c->v.p, c->f.p, c->natoms, cells ? &cc : nullptr,
                                 s);
        else
            e = launch_drift(c->atom_cluster.p, c->d_cdesc.p, c->d_state.p, c->rp.p, c->v.p, c->f.p, c->natoms,
                             c->mass, c->dt, half_kick(c), 0, s);
        if (e != hipSuccess) return e;
        if (capturing) c->capture_sample = (k == std::max<int64_t>(0, nsteps - 2));
        e = enqueue_sweeps(c, s, capturing, 1, k == nsteps - 1, fin && cells);
        if (e != hipSuccess) return e;
        if (!fuse && (e = launch_finalize(A, c->d_tile_sums.p, c->nclusters, 1, s)) != hipSuccess) return e;
    }
    c->capture_sample = false;
    if (fuse && nsteps > 0) return launch_finalize(A, c->d_tile_sums.p, c->nclusters, (int)nsteps, s);
    return hipSuccess;
}

// Graph slot `slot` holding runs of `len` steps, captured when missing,
// of another length or taken with another profiling setting.
int ensure_graph(scmd_ctx *c, int slot, int64_t len) {
    scmd_ctx::GraphSlot &G = c->graphs[slot];
    if (G.exec && G.len == len && G.profiled == c->profiling) return SCMD_OK;
    // an earlier replay of the graph being replaced may still run
    if (G.exec) HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph_slot(c, slot);
    hipGraph_t g = nullptr;
    c->ev_capture = &G.ev;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_run(c, c->cap_stream, true, len);
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    c->ev_capture = nullptr;
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        for (int i : G.ev) c->ev_free.push_back(i);
        G.ev.clear();
        if (c->profiling && c->graph_events_ok) {
            // event records inside capture unsupported: profile eagerly instead
            c->graph_events_ok = false;
            (void)hipGetLastError();
            return ensure_graph(c, slot, len);
        }
        return fail(c, SCMD_EDEVICE, std::string("graph capture failed: ") +
                                         hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipError_t e3 = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
        G.exec = nullptr;
        return fail(c, SCMD_EDEVICE, std::string("graph instantiate failed: ") + hipGetErrorString(e3));
    }
    G.len = len;
    G.profiled = c->profiling;
    return SCMD_OK;
}

int check_ready(scmd_ctx *c) {
    if (!c) return SCMD_EINVAL;
    if (!ready(c)) return fail(c, SCMD_ESTATE, "init_clusters, set_potential and set_integrator must come first");
    return SCMD_OK;
}

int sync_and_check(scmd_ctx *c) {
    HIP_TRY(c, hipMemcpyAsync(c->h_flag, c->d_flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->profiling) harvest_events(c);
    if (*c->h_flag) return fail(c, SCMD_ENONFINITE, "a cluster energy became non-finite (coincident or overlapping atoms?)");
    return SCMD_OK;
}

// nsteps steps as replays of the kGraphSteps-step graph plus one replay of
// a graph of the remainder (kept for the next run of the same remainder);
// every replay ends with the per-cluster finalize, so the state is complete
// after it.  Eager launches only when profiling events cannot be captured.
int enqueue_chunk(scmd_ctx *c, int64_t nsteps) {
    const bool use_graph = !(c->profiling && !c->graph_events_ok);
    int64_t full = use_graph ? nsteps / kGraphSteps : 0;
    int64_t rem = nsteps - full * kGraphSteps;
    if (full > 0) {
        int rc = ensure_graph(c, 0, kGraphSteps);
        if (rc != SCMD_OK) return rc;
        for (int64_t r = 0; r < full; ++r) HIP_TRY(c, hipGraphLaunch(c->graphs[0].exec, c->stream));
        c->graphs[0].unread = c->profiling != 0;
    }
    if (rem > 0 && use_graph) {
        int rc = ensure_graph(c, 1, rem);
        if (rc != SCMD_OK) return rc;
        HIP_TRY(c, hipGraphLaunch(c->graphs[1].exec, c->stream));
        c->graphs[1].unread = c->profiling != 0;
    } else if (rem > 0) {
        HIP_TRY(c, enqueue_run(c, c->stream, false, rem));
    }
    c->step += nsteps;
    return SCMD_OK;
}

int enqueue_steps(scmd_ctx *c, int64_t nsteps) {
    int rc = ensure_plan(c);
    if (rc != SCMD_OK) return rc;
    if (!c->have_forces) {
        HIP_TRY(c, enqueue_forces(c, c->stream, false, 0));
        c->have_forces = true;
    }
    while (nsteps > 0) {
        int64_t chunk = nsteps;
        if (c->sample_every > 0) chunk = std::min(chunk, c->sample_every - c->step % c->sample_every);
        rc = enqueue_chunk(c, chunk);
        if (rc != SCMD_OK) return rc;
        nsteps -= chunk;
        if (c->sample_every > 0 && c->step % c->sample_every == 0) {
            const int slot = (int)(c->sample_total % c->sample_cap);
            HIP_TRY(c, launch_sample(c->d_state.p, c->nclusters, c->d_samples.p, slot, c->step, c->stream));
            ++c->sample_total;
        }
    }
    return SCMD_OK;
}

int copy_state_table(scmd_ctx *c, std::vector<ClusterState> &st) {
    st.resize(c->nclusters);
    if (c->nclusters > 0)
        HIP_TRY(c, hipMemcpy(st.data(), c->d_state.p, st.size() * sizeof(ClusterState), hipMemcpyDeviceToHost));
    return SCMD_OK;
}

int copy_aos(scmd_ctx *c, const double4 *src, double *out, const std::vector<double> *scale_per_atom) {
    std::vector<double4> tmp(c->natoms);
    if (c->natoms > 0)
        HIP_TRY(c, hipMemcpy(tmp.data(), src, tmp.size() * sizeof(double4), hipMemcpyDeviceToHost));
    for (int i = 0; i < c->natoms; ++i) {
        double s = scale_per_atom ? (*scale_per_atom)[i] : 1.0;
        if (scale_per_atom) {
            out[3 * i + 0] = s * tmp[i].x;
            out[3 * i + 1] = s * tmp[i].y;
            out[3 * i + 2] = s * tmp[i].z;
        } else {
            out[3 * i + 0] = tmp[i].x;
            out[3 * i + 1] = tmp[i].y;
            out[3 * i + 2] = tmp[i].z;
        }
    }
    return SCMD_OK;
}

void release_device(scmd_ctx *c) {
    drop_graph(c);
    c->rp.release();
    c->v.release();
    c->f.release();
    c->rho.release();
    c->dpv.release();
    c->d_samples.release();
    c->atom_cluster.release();
    c->d_cdesc.release();
    c->d_state.release();
    c->d_items.release();
    c->d_order.release();
    c->d_tiles.release();
    c->d_part.release();
    c->d_tile_sums.release();
    c->xp.release();
    c->d_sitems.release();
    c->d_sorder.release();
    c->d_stiles.release();
    c->d_ipart.release();
    c->d_jpart.release();
    c->restore_scratch.release();
    for (auto &fs : c->frames) fs.buf.release();
    c->frames.clear();
    c->diff_seg.release();
    c->diff_ncentral.release();
    if (c->cells) {
        cell_list_destroy(c->cells);
        c->cells = nullptr;
    }
}

struct StateHeader {
    char magic[8];
    int32_t version;
    int32_t nclusters;
    int64_t natoms;
    int64_t step;
    int32_t have_forces;
    int32_t pad;
};

// offsets, r, v, F (double4), rho, cluster tables, and the positions of the
// cell list's last build (double4; zero without a cell list)
size_t state_bytes(const scmd_ctx *c) {
    return sizeof(StateHeader) + (c->nclusters + 1) * sizeof(int64_t) + 4 * (size_t)c->natoms * sizeof(double4) +
           (size_t)c->natoms * sizeof(double) + (size_t)c->nclusters * (sizeof(ClusterDesc) + sizeof(ClusterState));
}

// After a thermostat setting changed: the device table (when a plan holds
// one) and the captured steps, which branch on the kind at capture time.
int apply_thermostat_change(scmd_ctx *c) {
    if (c->plan_ok && c->d_cdesc.p) {
        HIP_TRY(c, hipSetDevice(c->device));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, upload_cdesc(c));
    }
    drop_graph(c);
    return SCMD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int scmd_abi_version(void) { return SCMD_ABI_VERSION; }

const char *scmd_status_string(int status) {
    switch (status) {
        case SCMD_OK: return "ok";
        case SCMD_EINVAL: return "invalid argument";
        case SCMD_ENOMEM: return "out of memory";
        case SCMD_EDEVICE: return "device or HIP runtime error";
        case SCMD_ENONFINITE: return "non-finite energy";
        case SCMD_ESTATE: return "call out of order";
        case SCMD_EBOX: return "reserved (cell grid)";
        case SCMD_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char *scmd_last_error(const scmd_ctx *ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

int scmd_create(scmd_ctx **out, int device, void *hip_stream) {
    if (!out) {
        g_create_error = "out is NULL";
        return SCMD_EINVAL;
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        g_create_error = std::string("no HIP device: ") + (e != hipSuccess ? hipGetErrorString(e) : "count is 0");
        return SCMD_EDEVICE;
    }
    if (device < 0 || device >= count) {
        g_create_error = "device index out of range";
        return SCMD_EDEVICE;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
        return SCMD_EDEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = std::string("this library is built for gfx950, device is ") + prop.gcnArchName;
        return SCMD_EDEVICE;
    }
    scmd_ctx *c = nullptr;
    try {
        c = new scmd_ctx();
    } catch (...) {
        g_create_error = "host allocation failed";
        return SCMD_ENOMEM;
    }
    c->device = device;
    if ((e = hipSetDevice(device)) != hipSuccess) {
        delete c;
        g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return SCMD_EDEVICE;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
            delete c;
            g_create_error = std::string("hipStreamCreate: ") + hipGetErrorString(e);
            return SCMD_EDEVICE;
        }
        c->own_stream = true;
    }
    if ((e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipHostMalloc((void **)&c->h_flag, sizeof(int), hipHostMallocDefault)) != hipSuccess ||
        (e = c->d_flag.ensure(1)) != hipSuccess) {
        g_create_error = std::string("context setup: ") + hipGetErrorString(e);
        scmd_destroy(c);
        return SCMD_EDEVICE;
    }
    *c->h_flag = 0;
    if ((e = hipMemset(c->d_flag.p, 0, sizeof(int))) != hipSuccess) {
        g_create_error = std::string("hipMemset: ") + hipGetErrorString(e);
        scmd_destroy(c);
        return SCMD_EDEVICE;
    }
    // the device's scratch array (scmd_rdf_noalloc), looked up while the
    // device is current
    void *scr = nullptr;
    if ((e = scratch_address(device, &scr)) != hipSuccess) {
        g_create_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        scmd_destroy(c);
        return SCMD_EDEVICE;
    }
    c->scratch = scr;
    *out = c;
    return SCMD_OK;
}

int scmd_destroy(scmd_ctx *ctx) {
    if (!ctx) return SCMD_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    release_device(ctx);
    ctx->d_flag.release();
    for (auto &e : ctx->evs) {
        if (e.a) (void)hipEventDestroy(e.a);
        if (e.b) (void)hipEventDestroy(e.b);
    }
    if (ctx->h_flag) (void)hipHostFree(ctx->h_flag);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return SCMD_OK;
}

int scmd_init_clusters(scmd_ctx *ctx, int n_clusters, const int64_t *offsets, const double *pos, const double *vel,
                       double mass_u) {
    if (!ctx) return SCMD_EINVAL;
    SCMD_GUARD({
        if (n_clusters < 1 || !offsets) return fail(ctx, SCMD_EINVAL, "need n_clusters >= 1 and offsets");
        if (!(mass_u > 0.0) || !std::isfinite(mass_u)) return fail(ctx, SCMD_EINVAL, "mass_u must be > 0");
        if (offsets[0] != 0) return fail(ctx, SCMD_EINVAL, "offsets[0] must be 0");
        for (int k = 0; k < n_clusters; ++k)
            if (offsets[k + 1] < offsets[k]) return fail(ctx, SCMD_EINVAL, "offsets must be non-decreasing");
        const int64_t natoms = offsets[n_clusters];
        if (natoms >= (int64_t(1) << 30)) return fail(ctx, SCMD_EINVAL, "too many atoms (limit 2^30)");
        if (natoms > 0 && !pos) return fail(ctx, SCMD_EINVAL, "pos is NULL");
        for (int64_t i = 0; i < 3 * natoms; ++i) {
            if (!std::isfinite(pos[i]) || (vel && !std::isfinite(vel[i])))
                return fail(ctx, SCMD_EINVAL, "non-finite position or velocity");
            if (std::fabs(pos[i]) > 1e12) return fail(ctx, SCMD_EINVAL, "position beyond 1e12 A");
        }
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        release_device(ctx);
        ctx->have_clusters = false;
        ctx->plan_ok = false;
        ctx->have_forces = false;
        ctx->step = 0;
        ctx->sample_every = 0;
        ctx->sample_cap = 0;
        ctx->sample_total = 0;
        ctx->nclusters = n_clusters;
        ctx->natoms = (int)natoms;
        ctx->mass = mass_u;
        ctx->offsets.assign(offsets, offsets + n_clusters + 1);
        ctx->cdesc.assign(n_clusters, ClusterDesc{});
        for (auto &d : ctx->cdesc) {
            d.kind = SCMD_NVE;
            d.tau = 100.0;
        }
        std::vector<double4> r4(natoms), v4(natoms);
        std::vector<int32_t> ac(natoms);
        for (int64_t i = 0; i < natoms; ++i) {
            r4[i] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.0);
            v4[i] = vel ? make_double4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.0) : make_double4(0, 0, 0, 0);
        }
        for (int k = 0; k < n_clusters; ++k)
            for (int64_t i = offsets[k]; i < offsets[k + 1]; ++i) ac[i] = k;
        const size_t na = std::max<int64_t>(natoms, 1);
        HIP_TRY(ctx, ctx->rp.ensure(na));
        HIP_TRY(ctx, ctx->v.ensure(na));
        HIP_TRY(ctx, ctx->f.ensure(na));
        HIP_TRY(ctx, ctx->rho.ensure(na));
        HIP_TRY(ctx, ctx->dpv.ensure(3 * na));
        HIP_TRY(ctx, ctx->atom_cluster.ensure(na));
        HIP_TRY(ctx, ctx->d_state.ensure(n_clusters));
        HIP_TRY(ctx, ctx->d_cdesc.ensure(n_clusters));
        if (natoms > 0) {
            HIP_TRY(ctx, hipMemcpy(ctx->rp.p, r4.data(), natoms * sizeof(double4), hipMemcpyHostToDevice));
            HIP_TRY(ctx, hipMemcpy(ctx->v.p, v4.data(), natoms * sizeof(double4), hipMemcpyHostToDevice));
            HIP_TRY(ctx, hipMemcpy(ctx->atom_cluster.p, ac.data(), natoms * sizeof(int32_t), hipMemcpyHostToDevice));
            HIP_TRY(ctx, hipMemset(ctx->f.p, 0, natoms * sizeof(double4)));
            HIP_TRY(ctx, hipMemset(ctx->rho.p, 0, natoms * sizeof(double)));
        }
        std::vector<ClusterState> st(n_clusters);
        for (auto &s : st) {
            std::memset(&s, 0, sizeof(s));
            s.lambda = 1.0;
        }
        HIP_TRY(ctx, hipMemcpy(ctx->d_state.p, st.data(), st.size() * sizeof(ClusterState), hipMemcpyHostToDevice));
        HIP_TRY(ctx, hipMemset(ctx->d_flag.p, 0, sizeof(int)));
        *ctx->h_flag = 0;
        ctx->have_clusters = true;
        return SCMD_OK;
    })
}

int scmd_set_potential(scmd_ctx *ctx, const scmd_sc_params *p) {
    if (!ctx) return SCMD_EINVAL;
    if (!p) return fail(ctx, SCMD_EINVAL, "params is NULL");
    if (!(p->eps > 0.0) || !(p->a > 0.0) || !(p->c >= 0.0) || !std::isfinite(p->eps) || !std::isfinite(p->a) ||
        !std::isfinite(p->c))
        return fail(ctx, SCMD_EINVAL, "need eps > 0, a > 0, c >= 0");
    if (p->m < 1 || p->n <= p->m || p->n > 24) return fail(ctx, SCMD_EINVAL, "need 1 <= m < n <= 24");
    if (!(p->rc >= 0.0) || !std::isfinite(p->rc)) return fail(ctx, SCMD_EINVAL, "need rc >= 0");
    if (ctx->have_integ) {
        if (ctx->neighbour == SCMD_ALLPAIRS && p->rc > 0.0)
            return fail(ctx, SCMD_EINVAL, "all-pairs mode needs rc == 0 (use SCMD_CELLLIST for a cutoff)");
        if (ctx->neighbour == SCMD_CELLLIST && !(p->rc > 0.0))
            return fail(ctx, SCMD_EINVAL, "cell-list mode needs rc > 0");
    }
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->params = *p;
    ctx->pc = make_pot(*p);
    ctx->have_pot = true;
    ctx->have_forces = false;
    ctx->plan_ok = false;
    drop_graph(ctx);
    return SCMD_OK;
}

int scmd_set_integrator(scmd_ctx *ctx, double dt_fs, int precision, int neighbour) {
    if (!ctx) return SCMD_EINVAL;
    if (!(dt_fs > 0.0) || !std::isfinite(dt_fs)) return fail(ctx, SCMD_EINVAL, "need dt_fs > 0");
    if (precision != SCMD_FP64 && precision != SCMD_MIXED) return fail(ctx, SCMD_EINVAL, "unknown precision");
    if (neighbour != SCMD_ALLPAIRS && neighbour != SCMD_CELLLIST) return fail(ctx, SCMD_EINVAL, "unknown neighbour mode");
    if (ctx->have_pot) {
        if (neighbour == SCMD_ALLPAIRS && ctx->params.rc > 0.0)
            return fail(ctx, SCMD_EINVAL, "all-pairs mode needs rc == 0 (use SCMD_CELLLIST for a cutoff)");
        if (neighbour == SCMD_CELLLIST && !(ctx->params.rc > 0.0))
            return fail(ctx, SCMD_EINVAL, "cell-list mode needs rc > 0");
    }
    if (neighbour == SCMD_CELLLIST && !cell_list_available())
        return fail(ctx, SCMD_EUNSUPPORTED, "cell-list mode is not built into this library");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->dt = dt_fs;
    ctx->precision = precision;
    ctx->neighbour = neighbour;
    ctx->have_integ = true;
    ctx->have_forces = false;
    ctx->plan_ok = false;
    drop_graph(ctx);
    return SCMD_OK;
}

int scmd_set_thermostat(scmd_ctx *ctx, int cluster, int kind, double T_start_K, double T_end_K, int64_t ramp_steps,
                        double tau_fs) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (cluster < -1 || cluster >= ctx->nclusters) return fail(ctx, SCMD_EINVAL, "cluster index out of range");
    if (kind == SCMD_LANGEVIN) return fail(ctx, SCMD_EINVAL, "the Langevin bath is set with scmd_set_langevin");
    if (kind != SCMD_NVE && kind != SCMD_BERENDSEN) return fail(ctx, SCMD_EINVAL, "unknown thermostat kind");
    if (kind == SCMD_BERENDSEN) {
        if (!(tau_fs > 0.0) || !std::isfinite(tau_fs)) return fail(ctx, SCMD_EINVAL, "need tau_fs > 0");
        if (!(T_start_K >= 0.0) || !(T_end_K >= 0.0) || !std::isfinite(T_start_K) || !std::isfinite(T_end_K))
            return fail(ctx, SCMD_EINVAL, "temperatures must be finite and >= 0");
    }
    const int a = cluster < 0 ? 0 : cluster, b = cluster < 0 ? ctx->nclusters : cluster + 1;
    for (int k = a; k < b; ++k) {
        ClusterDesc &d = ctx->cdesc[k];
        d.kind = kind;
        if (kind == SCMD_BERENDSEN) {
            d.T_start = T_start_K;
            d.T_end = T_end_K;
            d.ramp = ramp_steps;
            d.tau = tau_fs;
            d.ramp_origin = ctx->step;
        }
    }
    return apply_thermostat_change(ctx);
}

int scmd_set_langevin(scmd_ctx *ctx, int cluster, double T_start_K, double T_end_K, int64_t ramp_steps,
                      double gamma_per_ps, uint64_t seed) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (cluster < -1 || cluster >= ctx->nclusters) return fail(ctx, SCMD_EINVAL, "cluster index out of range");
    if (!(gamma_per_ps >= 0.0) || !std::isfinite(gamma_per_ps)) return fail(ctx, SCMD_EINVAL, "need gamma >= 0");
    if (!(T_start_K >= 0.0) || !(T_end_K >= 0.0) || !std::isfinite(T_start_K) || !std::isfinite(T_end_K))
        return fail(ctx, SCMD_EINVAL, "temperatures must be finite and >= 0");
    const int a = cluster < 0 ? 0 : cluster, b = cluster < 0 ? ctx->nclusters : cluster + 1;
    for (int k = a; k < b; ++k) {
        ClusterDesc &d = ctx->cdesc[k];
        d.kind = SCMD_LANGEVIN;
        d.T_start = T_start_K;
        d.T_end = T_end_K;
        d.ramp = ramp_steps;
        d.gamma = gamma_per_ps;
        d.seed = seed;
        d.ramp_origin = ctx->step;
    }
    return apply_thermostat_change(ctx);
}

int scmd_set_cell_skin(scmd_ctx *ctx, double skin_A) {
    if (!ctx) return SCMD_EINVAL;
    if (!(skin_A >= 0.0) || !std::isfinite(skin_A)) return fail(ctx, SCMD_EINVAL, "skin must be finite and >= 0");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        ctx->cell_skin = skin_A;
        if (ctx->neighbour == SCMD_CELLLIST) {
            ctx->plan_ok = false;  // new cells and lists at the next evaluation
            drop_graph(ctx);
        }
        return SCMD_OK;
    })
}

int scmd_get_cell_rebuilds(scmd_ctx *ctx, int64_t *rebuilds) {
    if (!ctx || !rebuilds) return SCMD_EINVAL;
    if (ctx->neighbour != SCMD_CELLLIST || !ctx->cells || !ctx->plan_ok) {
        *rebuilds = 0;
        return SCMD_OK;
    }
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, cell_list_rebuilds(ctx->cells, rebuilds));
        return SCMD_OK;
    })
}

int scmd_set_tuning(scmd_ctx *ctx, const scmd_tuning *t) {
    if (!ctx) return SCMD_EINVAL;
    scmd_tuning z{};
    if (t) {
        if (t->pairs == 2) {
            if (t->ipt != 0 && t->ipt != 2 && t->ipt != 4 && t->ipt != 8)
                return fail(ctx, SCMD_EINVAL, "symmetric sweeps take ipt 2, 4 or 8");
        } else if (t->pairs == 3) {
            if (t->waves_j != 0 && t->waves_j != 4 && t->waves_j != 8 && t->waves_j != 16)
                return fail(ctx, SCMD_EINVAL, "row sweeps take waves_j 4, 8 or 16");
        } else if (t->ipt != 0 || t->waves_i != 0 || t->waves_j != 0) {
            if (!shape_supported(t->ipt, t->waves_i, t->waves_j))
                return fail(ctx, SCMD_EINVAL, "unsupported (ipt, waves_i, waves_j) launch shape");
        }
        if (t->target_items < 0) return fail(ctx, SCMD_EINVAL, "target_items must be >= 0");
        if (t->pairs < 0 || t->pairs > 3) return fail(ctx, SCMD_EINVAL, "pairs must be 0, 1, 2 or 3");
        z = *t;
    }
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->tuning = z;
    ctx->plan_ok = false;
    drop_graph(ctx);
    return SCMD_OK;
}

int scmd_compute(scmd_ctx *ctx) {
    int rc = check_ready(ctx);
    if (rc != SCMD_OK) return rc;
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        rc = ensure_plan(ctx);
        if (rc != SCMD_OK) return rc;
        HIP_TRY(ctx, enqueue_forces(ctx, ctx->stream, false, 0));
        ctx->have_forces = true;
        return sync_and_check(ctx);
    })
}

int scmd_step_async(scmd_ctx *ctx, int64_t nsteps) {
    int rc = check_ready(ctx);
    if (rc != SCMD_OK) return rc;
    if (nsteps < 0) return fail(ctx, SCMD_EINVAL, "nsteps must be >= 0");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        if (*ctx->h_flag) return fail(ctx, SCMD_ENONFINITE, "a previous step produced a non-finite energy");
        return enqueue_steps(ctx, nsteps);
    })
}

int scmd_synchronize(scmd_ctx *ctx) {
    if (!ctx) return SCMD_EINVAL;
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        if (!ctx->have_clusters) {
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            return SCMD_OK;
        }
        return sync_and_check(ctx);
    })
}

int scmd_step(scmd_ctx *ctx, int64_t nsteps) {
    int rc = scmd_step_async(ctx, nsteps);
    if (rc != SCMD_OK) return rc;
    return scmd_synchronize(ctx);
}

int scmd_get_step(scmd_ctx *ctx, int64_t *step) {
    if (!ctx || !step) return SCMD_EINVAL;
    *step = ctx->step;
    return SCMD_OK;
}

int scmd_get_energy(scmd_ctx *ctx, int cluster, double out3[3]) {
    int rc = check_ready(ctx);
    if (rc != SCMD_OK) return rc;
    if (!out3) return fail(ctx, SCMD_EINVAL, "out is NULL");
    if (cluster < -1 || cluster >= ctx->nclusters) return fail(ctx, SCMD_EINVAL, "cluster index out of range");
    if (!ctx->have_forces) return fail(ctx, SCMD_ESTATE, "compute or step first");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        rc = sync_and_check(ctx);
        if (rc != SCMD_OK) return rc;
        std::vector<ClusterState> st;
        rc = copy_state_table(ctx, st);
        if (rc != SCMD_OK) return rc;
        double ep = 0.0, ek = 0.0;
        for (int k = 0; k < ctx->nclusters; ++k) {
            if (cluster >= 0 && k != cluster) continue;
            ep += st[k].epot;
            ek += st[k].ekin;
        }
        out3[0] = ep;
        out3[1] = ek;
        out3[2] = ep + ek;
        return SCMD_OK;
    })
}

int scmd_set_sampling(scmd_ctx *ctx, int64_t every, int capacity) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (every < 0) return fail(ctx, SCMD_EINVAL, "every must be >= 0");
    if (every > 0 && capacity < 1) return fail(ctx, SCMD_EINVAL, "capacity must be >= 1");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        ctx->sample_every = 0;
        ctx->sample_cap = 0;
        ctx->sample_total = 0;
        if (every > 0) {
            const size_t need = (size_t)capacity * (size_t)ctx->nclusters * 5;
            if (ctx->d_samples.ensure(need) != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, SCMD_ENOMEM, "sample buffer allocation failed");
            }
            ctx->sample_every = every;
            ctx->sample_cap = capacity;
        }
        return SCMD_OK;
    })
}

int scmd_get_samples(scmd_ctx *ctx, int cluster, double *out, int max_samples, int *n_out, int64_t *recorded) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (cluster < 0 || cluster >= ctx->nclusters) return fail(ctx, SCMD_EINVAL, "cluster index out of range");
    if (!n_out || max_samples < 0 || (!out && max_samples > 0))
        return fail(ctx, SCMD_EINVAL, "need n_out, max_samples >= 0 and out");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        int rc = sync_and_check(ctx);
        if (rc != SCMD_OK) return rc;
        const int64_t held = ctx->sample_cap > 0 ? std::min<int64_t>(ctx->sample_total, ctx->sample_cap) : 0;
        const int64_t take = std::min<int64_t>(held, max_samples);
        if (take > 0) {
            std::vector<double> ring((size_t)ctx->sample_cap * ctx->nclusters * 5);
            HIP_TRY(ctx, hipMemcpy(ring.data(), ctx->d_samples.p, ring.size() * sizeof(double), hipMemcpyDeviceToHost));
            // the newest `take` samples, oldest first
            for (int64_t k = 0; k < take; ++k) {
                const int64_t idx = ctx->sample_total - take + k;  // sample number
                const size_t slot = (size_t)(idx % ctx->sample_cap);
                const double *src = ring.data() + (slot * ctx->nclusters + cluster) * 5;
                for (int q = 0; q < 5; ++q) out[5 * k + q] = src[q];
            }
        }
        *n_out = (int)take;
        if (recorded) *recorded = ctx->sample_total;
        return SCMD_OK;
    })
}

int scmd_get_temperature(scmd_ctx *ctx, int cluster, double *T_K, int64_t *ndof) {
    int rc = check_ready(ctx);
    if (rc != SCMD_OK) return rc;
    if (!T_K) return fail(ctx, SCMD_EINVAL, "T_K is NULL");
    if (cluster < 0 || cluster >= ctx->nclusters) return fail(ctx, SCMD_EINVAL, "cluster index out of range");
    if (!ctx->have_forces) return fail(ctx, SCMD_ESTATE, "compute or step first");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        rc = sync_and_check(ctx);
        if (rc != SCMD_OK) return rc;
        std::vector<ClusterState> st;
        rc = copy_state_table(ctx, st);
        if (rc != SCMD_OK) return rc;
        *T_K = st[cluster].temp;
        if (ndof) *ndof = ndof_for(ctx->cdesc[cluster].kind, ctx->offsets[cluster + 1] - ctx->offsets[cluster]);
        return SCMD_OK;
    })
}

int scmd_get_positions(scmd_ctx *ctx, double *out) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (!out && ctx->natoms > 0) return fail(ctx, SCMD_EINVAL, "out is NULL");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        return copy_aos(ctx, ctx->rp.p, out, nullptr);
    })
}

int scmd_get_velocities(scmd_ctx *ctx, double *out) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (!out && ctx->natoms > 0) return fail(ctx, SCMD_EINVAL, "out is NULL");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        std::vector<ClusterState> st;
        int rc = copy_state_table(ctx, st);
        if (rc != SCMD_OK) return rc;
        std::vector<double> lam(ctx->natoms);
        for (int k = 0; k < ctx->nclusters; ++k)
            for (int64_t i = ctx->offsets[k]; i < ctx->offsets[k + 1]; ++i) lam[i] = st[k].lambda;
        return copy_aos(ctx, ctx->v.p, out, &lam);
    })
}

int scmd_get_forces(scmd_ctx *ctx, double *out) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (!ctx->have_forces) return fail(ctx, SCMD_ESTATE, "compute or step first");
    if (!out && ctx->natoms > 0) return fail(ctx, SCMD_EINVAL, "out is NULL");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        return copy_aos(ctx, ctx->f.p, out, nullptr);
    })
}

int scmd_get_density(scmd_ctx *ctx, double *out) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (!ctx->have_forces) return fail(ctx, SCMD_ESTATE, "compute or step first");
    if (!out && ctx->natoms > 0) return fail(ctx, SCMD_EINVAL, "out is NULL");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->natoms > 0)
            HIP_TRY(ctx, hipMemcpy(out, ctx->rho.p, ctx->natoms * sizeof(double), hipMemcpyDeviceToHost));
        return SCMD_OK;
    })
}

int scmd_rdf(scmd_ctx *ctx, int cluster, double r_select, double dr, int nbins, uint64_t *counts,
             int64_t *n_ref) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (cluster < 0 || cluster >= ctx->nclusters) return fail(ctx, SCMD_EINVAL, "cluster index out of range");
    if (!(dr > 0.0) || !std::isfinite(dr)) return fail(ctx, SCMD_EINVAL, "need a finite dr > 0");
    if (!std::isfinite(r_select)) return fail(ctx, SCMD_EINVAL, "r_select must be finite");
    if (nbins < 1 || nbins > kRdfMaxBins) return fail(ctx, SCMD_EINVAL, "nbins must be in [1, 32768]");
    if (!counts || !n_ref) return fail(ctx, SCMD_EINVAL, "counts or n_ref is NULL");
    const int off = (int)ctx->offsets[cluster];
    const int n = (int)(ctx->offsets[cluster + 1] - ctx->offsets[cluster]);
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, ctx->rdf_refs.ensure(std::max(n, 1)));
        HIP_TRY(ctx, ctx->rdf_nref.ensure(1));
        HIP_TRY(ctx, ctx->rdf_counts.ensure(nbins));
        HIP_TRY(ctx, launch_rdf(ctx->rp.p, off, n, r_select, dr, nbins, ctx->rdf_refs.p, ctx->rdf_nref.p,
                                ctx->rdf_counts.p, true, nullptr, ctx->stream));
        std::vector<unsigned long long> h(nbins);
        int nr = 0;
        HIP_TRY(ctx, hipMemcpyAsync(h.data(), ctx->rdf_counts.p, nbins * sizeof(unsigned long long),
                                    hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(&nr, ctx->rdf_nref.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        for (int b = 0; b < nbins; ++b) counts[b] += h[b];
        *n_ref += nr;
        return SCMD_OK;
    })
}

int scmd_rdf_noalloc(scmd_ctx *ctx, int cluster, double r_select, double dr, int nbins, uint64_t *dev_counts,
                     int64_t *dev_n_ref) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (cluster < 0 || cluster >= ctx->nclusters) return fail(ctx, SCMD_EINVAL, "cluster index out of range");
    if (!(dr > 0.0) || !std::isfinite(dr)) return fail(ctx, SCMD_EINVAL, "need a finite dr > 0");
    if (!std::isfinite(r_select)) return fail(ctx, SCMD_EINVAL, "r_select must be finite");
    if (nbins < 1 || nbins > kRdfMaxBins) return fail(ctx, SCMD_EINVAL, "nbins must be in [1, 32768]");
    if (!dev_counts || !dev_n_ref) return fail(ctx, SCMD_EINVAL, "dev_counts or dev_n_ref is NULL");
    const int off = (int)ctx->offsets[cluster];
    const int n = (int)(ctx->offsets[cluster + 1] - ctx->offsets[cluster]);
    if (n > kScratchRefs)
        return fail(ctx, SCMD_EINVAL, "cluster larger than the fixed scratch array (1048576 atoms)");
    if (!ctx->scratch) return fail(ctx, SCMD_EDEVICE, "no scratch address for this device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // scratch layout: the count in the first 256 bytes, then the references
    int *nref = (int *)ctx->scratch;
    int32_t *refs = (int32_t *)((unsigned char *)ctx->scratch + 256);
    HIP_TRY(ctx, launch_rdf(ctx->rp.p, off, n, r_select, dr, nbins, refs, nref, (unsigned long long *)dev_counts,
                            false, (long long *)dev_n_ref, ctx->stream));
    return SCMD_OK;
}

int scmd_set_frames(scmd_ctx *ctx, int cluster, int capacity) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (cluster < 0 || cluster >= ctx->nclusters) return fail(ctx, SCMD_EINVAL, "cluster index out of range");
    if (capacity < 0) return fail(ctx, SCMD_EINVAL, "capacity must be >= 0");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        for (size_t k = 0; k < ctx->frames.size(); ++k) {
            if (ctx->frames[k].cluster == cluster) {
                ctx->frames[k].buf.release();
                ctx->frames.erase(ctx->frames.begin() + (long)k);
                break;
            }
        }
        if (capacity == 0) return SCMD_OK;
        const size_t n = (size_t)(ctx->offsets[cluster + 1] - ctx->offsets[cluster]);
        scmd_ctx::FrameStore fs;
        fs.cluster = cluster;
        fs.cap = capacity;
        if (fs.buf.ensure(std::max<size_t>((size_t)capacity * n, 1)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, SCMD_ENOMEM, "frame store allocation failed");
        }
        ctx->frames.push_back(fs);
        return SCMD_OK;
    })
}

int scmd_record_frame(scmd_ctx *ctx) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        for (auto &fs : ctx->frames) {
            const int off = (int)ctx->offsets[fs.cluster];
            const int n = (int)(ctx->offsets[fs.cluster + 1] - ctx->offsets[fs.cluster]);
            const size_t slot = (size_t)(fs.recorded % fs.cap);
            HIP_TRY(ctx, launch_store_frame(ctx->rp.p, off, n, fs.buf.p + slot * (size_t)n, ctx->stream));
            ++fs.recorded;
        }
        return SCMD_OK;
    })
}

int scmd_get_frame_count(scmd_ctx *ctx, int cluster, int64_t *recorded) {
    if (!ctx || !recorded) return SCMD_EINVAL;
    for (const auto &fs : ctx->frames) {
        if (fs.cluster == cluster) {
            *recorded = fs.recorded;
            return SCMD_OK;
        }
    }
    return fail(ctx, SCMD_EINVAL, "the cluster has no frame store");
}

int scmd_diffusion(scmd_ctx *ctx, int cluster, int64_t first, int nframes, double frame_dt_ps, double radius,
                   int segments, double *D_A2_per_ps, int64_t *n_central) {
    if (!ctx) return SCMD_EINVAL;
    if (!D_A2_per_ps || !n_central) return fail(ctx, SCMD_EINVAL, "D_A2_per_ps or n_central is NULL");
    const scmd_ctx::FrameStore *fs = nullptr;
    for (const auto &x : ctx->frames)
        if (x.cluster == cluster) fs = &x;
    if (!fs) return fail(ctx, SCMD_EINVAL, "the cluster has no frame store");
    if (segments < 1 || nframes < 0 || nframes / segments < 2)
        return fail(ctx, SCMD_EINVAL, "need segments >= 1 and at least two frames per segment");
    if (!(frame_dt_ps > 0.0) || !std::isfinite(frame_dt_ps)) return fail(ctx, SCMD_EINVAL, "need frame_dt_ps > 0");
    if (!(radius > 0.0) || !std::isfinite(radius)) return fail(ctx, SCMD_EINVAL, "need a finite radius > 0");
    if (first < 0 || first + nframes > fs->recorded || first < fs->recorded - fs->cap)
        return fail(ctx, SCMD_EINVAL, "frames outside those the store holds");
    const int n = (int)(ctx->offsets[cluster + 1] - ctx->offsets[cluster]);
    if (n < 1) return fail(ctx, SCMD_EINVAL, "empty cluster");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, ctx->diff_seg.ensure((size_t)segments + 1));
        HIP_TRY(ctx, ctx->diff_ncentral.ensure(1));
        const int seg = nframes / segments;
        HIP_TRY(ctx, launch_diffusion(fs->buf.p, n, fs->cap, first, seg, segments, radius, frame_dt_ps,
                                      ctx->diff_seg.p, ctx->diff_ncentral.p, ctx->diff_seg.p + segments,
                                      ctx->stream));
        double d = 0.0;
        int nc = 0;
        HIP_TRY(ctx, hipMemcpyAsync(&d, ctx->diff_seg.p + segments, sizeof(double), hipMemcpyDeviceToHost,
                                    ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(&nc, ctx->diff_ncentral.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (nc == 0) return fail(ctx, SCMD_EINVAL, "no atom within radius of the centre of mass");
        *D_A2_per_ps = d;
        *n_central = nc;
        return SCMD_OK;
    })
}

int scmd_get_forces_device(scmd_ctx *ctx, double *dev_out) {
    if (!ctx) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (!ctx->have_forces) return fail(ctx, SCMD_ESTATE, "compute or step first");
    if (!dev_out && ctx->natoms > 0) return fail(ctx, SCMD_EINVAL, "dev_out is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_aos_from4(ctx->f.p, dev_out, ctx->natoms, ctx->stream));
    return SCMD_OK;
}

int scmd_get_state(scmd_ctx *ctx, void *buf, size_t *bytes) {
    if (!ctx || !bytes) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    const size_t need = state_bytes(ctx);
    if (!buf) {
        *bytes = need;
        return SCMD_OK;
    }
    if (*bytes < need) return fail(ctx, SCMD_EINVAL, "buffer too small");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        char *p = (char *)buf;
        StateHeader h{};
        std::memcpy(h.magic, "SCMDSTA1", 8);
        h.version = 3;
        h.nclusters = ctx->nclusters;
        h.natoms = ctx->natoms;
        h.step = ctx->step;
        h.have_forces = ctx->have_forces ? 1 : 0;
        std::memcpy(p, &h, sizeof(h));
        p += sizeof(h);
        std::memcpy(p, ctx->offsets.data(), (ctx->nclusters + 1) * sizeof(int64_t));
        p += (ctx->nclusters + 1) * sizeof(int64_t);
        const size_t n4 = (size_t)ctx->natoms * sizeof(double4);
        if (ctx->natoms > 0) {
            HIP_TRY(ctx, hipMemcpy(p, ctx->rp.p, n4, hipMemcpyDeviceToHost));
            HIP_TRY(ctx, hipMemcpy(p + n4, ctx->v.p, n4, hipMemcpyDeviceToHost));
            HIP_TRY(ctx, hipMemcpy(p + 2 * n4, ctx->f.p, n4, hipMemcpyDeviceToHost));
            HIP_TRY(ctx, hipMemcpy(p + 3 * n4, ctx->rho.p, ctx->natoms * sizeof(double), hipMemcpyDeviceToHost));
        }
        p += 3 * n4 + (size_t)ctx->natoms * sizeof(double);
        std::memcpy(p, ctx->cdesc.data(), ctx->nclusters * sizeof(ClusterDesc));
        p += ctx->nclusters * sizeof(ClusterDesc);
        HIP_TRY(ctx, hipMemcpy(p, ctx->d_state.p, ctx->nclusters * sizeof(ClusterState), hipMemcpyDeviceToHost));
        p += ctx->nclusters * sizeof(ClusterState);
        std::memset(p, 0, (size_t)ctx->natoms * sizeof(double4));
        if (ctx->cells && ctx->plan_ok && ctx->neighbour == SCMD_CELLLIST)
            HIP_TRY(ctx, cell_list_get_ref(ctx->cells, (double4 *)p));
        *bytes = need;
        return SCMD_OK;
    })
}

int scmd_set_state(scmd_ctx *ctx, const void *buf, size_t bytes) {
    if (!ctx || !buf) return SCMD_EINVAL;
    if (!ctx->have_clusters) return fail(ctx, SCMD_ESTATE, "init_clusters first");
    if (bytes < sizeof(StateHeader)) return fail(ctx, SCMD_EINVAL, "blob too small");
    StateHeader h;
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, "SCMDSTA1", 8) != 0 || h.version != 3) return fail(ctx, SCMD_EINVAL, "not a state blob");
    if (h.nclusters != ctx->nclusters || h.natoms != ctx->natoms || bytes != state_bytes(ctx))
        return fail(ctx, SCMD_EINVAL, "blob has a different cluster layout");
    const char *p = (const char *)buf + sizeof(h);
    if (std::memcmp(p, ctx->offsets.data(), (ctx->nclusters + 1) * sizeof(int64_t)) != 0)
        return fail(ctx, SCMD_EINVAL, "blob has different cluster offsets");
    SCMD_GUARD({
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        p += (ctx->nclusters + 1) * sizeof(int64_t);
        const size_t n4 = (size_t)ctx->natoms * sizeof(double4);
        if (ctx->natoms > 0) {
            HIP_TRY(ctx, hipMemcpy(ctx->rp.p, p, n4, hipMemcpyHostToDevice));
            HIP_TRY(ctx, hipMemcpy(ctx->v.p, p + n4, n4, hipMemcpyHostToDevice));
            HIP_TRY(ctx, hipMemcpy(ctx->f.p, p + 2 * n4, n4, hipMemcpyHostToDevice));
            HIP_TRY(ctx, hipMemcpy(ctx->rho.p, p + 3 * n4, ctx->natoms * sizeof(double), hipMemcpyHostToDevice));
        }
        p += 3 * n4 + (size_t)ctx->natoms * sizeof(double);
        std::vector<ClusterDesc> cd(ctx->nclusters);
        std::memcpy(cd.data(), p, ctx->nclusters * sizeof(ClusterDesc));
        for (int k = 0; k < ctx->nclusters; ++k) {
            ctx->cdesc[k].kind = cd[k].kind;
            ctx->cdesc[k].T_start = cd[k].T_start;
            ctx->cdesc[k].T_end = cd[k].T_end;
            ctx->cdesc[k].tau = cd[k].tau;
            ctx->cdesc[k].ramp = cd[k].ramp;
            ctx->cdesc[k].gamma = cd[k].gamma;
            ctx->cdesc[k].seed = cd[k].seed;
            ctx->cdesc[k].ramp_origin = cd[k].ramp_origin;
        }
        p += ctx->nclusters * sizeof(ClusterDesc);
        HIP_TRY(ctx, hipMemcpy(ctx->d_state.p, p, ctx->nclusters * sizeof(ClusterState), hipMemcpyHostToDevice));
        p += ctx->nclusters * sizeof(ClusterState);
        if (ctx->plan_ok) HIP_TRY(ctx, upload_cdesc(ctx));
        drop_graph(ctx);
        if (ready(ctx) && ctx->neighbour == SCMD_CELLLIST) {
            // the cells and lists of the checkpointed run's last build, so
            // that stepping on repeats that run bit for bit
            int rc = ensure_plan(ctx);
            if (rc != SCMD_OK) return rc;
            bool have_ref = false;  // a blob of a context without a cell list holds zeros here
            for (size_t k = 0; k < 4 * (size_t)ctx->natoms && !have_ref; ++k) have_ref = ((const double *)p)[k] != 0.0;
            if (have_ref) {
                HIP_TRY(ctx, ctx->restore_scratch.ensure(std::max(ctx->natoms, 1)));
                HIP_TRY(ctx, cell_list_restore(ctx->cells, (const double4 *)p, ctx->restore_scratch.p, ctx->pc,
                                               ctx->precision, ctx->stream));
            } else {
                HIP_TRY(ctx, cell_list_invalidate(ctx->cells, ctx->stream));
            }
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        }
        ctx->step = h.step;
        ctx->have_forces = h.have_forces != 0;
        HIP_TRY(ctx, hipMemset(ctx->d_flag.p, 0, sizeof(int)));
        *ctx->h_flag = 0;
        return SCMD_OK;
    })
}

int scmd_set_profiling(scmd_ctx *ctx, int enable) {
    if (!ctx) return SCMD_EINVAL;
    ctx->profiling = enable ? 1 : 0;
    for (int k = 0; k < SCMD_KERNEL_COUNT; ++k) {
        ctx->prof_ms[k] = 0.0;
        ctx->prof_n[k] = 0;
    }
    return SCMD_OK;
}

int scmd_get_kernel_time(scmd_ctx *ctx, int kernel, double *avg_ms, int64_t *launches) {
    if (!ctx || !avg_ms) return SCMD_EINVAL;
    if (kernel < 0 || kernel >= SCMD_KERNEL_COUNT) return fail(ctx, SCMD_EINVAL, "unknown kernel class");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    harvest_events(ctx);
    *avg_ms = ctx->prof_n[kernel] > 0 ? ctx->prof_ms[kernel] / (double)ctx->prof_n[kernel] : 0.0;
    if (launches) *launches = ctx->prof_n[kernel];
    return SCMD_OK;
}

}  // extern "C"
