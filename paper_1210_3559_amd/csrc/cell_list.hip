// Cell-list sweeps for the truncated, shifted Sutton-Chen potential.
//
// The paper evaluates all pairs and calls a cutoff future work (Sec. 2,
// "Computational approach", last paragraphs); this variant truncates both
// power sums at rc and shifts them to zero there, and finds the pairs with
// r < rc through a cell list with a skin: cells of edge >= rl = rc + skin and
// per-atom lists of the candidates within rl, rebuilt once an atom has moved
// half the skin.
//
// Build (when due, every cluster independently, free boundaries):
//   bbox    per chunk of 1024 atoms of a cluster: min/max, merged per
//           cluster with 64-bit integer atomics on an order-preserving
//           encoding (exact, so the order does not matter);
//   count   per atom: the grid of its cluster, cells of edge h >= rc over
//           the box (h grows beyond rc only if the box would need more cells
//           than the cluster's cell capacity, so an escaping atom makes cells
//           coarser, never wrong); its cell; integer atomics count atoms per
//           cell (one atomic per cell and wavefront);
//   scan    exclusive prefix sum of the counts (one workgroup), which clears
//           the counts and resets the boxes for the next build;
//   scatter per atom: a slot in its cell (atomic cursor, again one atomic
//           per cell and wavefront);
//   order   per cell: every atom's slot becomes its rank by atom index, so
//           the cell-sorted order is deterministic; positions are gathered.
// Sweeps: one workgroup per cell (fullest cells first); the candidates of
// the 27 neighbouring cells (9 contiguous x-rows of the sorted arrays) are
// staged in LDS, and each wavefront takes the cell's atoms one at a time
// with its lanes across the candidates, testing them against rc before the
// pair terms.  Every atom's sum is complete after one sweep, so the sweep
// finishes its atoms itself (density: rho, P and the embedding energy; force:
// F and the kick), and the force sweep stores the cell's energy and v^2 sums,
// added in a fixed order, in the cell's slot of the per-cluster sums.
#include <algorithm>
#include <cmath>
#include <vector>

#include "cell_list.h"
#include "sweep_common.h"

namespace scmd {

struct CellGrid {
    double ox, oy, oz;  // origin (bounding-box minimum)
    double hx, hy, hz;  // cell edges (>= rc)
    int nx, ny, nz;     // cells per dimension this step
    int cx, cy, cz;     // per-dimension capacity
    int base;           // first cell of this cluster in the global cell arrays
    int off, n;         // atoms of the cluster
    int pad;
};

struct CellList {
    int nclusters = 0, natoms = 0, total_cap = 0;
    std::vector<int> cap_base, cap_n;  // per cluster: first cell and cell capacity (host)
    double rc = 0.0;
    double skin = 0.0;            // list margin: cells and lists cover rl = rc + skin
    double rl = 0.0;
    double4 *ref = nullptr;       // [natoms] positions at the last build (atom order)
    int *slot_of = nullptr;       // [natoms] atom -> its slot in the cell order of the last build
    int *flag = nullptr;          // [1] 1: the next force evaluation rebuilds the cells and lists
    unsigned long long *nbuilds = nullptr;  // [1] rebuilds since the plan
    CellGrid *grid = nullptr;     // [nclusters] this step's grids
    CellGrid *grid0 = nullptr;    // [nclusters] fixed fields (capacity, base, atoms)
    int *cell_cluster = nullptr;  // [total_cap]
    int *count = nullptr;         // [total_cap]
    int *start = nullptr;         // [total_cap + 1]
    int *cursor = nullptr;        // [total_cap]
    int *corder = nullptr;        // [total_cap] cells in the order the sweeps take them (fullest first)
    int *cell_of = nullptr;       // [natoms]
    int *perm = nullptr;          // cell slot -> atom, as scattered
    int *sperm = nullptr;         // cell slot -> atom, sorted by atom index within each cell
    long long *box = nullptr;     // [6 * nclusters] order-preserving encodings of min x,y,z, max x,y,z
    int4 *chunks = nullptr;       // bounding-box work: (cluster, first atom, end atom, -)
    int nchunks = 0;
    int *atom_cluster = nullptr;  // [natoms]
    double4 *rs = nullptr;        // sorted positions (density sweep; the force sweep reads P with them
                                  // from the density finish through sperm)
    uint16_t *nbr = nullptr;      // [natoms * kCellNbrCap] per sorted atom: staged candidates within rc
    int *nbr_n = nullptr;         // [natoms] number of such candidates (written by the density sweep)
    double *fin = nullptr;        // [4 * natoms] per sorted atom: the sweep's sums, read back by its finish
    double *emb = nullptr;        // [natoms] per sorted atom: embedding energy (density finish -> force finish)
};

namespace {

using namespace dev;

template <typename T>
hipError_t dalloc(T **p, size_t n) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

// ---------------------------------------------------------------------------
// Build kernels
// ---------------------------------------------------------------------------
constexpr int kBBoxBlock = 256;
constexpr int kBBoxChunk = 1024;  // atoms per bounding-box workgroup

// Partial bounding boxes and the check of the lists of the last build (see
// CellCheck), for evaluations whose positions no drift kernel checked: one
// workgroup per chunk of at most kBBoxChunk atoms of one cluster.
__global__ __launch_bounds__(kBBoxBlock) void k_cell_bbox(const int4 *__restrict__ chunks,
                                                          const double4 *__restrict__ rp, CellCheck cc) {
    __shared__ double sh[6 * (kBBoxBlock / 64)];
    const int4 ch = chunks[blockIdx.x];
    CellBox b;
    for (int i = ch.y + threadIdx.x; i < ch.z; i += kBBoxBlock) cell_check_atom(cc, i, rp[i], b);
    cell_check_merge<kBBoxBlock>(cc, ch.x, b, sh);
}

// Reset the bounding-box accumulators (min slots to +inf, max slots to -inf).
__global__ __launch_bounds__(64) void k_cell_box_reset(long long *__restrict__ box, int nclusters) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 6 * nclusters) return;
    box[k] = ord_encode((k % 6) < 3 ? INFINITY : -INFINITY);
}

// Cells of edge >= rc over a cluster's bounding box (h grows beyond rc only
// when the box needs more cells than the capacity).  g holds the fixed fields
// (capacity, base, atoms); the result adds origin, edges and cell counts.
__device__ __forceinline__ CellGrid grid_from_box(CellGrid g, const long long *__restrict__ b, double rc) {
    const int cap[3] = {g.cx, g.cy, g.cz};
    double o[3], h[3];
    int n[3];
    for (int d = 0; d < 3; ++d) {
        const double lo = ord_decode(b[d]), hi = ord_decode(b[3 + d]);
        const double ext = g.n > 0 ? hi - lo : 0.0;
        o[d] = g.n > 0 ? lo : 0.0;
        const double want = floor(ext / rc) + 1.0;
        if (!(want <= (double)cap[d])) {  // too many cells (or non-finite): coarser cells, edge still >= rc
            n[d] = cap[d];
            h[d] = ext / (double)(cap[d] - 1);
            if (!(h[d] >= rc)) h[d] = rc;
            if (!isfinite(h[d])) {
                n[d] = 1;
                h[d] = INFINITY;
            }
        } else {
            n[d] = (int)want;
            h[d] = rc;
        }
    }
    g.ox = o[0];
    g.oy = o[1];
    g.oz = o[2];
    g.hx = h[0];
    g.hy = h[1];
    g.hz = h[2];
    g.nx = n[0];
    g.ny = n[1];
    g.nz = n[2];
    return g;
}

__global__ __launch_bounds__(256) void k_cell_clear(int *__restrict__ count, int total) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < total) count[k] = 0;
}

__device__ __forceinline__ int cell_coord(double x, double o, double h, int n) {
    const double t = (x - o) / h;
    int i = t >= 0.0 ? (int)fmin(t, (double)(n - 1)) : 0;
    return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

// Lanes of a wavefront that land in the same cell share one atomic: the
// lowest such lane (the leader) adds their number to ctr[cell] and every lane
// of the group gets old value + its rank among them (by lane, i.e. by atom
// index).  Lanes with cell < 0 take no part.  The groups are found first
// (ballots only); then all leaders issue their atomics in one instruction, so
// the wavefront waits for one round trip.  Consecutive atoms are mostly close,
// so a wavefront touches few cells and the device-scope atomics drop
// several-fold.
template <bool RET>
__device__ __forceinline__ int wave_cell_add(int *__restrict__ ctr, int cell, int lane) {
    unsigned long long todo = __ballot(cell >= 0);
    const unsigned long long below = (1ull << lane) - 1ull;
    int leader = -1, rank = 0, size = 0;
    while (todo) {
        const int l = __builtin_ctzll(todo);
        const int lc = __builtin_amdgcn_readlane(cell, l);
        const unsigned long long same = __ballot(cell == lc);
        if (cell == lc) {
            leader = l;
            rank = __popcll(same & below);
            size = __popcll(same);
        }
        todo &= ~same;
    }
    if (!RET) {
        if (cell >= 0 && rank == 0) atomicAdd(&ctr[cell], size);
        return -1;
    }
    int base = 0;
    if (cell >= 0 && rank == 0) base = atomicAdd(&ctr[cell], size);
    base = __shfl(base, leader < 0 ? lane : leader, 64);
    return cell >= 0 ? base + rank : -1;
}

// Per atom: the grid of its cluster from this step's bounding box (every
// thread of a cluster computes the same grid; the cluster's first atom stores
// it for the sweeps), its cell, and the per-cell counts.  Thread t takes the
// atom at slot t of the previous build's cell order (prev), so the lanes of
// a wavefront mostly fall into a few cells and share their atomics even
// after the atoms have mixed (the atom order itself carries no locality in a
// liquid).
__global__ __launch_bounds__(256) void k_cell_count(const CellGrid *__restrict__ grid0, CellGrid *__restrict__ grid,
                                                    const long long *__restrict__ box, double rc,
                                                    const int *__restrict__ atom_cluster,
                                                    const double4 *__restrict__ rp, const int *__restrict__ prev,
                                                    int *__restrict__ cell_of, int *__restrict__ count, int natoms,
                                                    const int *__restrict__ flag) {
    if (*flag == 0) return;  // the lists of the last build still hold
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t < natoms ? prev[t] : natoms;
    int cell = -1;
    if (i < natoms) {
        const int c = atom_cluster[i];
        const CellGrid g = grid_from_box(grid0[c], box + 6 * c, rc);
        if (i == g.off) grid[c] = g;
        const double4 q = rp[i];
        const int ix = cell_coord(q.x, g.ox, g.hx, g.nx);
        const int iy = cell_coord(q.y, g.oy, g.hy, g.ny);
        const int iz = cell_coord(q.z, g.oz, g.hz, g.nz);
        cell = g.base + (iz * g.ny + iy) * g.nx + ix;
        cell_of[i] = cell;
    }
    (void)wave_cell_add<false>(count, cell, threadIdx.x & 63);
}

constexpr int kScanBlock = 1024;

constexpr int kOrderBins = 256;

// Exclusive prefix sum of count[0..total) into start[0..total] (and cursor),
// one workgroup: per-thread chunk sums, wavefront scans, a scan of the
// wavefront totals.  Also the order in which the sweeps take the cells:
// fullest first (a counting sort on the atom count, clamped at 255), so that
// the longest workgroups start first and the short ones fill in behind them
// (the order within one count depends on timing; each cell's sums do not
// depend on which workgroup takes it).  The counts are cleared behind the
// read and the bounding boxes reset, ready for the next build.
__global__ __launch_bounds__(kScanBlock) void k_cell_scan(int *__restrict__ count, int *__restrict__ start,
                                                          int *__restrict__ cursor, int *__restrict__ corder,
                                                          int total, long long *__restrict__ box, int nclusters,
                                                          const int *__restrict__ flag,
                                                          unsigned long long *__restrict__ nbuilds) {
    __shared__ int wsum[kScanBlock / 64];
    __shared__ int bins[kOrderBins];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (*flag == 0) {  // no build: only reset the boxes for the next check
        for (int k = t; k < 6 * nclusters; k += kScanBlock) box[k] = ord_encode((k % 6) < 3 ? INFINITY : -INFINITY);
        return;
    }
    if (t == 0) *nbuilds += 1ull;
    for (int q = t; q < kOrderBins; q += kScanBlock) bins[q] = 0;
    const int per = (total + kScanBlock - 1) / kScanBlock;
    const int a = min(total, t * per), b = min(total, a + per);
    int s = 0;
    for (int k = a; k < b; ++k) s += count[k];
    int x = s;  // inclusive scan over the wavefront
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
        int v = lane < kScanBlock / 64 ? wsum[lane] : 0;
#pragma unroll
        for (int d = 1; d < kScanBlock / 64; d <<= 1) {
            const int y = __shfl_up(v, d, 64);
            if (lane >= d) v += y;
        }
        if (lane < kScanBlock / 64) wsum[lane] = v;
    }
    __syncthreads();
    int run = x - s + (w > 0 ? wsum[w - 1] : 0);
    for (int k = a; k < b; ++k) {
        const int c = count[k];
        start[k] = run;
        cursor[k] = run;
        run += c;
        if (c == 0) {  // the empty cells (most of the capacity): one LDS atomic per wavefront
            const unsigned long long zm = __ballot(1);
            if (lane == __builtin_ctzll(zm)) atomicAdd(&bins[kOrderBins - 1], __popcll(zm));
        } else {
            atomicAdd(&bins[kOrderBins - 1 - min(c, kOrderBins - 1)], 1);
        }
    }
    if (t == kScanBlock - 1) start[total] = wsum[kScanBlock / 64 - 1];
    __syncthreads();
    if (w == 0) {  // exclusive scan of the bins, four per lane
        int v[4], sum = 0;
        for (int q = 0; q < 4; ++q) {
            v[q] = bins[4 * lane + q];
            sum += v[q];
        }
        int y = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(y, d, 64);
            if (lane >= d) y += u;
        }
        int e = y - sum;
        for (int q = 0; q < 4; ++q) {
            bins[4 * lane + q] = e;
            e += v[q];
        }
    }
    __syncthreads();
    for (int k = a; k < b; ++k) {
        const int c = count[k];
        int pos;
        if (c == 0) {
            const unsigned long long zm = __ballot(1);
            const int leader = __builtin_ctzll(zm);
            int b0 = 0;
            if (lane == leader) b0 = atomicAdd(&bins[kOrderBins - 1], __popcll(zm));
            pos = __builtin_amdgcn_readlane(b0, leader) +
                  __builtin_amdgcn_mbcnt_hi((unsigned)(zm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)zm, 0u));
        } else {
            pos = atomicAdd(&bins[kOrderBins - 1 - min(c, kOrderBins - 1)], 1);
        }
        corder[pos] = k;
        count[k] = 0;
    }
    for (int k = t; k < 6 * nclusters; k += kScanBlock) box[k] = ord_encode((k % 6) < 3 ? INFINITY : -INFINITY);
}

// Per atom, in the previous build's cell order as for the counts: a slot in
// its cell (which slot depends on timing; k_cell_order ranks them).
__global__ __launch_bounds__(256) void k_cell_scatter(const int *__restrict__ cell_of, const int *__restrict__ prev,
                                                      int *__restrict__ cursor, int *__restrict__ perm, int natoms,
                                                      const int *__restrict__ flag) {
    if (*flag == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t < natoms ? prev[t] : natoms;
    const int cell = i < natoms ? cell_of[i] : -1;
    const int slot = wave_cell_add<true>(cursor, cell, threadIdx.x & 63);
    if (i < natoms) perm[slot] = i;
}

// One wavefront per cell: the slot of each atom is its rank (the number of
// atoms of the cell with a smaller index), so sperm lists every cell's atoms
// in index order whatever order the atomic scatter produced; the sorted
// positions are gathered at the same time.  Cells larger than the LDS buffer
// (only after an atom escaped and the cells coarsened) rank from global
// memory.
constexpr int kOrderLds = 1024;

__global__ __launch_bounds__(64) void k_cell_order(const int *__restrict__ start, const int *__restrict__ perm,
                                                   int *__restrict__ sperm, const double4 *__restrict__ rp,
                                                   double4 *__restrict__ rs, double4 *__restrict__ ref,
                                                   int *__restrict__ slot_of, const int *__restrict__ flag) {
    __shared__ int sh[kOrderLds];
    if (*flag == 0) return;
    const int a = start[blockIdx.x], n = start[blockIdx.x + 1] - a;
    if (n == 0) return;
    const bool local = n <= kOrderLds;
    if (local) {
        for (int k = threadIdx.x; k < n; k += 64) sh[k] = perm[a + k];
        __syncthreads();
    }
    const int *src = local ? sh : perm + a;
    for (int k = threadIdx.x; k < n; k += 64) {
        const int v = src[k];
        int rank = 0;
        for (int q = 0; q < n; ++q) rank += src[q] < v ? 1 : 0;
        sperm[a + rank] = v;
        slot_of[v] = a + rank;
        const double4 q = rp[v];
        rs[a + rank] = q;
        ref[v] = q;
    }
}

// ---------------------------------------------------------------------------
// Sweeps
// ---------------------------------------------------------------------------
// One workgroup of kCellWaves wavefronts per cell, the cells taken in the
// scan's order (fullest first).  The cell's 27-cell neighbourhood is 9
// x-rows, each contiguous in the sorted arrays; their atoms (the candidates,
// concatenated row after row) are staged in LDS when they fit.  Wavefront w
// takes the cell's atoms w, w + kCellWaves, ... one at a time; for each, its
// lanes test the candidates against rc, the hits go through a queue to full
// passes of the pair terms (the force sweep reads the hits the density sweep
// stored), and a fixed-order DPP reduction adds the 64 lane sums.  The hits
// and their order depend only on the positions, so every atom's sum has one
// order whatever the launch (deterministic).  The atom itself sits in the own
// row at one known candidate index (the self pair).  Neighbourhoods larger
// than the LDS buffer (only when cells coarsened after an atom escaped) read
// every candidate from global memory and mask the pairs beyond rc.
constexpr int kCellWaves = 16;
constexpr int kCellStage = 2240;  // staged candidates (70 KiB + the queues: two workgroups per CU)
constexpr int kCellQueue = 128;   // in-range candidates queued per wavefront (< 64 left + 64 new)
constexpr int kCellNbrCap = 512;  // listed candidates within rc per atom (an atom with more re-tests)

template <int PREC, bool GEN, bool FORCE>
__global__ __launch_bounds__(64 * kCellWaves) void k_cell_sweep(const CellGrid *__restrict__ grid,
                                                                const int *__restrict__ corder,
                                                                const int *__restrict__ cell_cluster,
                                                                const int *__restrict__ start,
                                                                const double4 *__restrict__ rs,
                                                                const int *__restrict__ sperm,
                                                                double *__restrict__ fin,
                                                                double *__restrict__ emb,
                                                                uint16_t *__restrict__ nbr,
                                                                int *__restrict__ nbr_n,
                                                                const double4 *__restrict__ xp, PotConst pc,
                                                                int *__restrict__ flag, double rl2,
                                                                DensityOut dout, ForceOut fout, int finish) {
    constexpr int Q = FORCE ? 4 : 1;
    // staged candidates as four arrays (x, y, z, w): lanes reading
    // consecutive candidates touch consecutive 8-byte words, conflict-free
    extern __shared__ double lds_c[];
    double *const lx = lds_c, *const ly = lds_c + kCellStage, *const lz = lds_c + 2 * kCellStage,
                  *const lw = lds_c + 3 * kCellStage;
    __shared__ int seg_lo[9], seg_len[9], seg_off[10];
    __shared__ int queue[kCellWaves][kCellQueue];
    // A density sweep after a (re)build lists every atom's candidates within
    // rl = rc + skin while it runs; until the next build both sweeps read
    // those lists.  The force sweep ends the build (no later kernel of this
    // evaluation reads the flag).
    const bool build = !FORCE && *flag != 0;
    if (FORCE && blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
    const int cell = corder[blockIdx.x];
    const CellGrid g = grid[cell_cluster[cell]];
    const int local = cell - g.base;
    const int s0 = start[cell], cnt = local < g.nx * g.ny * g.nz ? start[cell + 1] - s0 : 0;
    // the cell's slot of the cluster sums (embedding energy, pair energy,
    // v^2), stored by the force sweep; cells without atoms, also those
    // beyond this build's grid, hold zeros
    if (cnt == 0) {  // uniform per workgroup
        if (FORCE && finish && threadIdx.x == 0) {
            double *const cell_sums = fout.tile_sums + (size_t)cell * kTileSums;
            cell_sums[0] = 0.0;
            cell_sums[1] = 0.0;
            cell_sums[2] = 0.0;
        }
        return;
    }
    const int ix = local % g.nx, iy = (local / g.nx) % g.ny, iz = local / (g.nx * g.ny);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 9) {
        const int jz = iz + tid / 3 - 1, jy = iy + tid % 3 - 1;
        int ja = 0, jb = 0;
        if (jz >= 0 && jz < g.nz && jy >= 0 && jy < g.ny) {
            const int row = g.base + (jz * g.ny + jy) * g.nx;
            ja = start[row + max(ix - 1, 0)];
            jb = start[row + min(ix + 1, g.nx - 1) + 1];
        }
        seg_lo[tid] = ja;
        seg_len[tid] = jb - ja;
    }
    __syncthreads();
    if (tid == 0) {
        seg_off[0] = 0;
        for (int r = 0; r < 9; ++r) seg_off[r + 1] = seg_off[r] + seg_len[r];
    }
    __syncthreads();
    const int M = __builtin_amdgcn_readfirstlane(seg_off[9]);
    const int M64 = (M + 63) & ~63;  // candidates padded to whole wavefronts
    const bool staged = M64 <= kCellStage;
    // sorted atom of candidate p (p < M)
    auto cand = [&](int p) {
        int r = 0;
        while (p >= seg_off[r + 1]) ++r;
        return seg_lo[r] + (p - seg_off[r]);
    };
    // the record of sorted atom k: position (density sweep), position and P
    // from the density sweep's finish (force sweep)
    auto rec = [&](int k) { return FORCE ? xp[sperm[k]] : rs[k]; };
    if (staged) {
        for (int p = tid; p < M; p += 64 * kCellWaves) {
            const double4 q = rec(cand(p));
            lx[p] = q.x;
            ly[p] = q.y;
            lz[p] = q.z;
            lw[p] = q.w;
        }
        // padding: far away, so r^2 is +inf and never within rc
        for (int p = M + tid; p < M64; p += 64 * kCellWaves) {
            lx[p] = 1.0e300;
            ly[p] = 1.0e300;
            lz[p] = 1.0e300;
            lw[p] = 0.0;
        }
    }
    __syncthreads();
    const float Af = (float)pc.A;
    // the own cell lies in the own row (segment 4): atom k is candidate
    // seg_off[4] + (k - seg_lo[4])
    const int self0 = seg_off[4] - seg_lo[4];
    for (int a = wave; a < cnt; a += kCellWaves) {
        const int k = s0 + a;
        const double4 qi = rec(k);
        const double c_i = -qi.w;
        const float cif = (float)c_i;
        const int self_p = self0 + k;
        double acc[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q] = 0.0;
        // the pair terms of one candidate (self or void when `off`)
        auto staged_cand = [&](int p) { return make_double4(lx[p], ly[p], lz[p], lw[p]); };
        auto pair_terms = [&](const double4 &q, bool off) {
            if constexpr (FORCE)
                force_pair<PREC, GEN, true, true>(qi.x - q.x, qi.y - q.y, qi.z - q.z, off, c_i, q.w, cif,
                                                  (float)q.w, acc[0], acc[1], acc[2], acc[3], pc, Af);
            else
                density_pair<PREC, GEN, true, true>(qi.x - q.x, qi.y - q.y, qi.z - q.z, off, acc[0], pc);
        };
        uint16_t *const list = nbr + (size_t)k * kCellNbrCap;
        const int listed = !build && staged ? __builtin_amdgcn_readfirstlane(nbr_n[k]) : -1;
        if (!build && staged && listed <= kCellNbrCap) {
            // the density sweep of the last build listed the candidates
            // within rl (same cells; no atom has moved half the skin since,
            // so every pair now closer than rc is among them); lanes take the
            // entries in the order the queue below handed them out
            for (int base = 0; base < listed; base += 64) {
                const bool v = base + lane < listed;
                const int e = list[v ? base + lane : base];  // in bounds for every lane
                pair_terms(staged_cand(v ? e : 0), !v);
            }
        } else if (staged) {
            // Only about a fifth of the candidates lie within rc.  A first pass
            // tests r^2 < rt^2 and queues the hits (ring buffer per
            // wavefront); every 64 queued hits make one pass of the pair
            // terms with all lanes busy.  The pair terms apply the cutoff
            // themselves.  On a build the test radius is rl and the density
            // sweep stores the hits as they leave the queue (up to kCellNbrCap
            // per atom, one coalesced store per 64) for the sweeps until the
            // next build; otherwise (an atom whose list overflowed) it is rc
            // with the pair terms' own expression, so no pair changes side.
            const double rt2 = build ? rl2 : pc.rc2;
            int *qu = queue[wave];
            int head = 0, qn = 0, total = 0;  // wavefront-uniform
            for (int base = 0; base < M64; base += 64) {
                const int p = base + lane;
                const double dx = qi.x - lx[p], dy = qi.y - ly[p], dz = qi.z - lz[p];
                const bool in =
                    (__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)) < rt2) & (lane != self_p - base);
                const unsigned long long hit = __ballot(in);
                const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(hit >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((unsigned)hit, 0u));
                if (in) qu[(head + qn + rank) & (kCellQueue - 1)] = p;
                qn += __popcll(hit);
                if (qn >= 64) {
                    __builtin_amdgcn_wave_barrier();
                    const int e = qu[(head + lane) & (kCellQueue - 1)];
                    head = (head + 64) & (kCellQueue - 1);
                    qn -= 64;
                    if (build && total + 64 <= kCellNbrCap) list[total + lane] = (uint16_t)e;
                    total += 64;
                    pair_terms(staged_cand(e), false);
                }
            }
            if (qn > 0) {
                __builtin_amdgcn_wave_barrier();
                const bool v = lane < qn;
                // lanes past the queue read candidate 0 (valid: the own cell
                // is not empty) and add nothing
                const int e = v ? qu[(head + lane) & (kCellQueue - 1)] : 0;
                if (build && v && total + lane < kCellNbrCap) list[total + lane] = (uint16_t)e;
                total += qn;
                pair_terms(staged_cand(e), !v);
            }
            if (build && lane == 0) nbr_n[k] = total;
        } else {
#pragma unroll 2
            for (int p = lane; p < M; p += 64) pair_terms(staged ? staged_cand(p) : rec(cand(p)), p == self_p);
        }
        if constexpr (FORCE) unscale_force<PREC, GEN>(acc[0], acc[1], acc[2], acc[3]);
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q] = wave_total(acc[q]);
        if (lane == 0 && finish) {
#pragma unroll
            for (int q = 0; q < Q; ++q) fin[(size_t)k * 4 + q] = acc[q];
        }
    }
    if (!finish) return;
    // Finish: thread a takes the cell's atoms a, a + 1024, ... (their sums,
    // stored above by the wavefronts of this workgroup, are visible after
    // the barrier), so the loads of the per-atom epilogue are issued once per
    // cell rather than on every wavefront's path.
    __syncthreads();
    if constexpr (!FORCE) {
        // the embedding energies wait per sorted atom for the force sweep,
        // which adds them into the cell's sums (no reduction here: it would
        // hold every wavefront of the cell until the finish is done)
        for (int a = tid; a < cnt; a += 64 * kCellWaves) {
            const int k = s0 + a;
            emb[k] = density_atom(sperm[k], fin[(size_t)k * 4], dout, pc);
        }
    } else {
        // the cell's sums: each wavefront's in a fixed order (DPP), then the
        // wavefronts' in order
        double se = 0.0, sp = 0.0, sv = 0.0;
        for (int a = tid; a < cnt; a += 64 * kCellWaves) {
            const int k = s0 + a;
            const double *t = fin + (size_t)k * 4;
            se += emb[k];
            force_atom(sperm[k], t[0], t[1], t[2], t[3], fout, pc, sp, sv);
        }
        se = wave_total(se);
        sp = wave_total(sp);
        sv = wave_total(sv);
        __shared__ double wsh[3][kCellWaves];
        if (lane == 0) {
            wsh[0][wave] = se;
            wsh[1][wave] = sp;
            wsh[2][wave] = sv;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double e = 0.0, p = 0.0, v2 = 0.0;
            for (int w = 0; w < kCellWaves; ++w) {
                e += wsh[0][w];
                p += wsh[1][w];
                v2 += wsh[2][w];
            }
            double *const cell_sums = fout.tile_sums + (size_t)cell * kTileSums;
            cell_sums[0] = e;
            cell_sums[1] = p;
            cell_sums[2] = v2;
        }
    }
}

template <bool FORCE>
hipError_t launch_cell_sweep(CellList *cl, const double4 *xp, const DensityOut &dout, const ForceOut &fout,
                             int finish, const PotConst &pc, int precision, hipStream_t s) {
    (void)hipGetLastError();
    const dim3 grid(cl->total_cap), block(64 * kCellWaves);
    const size_t lds = kCellStage * sizeof(double4);
#define SCMD_CELL_ARGS                                                                                          \
    cl->grid, cl->corder, cl->cell_cluster, cl->start, cl->rs, cl->sperm, cl->fin, cl->emb, cl->nbr, cl->nbr_n, xp, \
        pc, cl->flag, cl->rl * cl->rl, dout, fout, finish
    if (precision == SCMD_FP64) {
        if (pc.generic)
            hipLaunchKernelGGL((k_cell_sweep<SCMD_FP64, true, FORCE>), grid, block, lds, s, SCMD_CELL_ARGS);
        else
            hipLaunchKernelGGL((k_cell_sweep<SCMD_FP64, false, FORCE>), grid, block, lds, s, SCMD_CELL_ARGS);
    } else {
        if (pc.generic)
            hipLaunchKernelGGL((k_cell_sweep<SCMD_MIXED, true, FORCE>), grid, block, lds, s, SCMD_CELL_ARGS);
        else
            hipLaunchKernelGGL((k_cell_sweep<SCMD_MIXED, false, FORCE>), grid, block, lds, s, SCMD_CELL_ARGS);
    }
#undef SCMD_CELL_ARGS
    return hipGetLastError();
}

}  // namespace

bool cell_list_available() { return true; }

CellList *cell_list_create() {
    try {
        return new CellList();
    } catch (...) {
        return nullptr;
    }
}

void cell_list_destroy(CellList *cl) {
    if (!cl) return;
    void *ptrs[] = {cl->grid0, cl->grid,  cl->cell_cluster, cl->count,  cl->start, cl->cursor,
                    cl->cell_of, cl->perm, cl->sperm, cl->box, cl->chunks,
                    cl->atom_cluster, cl->rs, cl->nbr, cl->nbr_n, cl->corder, cl->ref,
                    cl->slot_of, cl->flag, cl->nbuilds, cl->fin, cl->emb};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete cl;
}

// The sweeps stage more than the default 64 KiB of dynamic LDS: raise each
// instantiation's limit (once per plan, outside any graph capture).
static hipError_t set_cell_sweep_lds() {
    const int lds = (int)(kCellStage * sizeof(double4));
    const void *fns[] = {reinterpret_cast<const void *>(k_cell_sweep<SCMD_FP64, false, false>),
                         reinterpret_cast<const void *>(k_cell_sweep<SCMD_FP64, false, true>),
                         reinterpret_cast<const void *>(k_cell_sweep<SCMD_FP64, true, false>),
                         reinterpret_cast<const void *>(k_cell_sweep<SCMD_FP64, true, true>),
                         reinterpret_cast<const void *>(k_cell_sweep<SCMD_MIXED, false, false>),
                         reinterpret_cast<const void *>(k_cell_sweep<SCMD_MIXED, false, true>),
                         reinterpret_cast<const void *>(k_cell_sweep<SCMD_MIXED, true, false>),
                         reinterpret_cast<const void *>(k_cell_sweep<SCMD_MIXED, true, true>)};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t cell_list_plan(CellList *cl, int nclusters, const int64_t *offsets, double rc, double skin,
                          const double4 *rp_dev) {
    if (hipError_t e0 = set_cell_sweep_lds(); e0 != hipSuccess) return e0;
    const int natoms = (int)offsets[nclusters];
    cl->nclusters = nclusters;
    cl->natoms = natoms;
    cl->rc = rc;
    cl->skin = skin;
    cl->rl = rc + skin;
    rc = cl->rl;  // cells cover the list radius
    std::vector<double4> r(natoms);
    hipError_t e;
    if (natoms > 0 && (e = hipMemcpy(r.data(), rp_dev, natoms * sizeof(double4), hipMemcpyDeviceToHost)) != hipSuccess)
        return e;
    // cell capacity per cluster: the cells of the initial box per dimension
    // plus four (room for the cluster to expand by about two cells on each
    // side before the grid coarsens), at most 1024
    std::vector<CellGrid> grids(nclusters);
    std::vector<int> cell_cluster;
    cl->cap_base.assign(nclusters, 0);
    cl->cap_n.assign(nclusters, 0);
    int base = 0;
    for (int c = 0; c < nclusters; ++c) {
        CellGrid g{};
        g.off = (int)offsets[c];
        g.n = (int)(offsets[c + 1] - offsets[c]);
        double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int i = g.off; i < g.off + g.n; ++i) {
            const double v[3] = {r[i].x, r[i].y, r[i].z};
            for (int d = 0; d < 3; ++d) {
                if (i == g.off || v[d] < lo[d]) lo[d] = v[d];
                if (i == g.off || v[d] > hi[d]) hi[d] = v[d];
            }
        }
        int cap[3];
        for (int d = 0; d < 3; ++d) {
            const int n0 = (int)std::floor((hi[d] - lo[d]) / rc) + 1;
            cap[d] = std::min(n0 + 4, 1024);
        }
        g.cx = cap[0];
        g.cy = cap[1];
        g.cz = cap[2];
        g.nx = g.ny = g.nz = 1;
        g.hx = g.hy = g.hz = rc;
        g.base = base;
        const int ncap = cap[0] * cap[1] * cap[2];
        cl->cap_base[c] = base;
        cl->cap_n[c] = ncap;
        cell_cluster.insert(cell_cluster.end(), ncap, c);
        base += ncap;
        grids[c] = g;
    }
    cl->total_cap = base;
    std::vector<int4> chunks;
    for (int c = 0; c < nclusters; ++c)
        for (int a = (int)offsets[c]; a < (int)offsets[c + 1]; a += kBBoxChunk)
            chunks.push_back(make_int4(c, a, std::min<int>(a + kBBoxChunk, (int)offsets[c + 1]), 0));
    cl->nchunks = (int)chunks.size();
    std::vector<int> ac(natoms);
    for (int c = 0; c < nclusters; ++c)
        for (int i = (int)offsets[c]; i < (int)offsets[c + 1]; ++i) ac[i] = c;
    if ((e = dalloc(&cl->grid, nclusters)) != hipSuccess) return e;
    if ((e = dalloc(&cl->grid0, nclusters)) != hipSuccess) return e;
    if ((e = dalloc(&cl->cell_cluster, base)) != hipSuccess) return e;
    if ((e = dalloc(&cl->count, base)) != hipSuccess) return e;
    if ((e = dalloc(&cl->start, base + 1)) != hipSuccess) return e;
    if ((e = dalloc(&cl->cursor, base)) != hipSuccess) return e;
    if ((e = dalloc(&cl->corder, base)) != hipSuccess) return e;
    if ((e = dalloc(&cl->cell_of, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->perm, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->sperm, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->box, 6 * nclusters)) != hipSuccess) return e;
    if ((e = dalloc(&cl->chunks, chunks.size())) != hipSuccess) return e;
    if (!chunks.empty() &&
        (e = hipMemcpy(cl->chunks, chunks.data(), chunks.size() * sizeof(int4), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_cell_box_reset, dim3((6 * nclusters + 63) / 64), dim3(64), 0, 0, cl->box, nclusters);
    // the counts start at zero; each build's scan clears them again
    if (base > 0) hipLaunchKernelGGL(k_cell_clear, dim3((base + 255) / 256), dim3(256), 0, 0, cl->count, base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
    if ((e = dalloc(&cl->atom_cluster, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->rs, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->nbr, (size_t)natoms * kCellNbrCap)) != hipSuccess) return e;
    if ((e = dalloc(&cl->nbr_n, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->fin, 4 * (size_t)natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->emb, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->ref, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->slot_of, natoms)) != hipSuccess) return e;
    if ((e = dalloc(&cl->flag, 1)) != hipSuccess) return e;
    if ((e = dalloc(&cl->nbuilds, 1)) != hipSuccess) return e;
    if ((e = hipMemset(cl->nbuilds, 0, sizeof(unsigned long long))) != hipSuccess) return e;
    {
        const int one = 1;  // the first evaluation builds
        if ((e = hipMemcpy(cl->flag, &one, sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) return e;
    }
    if (natoms > 0 && (e = hipMemset(cl->ref, 0, natoms * sizeof(double4))) != hipSuccess) return e;
    if ((e = hipMemcpy(cl->grid, grids.data(), nclusters * sizeof(CellGrid), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if ((e = hipMemcpy(cl->grid0, grids.data(), nclusters * sizeof(CellGrid), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if (base > 0 &&
        (e = hipMemcpy(cl->cell_cluster, cell_cluster.data(), base * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if (natoms > 0) {
        // before the first build the "previous cell order" is the atom order
        std::vector<int> ident(natoms);
        for (int i = 0; i < natoms; ++i) ident[i] = i;
        if ((e = hipMemcpy(cl->sperm, ident.data(), natoms * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        if ((e = hipMemcpy(cl->slot_of, ident.data(), natoms * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        if ((e = hipMemcpy(cl->atom_cluster, ac.data(), natoms * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// rebuild once an atom has moved half the skin (every step without one)
static double check_thr2(const CellList *cl) {
    const double half = 0.5 * cl->skin;
    return cl->skin > 0.0 ? half * half : -1.0;
}

CellCheck cell_list_check(CellList *cl) {
    return CellCheck{cl->ref, cl->slot_of, cl->rs, cl->box, cl->flag, check_thr2(cl)};
}

hipError_t cell_list_build(CellList *cl, const double4 *rp, bool checked, hipStream_t s) {
    (void)hipGetLastError();
    const int na = cl->natoms, tc = cl->total_cap;
    const double thr2 = check_thr2(cl);
    if (!checked && cl->nchunks > 0) {
        const CellCheck cc{cl->ref, cl->slot_of, cl->rs, cl->box, cl->flag, thr2};
        hipLaunchKernelGGL(k_cell_bbox, dim3(cl->nchunks), dim3(kBBoxBlock), 0, s, cl->chunks, rp, cc);
    }
    if (na > 0)
        hipLaunchKernelGGL(k_cell_count, dim3((na + 255) / 256), dim3(256), 0, s, cl->grid0, cl->grid, cl->box, cl->rl,
                           cl->atom_cluster, rp, cl->sperm, cl->cell_of, cl->count, na, cl->flag);
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(kScanBlock), 0, s, cl->count, cl->start, cl->cursor, cl->corder, tc,
                       cl->box, cl->nclusters, cl->flag, cl->nbuilds);
    if (na > 0)
        hipLaunchKernelGGL(k_cell_scatter, dim3((na + 255) / 256), dim3(256), 0, s, cl->cell_of, cl->sperm, cl->cursor,
                           cl->perm, na, cl->flag);
    // count and scatter read the previous build's order from sperm before
    // k_cell_order replaces it
    hipLaunchKernelGGL(k_cell_order, dim3(tc), dim3(64), 0, s, cl->start, cl->perm, cl->sperm, rp, cl->rs, cl->ref,
                       cl->slot_of, cl->flag);
    return hipGetLastError();
}

// flag values copied to the device (static: an asynchronous copy may read
// them after the call returns)
static const int kFlagSet = 1, kFlagClear = 0;

hipError_t cell_list_invalidate(CellList *cl, hipStream_t s) {
    return hipMemcpyAsync(cl->flag, &kFlagSet, sizeof(int), hipMemcpyHostToDevice, s);
}

hipError_t cell_list_rebuilds(CellList *cl, int64_t *out) {
    unsigned long long n = 0;
    hipError_t e = hipMemcpy(&n, cl->nbuilds, sizeof(n), hipMemcpyDeviceToHost);
    if (e == hipSuccess) *out = (int64_t)n;
    return e;
}

hipError_t cell_list_get_ref(CellList *cl, double4 *host_out) {
    if (cl->natoms == 0) return hipSuccess;
    return hipMemcpy(host_out, cl->ref, cl->natoms * sizeof(double4), hipMemcpyDeviceToHost);
}

hipError_t cell_list_restore(CellList *cl, const double4 *ref_host, double4 *scratch_dev, const PotConst &pc,
                             int precision, hipStream_t s) {
    if (cl->natoms == 0) return cell_list_invalidate(cl, s);
    hipError_t e = hipMemcpyAsync(scratch_dev, ref_host, cl->natoms * sizeof(double4), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    // cells and lists of the positions of the last build, as that build made
    // them: a build forced from those positions, then a density sweep that
    // lists the candidates and finishes no atom
    if ((e = cell_list_invalidate(cl, s)) != hipSuccess) return e;
    if ((e = cell_list_build(cl, scratch_dev, false, s)) != hipSuccess) return e;
    if ((e = launch_cell_sweep<false>(cl, nullptr, DensityOut{}, ForceOut{}, 0, pc, precision, s)) != hipSuccess)
        return e;
    // the density sweep left the flag set: clear it (the lists hold)
    return hipMemcpyAsync(cl->flag, &kFlagClear, sizeof(int), hipMemcpyHostToDevice, s);
}

hipError_t cell_list_density(CellList *cl, const SweepBuffers &B, const PotConst &pc, int precision,
                             hipStream_t s) {
    const DensityOut o{B.rp, B.xp, B.rho, B.tile_sums};
    return launch_cell_sweep<false>(cl, nullptr, o, ForceOut{}, 1, pc, precision, s);
}

hipError_t cell_list_force(CellList *cl, const SweepBuffers &B, const StepArgs &a, const PotConst &pc,
                           int precision, hipStream_t s) {
    const ForceOut fo{B.f, B.v, B.tile_sums, a.h, a.advance};
    return launch_cell_sweep<true>(cl, B.xp, DensityOut{}, fo, 1, pc, precision, s);
}

void cell_list_sum_slots(const CellList *cl, int cluster, int *first, int *count) {
    *first = cl->cap_base[cluster];
    *count = cl->cap_n[cluster];
}

int cell_list_total_slots(const CellList *cl) { return cl->total_cap; }

}  // namespace scmd
