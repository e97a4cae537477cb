// Internal declarations shared by the host runtime and the HIP kernels of
// the Sutton-Chen cluster-MD library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scmd {

// 1 u*A^2/fs^2 in eV (CODATA 2018 e and u) and k_B in eV/K.
constexpr double kEvPerUA2Fs2 = 103.64269652680505;
constexpr double kBoltzmannEv = 8.617333262145179e-05;

// Sentinel coordinates for lanes/atoms past the end of a tile.  Atom slots
// past the owned range sit at -kFar, j slots past a chunk at +kFar, so every
// pair touching a sentinel has r^2 ~ 1e301: all its power terms underflow to
// exactly zero in double precision (and to inf -> 0 through rsqrt/rcp in
// single precision), and no sentinel ever meets another at r = 0.
constexpr double kFar = 1.0e150;

// Sutton-Chen constants folded for the kernels.  With u = 1/r:
//   rho_i      = a^m sum_j u^m                      (density sweep)
//   F_i        = sum_j u^(m+2) [A u^(n-m) - P_i - P_j] (r_i - r_j)
//                with A = eps n a^n and P_k = eps (c m / 2) a^m psi_k,
//   E_pair_i   = (eps/2) a^n sum_j u^n,  E_emb_i = -eps c sqrt(rho_i).
// Cutoff variant: shifted powers (a/r)^k - (a/rc)^k for r < rc.
struct PotConst {
    double am;        // a^m
    double A;         // eps * n * a^n
    double Pscale;    // eps * c * m / 2 * a^m   (P_k = Pscale * psi_k)
    double half_eps_an;  // eps/2 * a^n
    double eps_c;     // eps * c
    double rc2;       // rc^2 (0: all pairs)
    double inv_rc_m;  // rc^-m  (shift of u^m)
    double inv_rc_n;  // rc^-n  (shift of u^n)
    double A8;        // A / 8          (force term evaluated with 2u, (n, m) = (9, 6))
    double inv_rc_n512;  // 512 rc^-n   (shift of (2u)^9)
    int n, m;
    int cut;          // 1 when rc > 0
    int generic;      // 1 unless (n, m) == (9, 6)
};

// One cluster of a batch (device table).
struct ClusterDesc {
    int32_t off;        // first atom
    int32_t n;          // atoms
    int32_t tile0;      // first atom tile
    int32_t ntiles;     // atom tiles
    int64_t ndof;
    int32_t kind;       // thermostat kind
    int32_t pad;
    double T_start, T_end, tau;
    int64_t ramp;
    double gamma;       // Langevin damping constant, 1/ps
    double bath_c1;     // Langevin exp(-gamma dt) (set by the host for the current dt)
    uint64_t seed;      // Langevin noise key
    int64_t ramp_origin;  // step count at which the temperature ramp starts
};

// Mutable per-cluster state (device).
struct ClusterState {
    double lambda;      // thermostat factor not yet applied to the velocities
    double epot, ekin, temp, ttarget;
    int64_t step;       // completed steps
    int32_t nonfinite;
    int32_t pad;
};

// A pair-sweep work item: atoms [i0, i0+ni) of tile `tile` against j in
// [j0, j1), partial sums written to slot `slot`.
struct SweepItem {
    int32_t c, i0, ni, j0, j1, slot, tile, pad;
};

// An atom tile: atoms [i0, i0+ni) of cluster c whose partial sums sit in
// slots [first, first+nsplit).
struct ITile {
    int32_t c, i0, ni, first, nsplit, pad;
};

// Launch shapes of the all-pairs sweeps: (IPT atoms per lane, WI waves along
// i, WJ waves along j).  Tile = 64*IPT*WI atoms, block = 64*WI*WJ threads.
#define SCMD_SWEEP_SHAPES(X) \
    X(1, 4, 1)               \
    X(2, 4, 1)               \
    X(1, 2, 2)               \
    X(2, 2, 2)               \
    X(1, 1, 4)               \
    X(2, 1, 4)               \
    X(1, 2, 4)               \
    X(2, 2, 4)               \
    X(1, 4, 4)               \
    X(1, 1, 8)               \
    X(2, 1, 8)               \
    X(1, 2, 8)               \
    X(1, 1, 16)              \
    X(4, 1, 2)               \
    X(4, 1, 4)               \
    X(4, 2, 2)

struct SweepLaunch {
    const SweepItem *items;
    const int32_t *order;
    const ITile *tiles;
    int nitems;
    int ipt, wi, wj;
};

struct SweepBuffers {
    const double4 *rp;  // positions (drift output)
    double4 *xp;        // positions + P (density output, force input)
    double4 *f;
    double4 *v;
    double *rho;
    double *part;       // partial sums, slot-major
    double *tile_sums;  // kTileSums doubles per tile
    double2 *dpv;       // row sweeps of one cluster: drift inputs (p = r + dt h F, v), 3 pairs per atom
};

// The cell list's per-step check, run by whichever kernel last moved the
// atoms: an atom that has moved more than half the skin since the last
// build (|r - ref|^2 > thr2; thr2 < 0: every step) sets *flag; the
// positions are copied into that build's cell order (rs[slot_of[i]]); the
// cluster's bounding box is merged into box (6 order-preserving encodings
// per cluster: min x, y, z, max x, y, z).
struct CellCheck {
    const double4 *ref;
    const int *slot_of;
    double4 *rs;
    long long *box;
    int *flag;
    double thr2;
};

struct StepArgs {
    const ClusterDesc *cd;
    ClusterState *st;
    int *flag;          // non-finite flag
    double mass_u, dt, h;
    int advance;        // 1: kick + thermostat (second half of a step); 0: evaluate only
    int energy;         // 1: accumulate the pair energy (symmetric and row force sweeps skip it otherwise)
};

// Pair sweeps.  Tiles whose partner range is one item are finished inside
// the sweep; when any tile is split (has_split), the matching reduce kernel
// finishes the split tiles from their partial slots.
hipError_t launch_density(const SweepLaunch &L, const SweepBuffers &B, const PotConst &pc, int precision,
                          hipStream_t s);
hipError_t launch_force(const SweepLaunch &L, const SweepBuffers &B, const StepArgs &a, const PotConst &pc,
                        int precision, hipStream_t s);
// Reduce kernels finish every tile with at least min_split partial slots
// (2 after an all-pairs sweep, 1 after a cell-list sweep).
hipError_t launch_density_reduce(const ITile *tiles, int ntiles, int tile, const SweepBuffers &B,
                                 const PotConst &pc, int min_split, hipStream_t s);
hipError_t launch_force_reduce(const ITile *tiles, int ntiles, int tile, const SweepBuffers &B, const StepArgs &a,
                               const PotConst &pc, int min_split, hipStream_t s);
// Symmetric (each unordered pair once) all-pairs sweeps.  Tiles are 64
// atoms; IPT consecutive tiles of a cluster form a group held by one
// wavefront.  An item is a group against the later tiles [b0, b1) (global
// tile indices), or the group's own pairs when b0 == b1.
struct SymItem {
    int32_t c, g, t0, ng, b0, b1, slot, pad;  // g: group index within the cluster; t0: its first tile
};
// A 64-atom tile: its j-side partials sit at jbase + g for the nj groups
// before it; its i-side partials are items [item0, item0 + nitems) at lane
// block p of each item.
struct SymTile {
    int32_t c, i0, ni, jbase, nj, item0, nitems, p;
};
struct SymLaunch {
    const SymItem *items;
    const int32_t *order;
    const SymTile *tiles;
    int nitems, ntiles, ipt;
    double *ipart;  // nitems x 4 x 64*IPT
    double *jpart;  // sum(nj) x 3 x 64
};
// stage 0: the sweep (partials); stage 1: reduce + tile finish (density:
// rho, P, embedding sums; force: F, kick, pair-energy and v^2 sums).  FP64
// or mixed; (n, m) = (9, 6) and no cutoff only.
hipError_t launch_sym_density(const SymLaunch &L, const SweepBuffers &B, const PotConst &pc, int precision,
                              int stage, hipStream_t s);
hipError_t launch_sym_force(const SymLaunch &L, const SweepBuffers &B, const StepArgs &a, const PotConst &pc,
                            int precision, int stage, hipStream_t s);

// Row sweeps for small clusters: one workgroup of 64 * waves threads per
// tile of at most 64 atoms against every partner of the tile's cluster;
// each sweep finishes its tiles in the same launch (no partial slots).
struct RowLaunch {
    const ITile *tiles;
    const int32_t *order;  // launch order of the tiles
    const ClusterDesc *cd;
    int ntiles;
    int waves;             // 4, 8 or 16; tiles hold at most 8 * waves atoms
    int nmax;              // atoms of the largest cluster (LDS staging when <= kRowStageMax)
    // single cluster with equal runs: tile b = atoms [off + b ni, min(off + n,
    // off + (b+1) ni)) of cluster 0, computed without reading the tables
    int uni_off, uni_n, uni_ni;  // uni_ni = 0: use the tables
};
constexpr int kRowStageMax = 4096;  // clusters up to this size are staged in LDS (128 KiB)
// Drift folded into the row density sweep of staged clusters (a single
// cluster or a batch): every workgroup drifts its whole cluster while staging
// it (r + dt (lambda v + h F)); mode 2 first finishes the previous step's
// thermostat factor from the cluster's v^2 tile sums (the finalize's order,
// so the same bits) and the cluster's first tile stores it in st[c].lambda
// for the force sweep, whose epilogue (fused) applies lambda and the first
// half-kick and stores the positions.  Clusters in a Langevin bath have
// their drifted (r, v) stored by the previous force epilogue (or by
// launch_bath_prep before the run's first step) and are only staged.
struct RowDrift {
    int mode;   // 0: positions as they are; 1: drift with st[c].lambda; 2: new lambda, then drift
    int local;  // steps completed in this run before this one (ramp index st[c].step + local)
    int bath;   // clusters in a Langevin bath: 0 none, 1 all, 2 some (the kernel reads each one's kind)
};
// The drifted position is evaluated as p + (dt lambda) v with p = r + (dt h) F:
// mode 1 forms p from r and F, mode 2 reads p and v as stored by the previous
// fused force epilogue (48 bytes per atom), with the same rounding.
hipError_t launch_row_density(const RowLaunch &L, const SweepBuffers &B, const StepArgs &a, const RowDrift &dr,
                              const PotConst &pc, int precision, hipStream_t s);
// fused: per cluster, the Berendsen/NVE epilogue (lambda, both half-kicks,
// next drift inputs) or the Langevin one (second half-kick of the stored
// post-bath velocity, then the first half-kick and the A, O, A of the next
// step, whose drifted (r, v) are stored).  local = steps of this run
// completed before this one (the step is st[c].step + local + 1).
hipError_t launch_row_force(const RowLaunch &L, const SweepBuffers &B, const StepArgs &a, int fused, int local,
                            int bath, const PotConst &pc, int precision, hipStream_t s);
// Clusters in a Langevin bath, first step of a run on the fused row path:
// the first half-kick (after the pending thermostat factor) and the A, O, A
// of step st[c].step + 1, stored as the drifted (r, v) pairs.
hipError_t launch_bath_prep(const StepArgs &a, const int32_t *atom_cluster, const double4 *rp, const double4 *v,
                            const double4 *f, double2 *dpv, int natoms, hipStream_t s);

// Per-cluster energies, temperature and thermostat factor from the tile sums;
// step_add = steps completed since the cluster step counter was last stored
// (1 after every step; 0 for an evaluation without motion).
hipError_t launch_finalize(const StepArgs &a, const double *tile_sums, int nclusters, int step_add, hipStream_t s);
// Single cluster: the finish of the run's step `local` (>= 1, counted from the
// start of the run, counter not stored) fused with the drift of step local+1.
// cc (nullptr: none): the cell list's check on the drifted positions of the
// single cluster.
hipError_t launch_drift_fin(const StepArgs &a, const double *tile_sums, int local, double4 *rp, double4 *v,
                            const double4 *f, int natoms, const CellCheck *cc, hipStream_t s);


// Drift of every atom: v <- lambda v + (dt/2m) F, then r <- r + dt v, or
// for a cluster in a Langevin bath the A, O, A of its step st.step + local + 1.
hipError_t launch_drift(const int32_t *atom_cluster, const ClusterDesc *cd, const ClusterState *st, double4 *rp,
                        double4 *v, const double4 *f, int natoms, double mass_u, double dt, double h, int local,
                        hipStream_t s);
hipError_t launch_aos_from4(const double4 *src, double *dst, int natoms, hipStream_t s);
// Append the state of every cluster to ring slot `slot` (5 doubles per
// cluster: step, E_pot, E_kin, T, T_target).
hipError_t launch_sample(const ClusterState *st, int nclusters, double *ring, int slot, int64_t step, hipStream_t s);

// Pair-distance histogram of the atoms [off, off + n) (analysis.hip): refs
// (n entries) and nref receive the reference atoms; counts (nbins) is
// cleared first when `clear`, then the pairs are added to it; nref_total,
// when not null, has the number of reference atoms added to it.
hipError_t launch_rdf(const double4 *rp, int off, int n, double r_select, double dr, int nbins, int32_t *refs,
                      int *nref, unsigned long long *counts, bool clear, long long *nref_total, hipStream_t s);

// Frame store of the diffusion coefficient (analysis.hip): copy the atoms
// [off, off + n) of rp to dst (n entries).
hipError_t launch_store_frame(const double4 *rp, int off, int n, double4 *dst, hipStream_t s);
// Diffusion coefficient from the window of frames [first, first + segments *
// seg) of a ring of `cap` frames of n atoms: seg_d (segments entries) receives
// each segment's coefficient, *ncentral the central atoms, *d_out the mean
// (A^2/ps).
hipError_t launch_diffusion(const double4 *frames, int n, int cap, int64_t first, int seg, int segments,
                            double radius, double dt_ps, double *seg_d, int *ncentral, double *d_out,
                            hipStream_t s);

// Number of doubles per tile in tile_sums: [0] sum e_emb, [1] sum e_pair,
// [2] sum v^2.
constexpr int kTileSums = 4;

}  // namespace scmd
