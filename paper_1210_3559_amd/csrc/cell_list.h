// Cell-list variant of the pair sweeps (truncated, shifted potential).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scmd_internal.h"

namespace scmd {

struct CellList;

bool cell_list_available();
CellList *cell_list_create();
void cell_list_destroy(CellList *cl);
// Plan cell capacities and buffers for the clusters described by offsets
// (host) with cutoff rc, from the current positions rp (device).
// skin >= 0: cells and per-atom lists cover rc + skin and are rebuilt only
// once an atom has moved more than skin / 2 since the last build (skin = 0:
// every step).
hipError_t cell_list_plan(CellList *cl, int nclusters, const int64_t *offsets, double rc, double skin,
                          const double4 *rp);
// The force sweep stores each cell's energy and v^2 sums (kTileSums doubles)
// at the cell's index: cluster c owns slots [first, first + count) of
// total_slots, and the per-cluster finish adds those.
void cell_list_sum_slots(const CellList *cl, int cluster, int *first, int *count);
int cell_list_total_slots(const CellList *cl);
// Displacement check, then the rebuild of the cells when it is due (the
// density sweep of the same evaluation rebuilds the lists).  checked: the
// kernel that drifted the atoms already ran the check (cell_list_check) on
// these positions.
hipError_t cell_list_build(CellList *cl, const double4 *rp, bool checked, hipStream_t s);
// The check's arguments, for the drift kernel of a single cluster to run it.
CellCheck cell_list_check(CellList *cl);
// Rebuilds of the cells and lists since the plan (synchronous read).
hipError_t cell_list_rebuilds(CellList *cl, int64_t *out);
// Make the next evaluation rebuild (positions replaced from outside).
hipError_t cell_list_invalidate(CellList *cl, hipStream_t s);
// Positions of the last build (natoms, atom order) for checkpoints, and the
// restore of cells and lists from such positions (ref_host, copied through
// the natoms-entry device buffer scratch_dev) exactly as that build made
// them, so that a resumed run continues bit for bit.
hipError_t cell_list_get_ref(CellList *cl, double4 *host_out);
hipError_t cell_list_restore(CellList *cl, const double4 *ref_host, double4 *scratch_dev, const PotConst &pc,
                             int precision, hipStream_t s);
// Density and force sweeps over the cell list; each finishes its atoms with
// the same per-atom epilogues as the all-pairs reduce kernels (density: rho,
// P into xp; force: F, the kick when a.advance), and the force sweep stores
// every cell's sums in B.tile_sums (see cell_list_sum_slots).
hipError_t cell_list_density(CellList *cl, const SweepBuffers &B, const PotConst &pc, int precision,
                             hipStream_t s);
hipError_t cell_list_force(CellList *cl, const SweepBuffers &B, const StepArgs &a, const PotConst &pc,
                           int precision, hipStream_t s);
}  // namespace scmd
