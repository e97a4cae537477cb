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
// (host) with cutoff rc, from the current positions rp (device).  tiles
// (host)/ntiles/tile: the atom tiles whose partial slots the sweeps write
// (one slot per tile); tile must be a power of two.
// skin >= 0: cells and per-atom lists cover rc + skin and are rebuilt only
// once an atom has moved more than skin / 2 since the last build (skin = 0:
// every step).
hipError_t cell_list_plan(CellList *cl, int nclusters, const int64_t *offsets, double rc, double skin,
                          const double4 *rp, const ITile *tiles_host, int ntiles, int tile);
// Displacement check, then the rebuild of the cells when it is due (the
// density sweep of the same evaluation rebuilds the lists).
hipError_t cell_list_build(CellList *cl, const double4 *rp, hipStream_t s);
// Rebuilds of the cells and lists since the plan (synchronous read).
hipError_t cell_list_rebuilds(CellList *cl, int64_t *out);
// Make the next evaluation rebuild (positions replaced from outside).
hipError_t cell_list_invalidate(CellList *cl, hipStream_t s);
// Positions of the last build (natoms, atom order) for checkpoints, and the
// restore of cells and lists from such positions (ref_host, copied through
// the natoms-entry device buffer scratch_dev) exactly as that build made
// them, so that a resumed run continues bit for bit.
hipError_t cell_list_get_ref(CellList *cl, double4 *host_out);
hipError_t cell_list_restore(CellList *cl, const double4 *ref_host, double4 *scratch_dev, const SweepBuffers &B,
                             const PotConst &pc, int precision, hipStream_t s);
// Density and force sweeps over the cell list, finished per atom tile with
// the same epilogues as the all-pairs sweeps (tiles/ntiles/tile: the atom
// tiles of the plan, one partial slot per tile).
hipError_t cell_list_density(CellList *cl, const SweepBuffers &B, const ITile *tiles, int ntiles, int tile,
                             const PotConst &pc, int precision, hipStream_t s);
hipError_t cell_list_force(CellList *cl, const SweepBuffers &B, const StepArgs &a, const ITile *tiles, int ntiles,
                           int tile, const PotConst &pc, int precision, hipStream_t s);
}  // namespace scmd
