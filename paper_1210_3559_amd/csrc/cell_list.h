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
hipError_t cell_list_plan(CellList *cl, int nclusters, const int64_t *offsets, double rc, const double4 *rp,
                          const ITile *tiles_host, int ntiles, int tile);
hipError_t cell_list_build(CellList *cl, const double4 *rp, hipStream_t s);
// Density and force sweeps over the cell list, finished per atom tile with
// the same epilogues as the all-pairs sweeps (tiles/ntiles/tile: the atom
// tiles of the plan, one partial slot per tile).
hipError_t cell_list_density(CellList *cl, const SweepBuffers &B, const ITile *tiles, int ntiles, int tile,
                             const PotConst &pc, int precision, hipStream_t s);
hipError_t cell_list_force(CellList *cl, const SweepBuffers &B, const StepArgs &a, const ITile *tiles, int ntiles,
                           int tile, const PotConst &pc, int precision, hipStream_t s);
}  // namespace scmd
