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
// Plan grids and buffers for the clusters described by offsets (host) with
// cutoff rc.  tiles/ntiles/tile: the atom tiles whose partial slots the
// sweeps write (one slot per tile).
hipError_t cell_list_plan(CellList *cl, int nclusters, const int64_t *offsets, double rc, const ITile *tiles_host,
                          int ntiles, int tile);
hipError_t cell_list_build(CellList *cl, const double4 *rp, hipStream_t s);
hipError_t cell_list_density(CellList *cl, const double4 *rp, double *part, const PotConst &pc, int precision,
                             hipStream_t s);
hipError_t cell_list_force(CellList *cl, const double4 *rp, double *part, const PotConst &pc, int precision,
                           hipStream_t s);
// True when a build found a cluster whose grid exceeded its cell cap (reads a
// flag from the device; synchronises with the stream of the last build).
bool cell_list_overflowed(CellList *cl);

}  // namespace scmd
