// Cell-list sweeps: placeholder until the cutoff variant lands.
#include "cell_list.h"

namespace scmd {

struct CellList {
    int dummy;
};

bool cell_list_available() { return false; }
CellList *cell_list_create() { return nullptr; }
void cell_list_destroy(CellList *) {}
hipError_t cell_list_plan(CellList *, int, const int64_t *, double, const ITile *, int, int) {
    return hipErrorNotSupported;
}
hipError_t cell_list_build(CellList *, const double4 *, hipStream_t) { return hipErrorNotSupported; }
hipError_t cell_list_density(CellList *, const double4 *, double *, const PotConst &, int, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t cell_list_force(CellList *, const double4 *, double *, const PotConst &, int, hipStream_t) {
    return hipErrorNotSupported;
}
bool cell_list_overflowed(CellList *) { return false; }

}  // namespace scmd
