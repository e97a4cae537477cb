// All-pairs Sutton-Chen sweeps for gfx950 (one-sided: every atom owns its sums).
//
// The paper reduces the many-body force to two successive two-body sweeps:
// first every density rho_i (Sec. 2.1 Eq. (rho)), then the forces, which need
// psi_j = rho_j^(-1/2) of every partner (Sec. 2 "Computational approach").
//
// Work decomposition.  An atom tile holds 64*IPT*WI atoms: WI wavefronts
// along i, each lane owning IPT atoms.  A work item is one tile against a
// contiguous j chunk of the same cluster; inside the workgroup the chunk is
// split again over WJ wavefronts, whose sums are combined in LDS in a fixed
// order.  The j index is uniform across a wavefront, so partner data
// (x, y, z[, P_j] packed in a 32-byte double4) comes through scalar loads into
// SGPRs and is read directly as a VALU operand: no LDS traffic and no barrier
// in the inner loop, and each partner fetched once per wave serves 64*IPT
// pairs from registers.
//
// A tile whose partner range is covered by one item is finished inside the
// sweep: the density sweep turns sums into rho, psi and the embedding energy,
// the force sweep stores F and applies the second half-kick, and both write
// per-tile energy sums.  When a tile's range is split over several items
// (small clusters, where more parallelism than tiles is needed), each item
// writes a partial sum to its own slot and a reduce kernel finishes the tile
// from the slots in slot order.  Kernel boundaries are the only global
// synchronisation: on gfx950 an agent-scope fence writes back and invalidates
// the XCD's L2, which costs far more than a launch.  Every reduction has a
// fixed order, so results are deterministic.
//
// Self pairs: the j range of a wavefront is split into the part that
// overlaps the tile's own atoms (where j == i is voided by pushing r^2 to a
// huge value, which makes every power term exactly zero) and the parts that
// do not (no mask at all).
#include "sweep_common.h"

namespace scmd {
namespace {

using namespace dev;

template <int IPT, int PREC, bool GEN, bool MASK>
__device__ __forceinline__ void density_range(const double4 *__restrict__ rp, int ja, int jb, const double *xi,
                                              const double *yi, const double *zi, const int *gi, double *acc,
                                              const PotConst &pc) {
#pragma unroll 4
    for (int j = ja; j < jb; ++j) {
        const double4 q = rp[j];
#pragma unroll
        for (int p = 0; p < IPT; ++p) {
            density_pair<PREC, GEN, MASK, false>(xi[p] - q.x, yi[p] - q.y, zi[p] - q.z, MASK && gi[p] == j, acc[p],
                                                 pc);
        }
    }
}

template <int IPT, int PREC, bool GEN, bool MASK>
__device__ __forceinline__ void force_range(const double4 *__restrict__ xp, int ja, int jb, const double *xi,
                                            const double *yi, const double *zi, const double *ci, const float *cif,
                                            const int *gi, double *fx, double *fy, double *fz, double *eu,
                                            const PotConst &pc, float Af) {
#pragma unroll 2
    for (int j = ja; j < jb; ++j) {
        const double4 q = xp[j];
        const float pjf = PREC == SCMD_FP64 ? 0.0f : (float)q.w;
#pragma unroll
        for (int p = 0; p < IPT; ++p) {
            force_pair<PREC, GEN, MASK, false>(xi[p] - q.x, yi[p] - q.y, zi[p] - q.z, MASK && gi[p] == j, ci[p], q.w,
                                               cif[p], pjf, fx[p], fy[p], fz[p], eu[p], pc, Af);
        }
    }
}

// j sub-range of wavefront wj within [j0, j1), split into unmasked / masked /
// unmasked segments around the tile's own atoms [t0, t1).
struct Segs {
    int a, b, c, d;  // [a,b) plain, [b,c) masked, [c,d) plain
};
__device__ __forceinline__ Segs segments(int j0, int j1, int wj, int WJ, int t0, int t1) {
    const int len = j1 - j0;
    const int ja = j0 + (int)(((int64_t)len * wj) / WJ);
    const int jb = j0 + (int)(((int64_t)len * (wj + 1)) / WJ);
    int lo = max(ja, t0), hi = min(jb, t1);
    if (lo >= hi) lo = hi = jb;
    return Segs{ja, lo, hi, jb};
}

template <int IPT, int WI, int WJ, int PREC, bool GEN>
__global__ __launch_bounds__(64 * WI * WJ) void k_density(const SweepItem *__restrict__ items,
                                                          const int32_t *__restrict__ order,
                                                          const ITile *__restrict__ tiles,
                                                          const double4 *__restrict__ rp, double4 *__restrict__ xp,
                                                          double *__restrict__ part, double *__restrict__ rho,
                                                          double *__restrict__ tile_sums, PotConst pc) {
    constexpr int TILE = 64 * IPT * WI;
    constexpr int BLOCK = 64 * WI * WJ;
    __shared__ double sh_x[WJ * TILE];
    __shared__ double sh_red[BLOCK];
    const SweepItem it = items[order[blockIdx.x]];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wi = wave % WI;
    const int wj = wave / WI;

    double xi[IPT], yi[IPT], zi[IPT], acc[IPT];
    int gi[IPT];
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        const int li = wi * 64 * IPT + p * 64 + lane;
        acc[p] = 0.0;
        if (li < it.ni) {
            gi[p] = it.i0 + li;
            const double4 q = rp[gi[p]];
            xi[p] = q.x;
            yi[p] = q.y;
            zi[p] = q.z;
        } else {
            gi[p] = -1;
            xi[p] = yi[p] = zi[p] = -kFar;
        }
    }
    const Segs sg = segments(it.j0, it.j1, wj, WJ, it.i0, it.i0 + it.ni);
    density_range<IPT, PREC, GEN, false>(rp, sg.a, sg.b, xi, yi, zi, gi, acc, pc);
    density_range<IPT, PREC, GEN, true>(rp, sg.b, sg.c, xi, yi, zi, gi, acc, pc);
    density_range<IPT, PREC, GEN, false>(rp, sg.c, sg.d, xi, yi, zi, gi, acc, pc);

    // combine the WJ wavefronts (fixed order) into sh_x[0 .. TILE)
#pragma unroll
    for (int p = 0; p < IPT; ++p) sh_x[wj * TILE + wi * 64 * IPT + p * 64 + lane] = acc[p];
    __syncthreads();
    if (WJ > 1) {
        for (int li = threadIdx.x; li < TILE; li += BLOCK) {
            double s = sh_x[li];
            for (int w = 1; w < WJ; ++w) s += sh_x[w * TILE + li];
            sh_x[li] = s;
        }
        __syncthreads();
    }

    const ITile T = tiles[it.tile];
    if (T.nsplit > 1) {
        double *out = part + (size_t)it.slot * TILE;
        for (int li = threadIdx.x; li < it.ni; li += BLOCK) out[li] = sh_x[li];
        return;
    }
    const DensityOut o{rp, xp, rho, tile_sums};
    double emb = 0.0;
    for (int li = threadIdx.x; li < T.ni; li += BLOCK) emb += density_atom(T.i0 + li, sh_x[li], o, pc);
    emb = block_sum<BLOCK>(emb, sh_red);
    if (threadIdx.x == 0) tile_sums[(size_t)it.tile * kTileSums + 0] = emb;
}

template <int IPT, int WI, int WJ, int PREC, bool GEN>
__global__ __launch_bounds__(64 * WI * WJ) void k_force(const SweepItem *__restrict__ items,
                                                        const int32_t *__restrict__ order,
                                                        const ITile *__restrict__ tiles,
                                                        const double4 *__restrict__ xp, double *__restrict__ part,
                                                        ForceOut o, PotConst pc) {
    constexpr int TILE = 64 * IPT * WI;
    constexpr int BLOCK = 64 * WI * WJ;
    __shared__ double sh_x[4 * WJ * TILE];
    __shared__ double sh_red[BLOCK];
    const SweepItem it = items[order[blockIdx.x]];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wi = wave % WI;
    const int wj = wave / WI;
    const float Af = (float)pc.A;

    double xi[IPT], yi[IPT], zi[IPT], ci[IPT], fx[IPT], fy[IPT], fz[IPT], eu[IPT];
    float cif[IPT];
    int gi[IPT];
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        const int li = wi * 64 * IPT + p * 64 + lane;
        fx[p] = fy[p] = fz[p] = eu[p] = 0.0;
        if (li < it.ni) {
            gi[p] = it.i0 + li;
            const double4 q = xp[gi[p]];
            xi[p] = q.x;
            yi[p] = q.y;
            zi[p] = q.z;
            ci[p] = -q.w;
        } else {
            gi[p] = -1;
            xi[p] = yi[p] = zi[p] = -kFar;
            ci[p] = 0.0;
        }
        cif[p] = (float)ci[p];
    }
    const Segs sg = segments(it.j0, it.j1, wj, WJ, it.i0, it.i0 + it.ni);
    force_range<IPT, PREC, GEN, false>(xp, sg.a, sg.b, xi, yi, zi, ci, cif, gi, fx, fy, fz, eu, pc, Af);
    force_range<IPT, PREC, GEN, true>(xp, sg.b, sg.c, xi, yi, zi, ci, cif, gi, fx, fy, fz, eu, pc, Af);
    force_range<IPT, PREC, GEN, false>(xp, sg.c, sg.d, xi, yi, zi, ci, cif, gi, fx, fy, fz, eu, pc, Af);
#pragma unroll
    for (int p = 0; p < IPT; ++p) unscale_force<PREC, GEN>(fx[p], fy[p], fz[p], eu[p]);

    // combine the WJ wavefronts: sh_x[(w*4 + q)*TILE + li]
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        const int li = wi * 64 * IPT + p * 64 + lane;
        sh_x[(wj * 4 + 0) * TILE + li] = fx[p];
        sh_x[(wj * 4 + 1) * TILE + li] = fy[p];
        sh_x[(wj * 4 + 2) * TILE + li] = fz[p];
        sh_x[(wj * 4 + 3) * TILE + li] = eu[p];
    }
    __syncthreads();
    if (WJ > 1) {
        for (int e = threadIdx.x; e < 4 * TILE; e += BLOCK) {
            double s = sh_x[e];
            for (int w = 1; w < WJ; ++w) s += sh_x[w * 4 * TILE + e];
            sh_x[e] = s;
        }
        __syncthreads();
    }

    const ITile T = tiles[it.tile];
    if (T.nsplit > 1) {
        double *out = part + (size_t)it.slot * 4 * TILE;
        for (int e = threadIdx.x; e < 4 * TILE; e += BLOCK)
            if ((e % TILE) < it.ni) out[e] = sh_x[e];
        return;
    }
    double epair = 0.0, v2 = 0.0;
    for (int li = threadIdx.x; li < T.ni; li += BLOCK)
        force_atom(T.i0 + li, sh_x[li], sh_x[TILE + li], sh_x[2 * TILE + li], sh_x[3 * TILE + li], o, pc, epair,
                   v2);
    epair = block_sum<BLOCK>(epair, sh_red);
    v2 = block_sum<BLOCK>(v2, sh_red);
    if (threadIdx.x == 0) {
        o.tile_sums[(size_t)it.tile * kTileSums + 1] = epair;
        o.tile_sums[(size_t)it.tile * kTileSums + 2] = v2;
    }
}

// ---------------------------------------------------------------------------
// Reduce kernels for split tiles: one workgroup of 256 threads per tile; G =
// 256 / TILE thread groups each sum every G-th slot (in order), then the
// group sums are added in group order.
// ---------------------------------------------------------------------------
constexpr int kRedBlock = 256;

template <int TILE, int Q>
__device__ __forceinline__ void reduce_slots(const ITile &T, const double *__restrict__ part, double *sh) {
    constexpr int G = TILE < kRedBlock ? kRedBlock / TILE : 1;
    const int t = threadIdx.x;
    if (G > 1) {
        const int li = t % TILE, g = t / TILE;
        if (li < T.ni) {
            double s[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) s[q] = 0.0;
            for (int k = g; k < T.nsplit; k += G) {
                const double *p = part + ((size_t)(T.first + k) * Q) * TILE + li;
#pragma unroll
                for (int q = 0; q < Q; ++q) s[q] += p[(size_t)q * TILE];
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) sh[(g * Q + q) * TILE + li] = s[q];
        }
        __syncthreads();
        if (t < TILE && t < T.ni) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double s = sh[q * TILE + t];
                for (int gg = 1; gg < G; ++gg) s += sh[(gg * Q + q) * TILE + t];
                sh[q * TILE + t] = s;
            }
        }
        __syncthreads();
    } else {
        for (int li = t; li < T.ni; li += kRedBlock) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                sh[q * TILE + li] = sum_slots(part + ((size_t)T.first * Q + q) * TILE + li, T.nsplit, (size_t)Q * TILE);
        }
        __syncthreads();
    }
}

template <int TILE>
__global__ __launch_bounds__(kRedBlock) void k_density_reduce(const ITile *__restrict__ tiles,
                                                              const double *__restrict__ part, DensityOut o,
                                                              PotConst pc, int min_split) {
    constexpr int G = TILE < kRedBlock ? kRedBlock / TILE : 1;
    __shared__ double sh[G * TILE];
    __shared__ double sh_red[kRedBlock];
    const ITile T = tiles[blockIdx.x];
    if (T.nsplit < min_split) return;
    reduce_slots<TILE, 1>(T, part, sh);
    double emb = 0.0;
    for (int li = threadIdx.x; li < T.ni; li += kRedBlock) emb += density_atom(T.i0 + li, sh[li], o, pc);
    emb = block_sum<kRedBlock>(emb, sh_red);
    if (threadIdx.x == 0) o.tile_sums[(size_t)blockIdx.x * kTileSums + 0] = emb;
}

template <int TILE>
__global__ __launch_bounds__(kRedBlock) void k_force_reduce(const ITile *__restrict__ tiles,
                                                            const double *__restrict__ part, ForceOut o,
                                                            PotConst pc, int min_split) {
    constexpr int G = TILE < kRedBlock ? kRedBlock / TILE : 1;
    __shared__ double sh[4 * G * TILE];
    __shared__ double sh_red[kRedBlock];
    const ITile T = tiles[blockIdx.x];
    if (T.nsplit < min_split) return;
    reduce_slots<TILE, 4>(T, part, sh);
    double epair = 0.0, v2 = 0.0;
    for (int li = threadIdx.x; li < T.ni; li += kRedBlock)
        force_atom(T.i0 + li, sh[li], sh[TILE + li], sh[2 * TILE + li], sh[3 * TILE + li], o, pc, epair, v2);
    epair = block_sum<kRedBlock>(epair, sh_red);
    v2 = block_sum<kRedBlock>(v2, sh_red);
    if (threadIdx.x == 0) {
        o.tile_sums[(size_t)blockIdx.x * kTileSums + 1] = epair;
        o.tile_sums[(size_t)blockIdx.x * kTileSums + 2] = v2;
    }
}

constexpr int kFinBlock = 256;

__global__ __launch_bounds__(kFinBlock) void k_finalize(FinalizeArgs a) {
    __shared__ double sh[12];
    cluster_finalize(blockIdx.x, a, sh, true);
}

template <int IPT, int WI, int WJ, int PREC, bool GEN>
hipError_t launch_shape(bool force, const SweepLaunch &L, const SweepBuffers &B, const ForceOut &o,
                        const PotConst &pc, hipStream_t s) {
    constexpr int BLOCK = 64 * WI * WJ;
    if (L.nitems <= 0) return hipSuccess;
    (void)hipGetLastError();
    if (force) {
        hipLaunchKernelGGL((k_force<IPT, WI, WJ, PREC, GEN>), dim3(L.nitems), dim3(BLOCK), 0, s, L.items, L.order,
                           L.tiles, B.xp, B.part, o, pc);
    } else {
        hipLaunchKernelGGL((k_density<IPT, WI, WJ, PREC, GEN>), dim3(L.nitems), dim3(BLOCK), 0, s, L.items, L.order,
                           L.tiles, B.rp, B.xp, B.part, B.rho, B.tile_sums, pc);
    }
    return hipGetLastError();
}

template <int PREC, bool GEN>
hipError_t dispatch_shape(bool force, const SweepLaunch &L, const SweepBuffers &B, const ForceOut &o,
                          const PotConst &pc, hipStream_t s) {
#define SCMD_SHAPE(I, WI_, WJ_)                                 \
    if (L.ipt == I && L.wi == WI_ && L.wj == WJ_)               \
        return launch_shape<I, WI_, WJ_, PREC, GEN>(force, L, B, o, pc, s);
    if constexpr (GEN) {
        // the generic-exponent path exists in one launch shape only
        SCMD_SHAPE(1, 4, 1)
    } else {
        SCMD_SWEEP_SHAPES(SCMD_SHAPE)
    }
#undef SCMD_SHAPE
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_density(const SweepLaunch &L, const SweepBuffers &B, const PotConst &pc, int precision,
                          hipStream_t s) {
    ForceOut o{};
    if (precision == SCMD_FP64)
        return pc.generic ? dispatch_shape<SCMD_FP64, true>(false, L, B, o, pc, s)
                          : dispatch_shape<SCMD_FP64, false>(false, L, B, o, pc, s);
    return pc.generic ? dispatch_shape<SCMD_MIXED, true>(false, L, B, o, pc, s)
                      : dispatch_shape<SCMD_MIXED, false>(false, L, B, o, pc, s);
}

hipError_t launch_force(const SweepLaunch &L, const SweepBuffers &B, const StepArgs &a, const PotConst &pc,
                        int precision, hipStream_t s) {
    ForceOut o{B.f, B.v, B.tile_sums, a.h, a.advance};
    if (precision == SCMD_FP64)
        return pc.generic ? dispatch_shape<SCMD_FP64, true>(true, L, B, o, pc, s)
                          : dispatch_shape<SCMD_FP64, false>(true, L, B, o, pc, s);
    return pc.generic ? dispatch_shape<SCMD_MIXED, true>(true, L, B, o, pc, s)
                      : dispatch_shape<SCMD_MIXED, false>(true, L, B, o, pc, s);
}

template <int TILE>
static hipError_t reduce_tile(bool force, const ITile *tiles, int ntiles, const SweepBuffers &B, const ForceOut &fo,
                              const PotConst &pc, int min_split, hipStream_t s) {
    (void)hipGetLastError();
    if (force) {
        hipLaunchKernelGGL((k_force_reduce<TILE>), dim3(ntiles), dim3(kRedBlock), 0, s, tiles, B.part, fo, pc,
                           min_split);
    } else {
        const DensityOut o{B.rp, B.xp, B.rho, B.tile_sums};
        hipLaunchKernelGGL((k_density_reduce<TILE>), dim3(ntiles), dim3(kRedBlock), 0, s, tiles, B.part, o, pc,
                           min_split);
    }
    return hipGetLastError();
}

static hipError_t reduce_dispatch(bool force, const ITile *tiles, int ntiles, int tile, const SweepBuffers &B,
                                  const ForceOut &fo, const PotConst &pc, int min_split, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    switch (tile) {
        case 64: return reduce_tile<64>(force, tiles, ntiles, B, fo, pc, min_split, s);
        case 128: return reduce_tile<128>(force, tiles, ntiles, B, fo, pc, min_split, s);
        case 256: return reduce_tile<256>(force, tiles, ntiles, B, fo, pc, min_split, s);
        case 512: return reduce_tile<512>(force, tiles, ntiles, B, fo, pc, min_split, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_density_reduce(const ITile *tiles, int ntiles, int tile, const SweepBuffers &B,
                                 const PotConst &pc, int min_split, hipStream_t s) {
    return reduce_dispatch(false, tiles, ntiles, tile, B, ForceOut{}, pc, min_split, s);
}

hipError_t launch_force_reduce(const ITile *tiles, int ntiles, int tile, const SweepBuffers &B, const StepArgs &a,
                               const PotConst &pc, int min_split, hipStream_t s) {
    const ForceOut fo{B.f, B.v, B.tile_sums, a.h, a.advance};
    return reduce_dispatch(true, tiles, ntiles, tile, B, fo, pc, min_split, s);
}

hipError_t launch_finalize(const StepArgs &a, const double *tile_sums, int nclusters, int step_add, hipStream_t s) {
    if (nclusters <= 0) return hipSuccess;
    const FinalizeArgs fa{a.cd, a.st, tile_sums, a.flag, a.mass_u, a.dt, a.advance, step_add, 1};
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_finalize, dim3(nclusters), dim3(kFinBlock), 0, s, fa);
    return hipGetLastError();
}

}  // namespace scmd
