// Symmetric (Newton's third law) all-pairs sweeps for large clusters.
//
// Both sweeps of the paper's scheme (Sec. 2.1 Eqs. (SC), (rho); Sec. 2
// "Computational approach") are symmetric in i and j: (a/r_ij)^m enters
// rho_i and rho_j alike, and the force term of a pair acts with opposite
// signs on i and j.  Here every unordered pair is evaluated once.
//
// Atoms of a cluster are cut into 64-atom tiles; IPT consecutive tiles form
// a group that sits in one wavefront (lane l owns atom l of each of the
// group's tiles).  A work item is one group against a run of later tiles:
// each j tile is loaded one atom per lane and then rotated through the
// wavefront with DPP wave_ror:1 64 times, so that every lane meets every j
// atom; the j tile carries its own force (or density) accumulators along.
// Pairs inside a group are done by a separate diagonal item, in which the
// group's own tiles rotate past it the same way: a pair of different tiles
// is evaluated once (its j sums return to their home lanes after the 64
// rotations and join the i sums of their tile), a pair inside one tile
// one-sidedly from both ends.
//
// Outputs are partial sums: the i side per item, the j side per (group,
// tile).  The reduce kernels add, for every atom, its group's i-side items in
// item order and then the j-side partials of every earlier group in group
// order: the result is deterministic.  Pair energy: each unordered pair adds
// 2 u^n to the i side (pairs inside a tile add u^n per ordered pair), so
// E_pair = (eps/2) a^n sum over all atoms, as in the one-sided sweeps.
#include "sweep_common.h"

namespace scmd {
namespace {

using namespace dev;

// Lane l receives the value of lane l-1 (mod 64): DPP wave_ror:1.  Every
// source lane is valid, so no "old" value is needed (bound_ctrl set).
__device__ __forceinline__ double ror1(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x13C, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x13C, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// i atoms of the group held by this lane.
template <int IPT>
struct IGroup {
    double x[IPT], y[IPT], z[IPT], c[IPT];  // c = -P_i
    int gi[IPT];
};

template <int IPT>
__device__ __forceinline__ void load_group(const SymItem &it, const SymTile *__restrict__ tiles,
                                           const double4 *__restrict__ src, IGroup<IPT> &G) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        G.gi[p] = -1;
        G.x[p] = G.y[p] = G.z[p] = -kFar;
        G.c[p] = 0.0;
        if (p < it.ng) {
            const SymTile t = tiles[it.t0 + p];
            if (lane < t.ni) {
                G.gi[p] = t.i0 + lane;
                const double4 q = src[G.gi[p]];
                G.x[p] = q.x;
                G.y[p] = q.y;
                G.z[p] = q.z;
                G.c[p] = -q.w;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Force sweep
// ---------------------------------------------------------------------------
template <int PREC, bool EN>
__device__ __forceinline__ void sym_force_pair(double dx, double dy, double dz, double ci, double pj, float cif,
                                               float pjf, double &fx, double &fy, double &fz, double &eu,
                                               double &gx, double &gy, double &gz, const PotConst &pc, float Af) {
    double f, un;
    if constexpr (PREC == SCMD_FP64) {
        // w = 2u; sums scaled by 2^8 (force) and 2^9 (u^n), see force_pair
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        const double w = rsq2_nr(r2);
        const double w2 = w * w;
        const double w3 = w2 * w;
        const double w4 = w2 * w2;
        const double w8 = w4 * w4;
        const double q = __builtin_fma(pc.A8, w3, ci) - pj;
        f = w8 * q;
        if constexpr (EN) un = w8 * w;
    } else {
        const double r2d = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        const float u = __builtin_amdgcn_rsqf((float)r2d);
        const float u2 = u * u;
        const float u3 = u2 * u;
        const float u4 = u2 * u2;
        const float u8 = u4 * u4;
        const float q = __builtin_fmaf(Af, u3, cif) - pjf;
        f = (double)(u8 * q);
        if constexpr (EN) un = (double)(u8 * u);
    }
    fx = __builtin_fma(f, dx, fx);
    fy = __builtin_fma(f, dy, fy);
    fz = __builtin_fma(f, dz, fz);
    gx = __builtin_fma(-f, dx, gx);
    gy = __builtin_fma(-f, dy, gy);
    gz = __builtin_fma(-f, dz, gz);
    if constexpr (EN) eu += un;
}

// EN: accumulate and store the pair energy (u^n); without it (steps whose
// energies nobody reads) the energy partials are neither summed nor stored.
template <int IPT, int PREC, bool EN>
__global__ __launch_bounds__(64) void k_sym_force(const SymItem *__restrict__ items, const int32_t *__restrict__ order,
                                                  const SymTile *__restrict__ tiles, const double4 *__restrict__ xp,
                                                  double *__restrict__ ipart, double *__restrict__ jpart,
                                                  PotConst pc) {
    const SymItem it = items[order[blockIdx.x]];
    const int lane = threadIdx.x & 63;
    const float Af = (float)pc.A;
    IGroup<IPT> G;
    load_group<IPT>(it, tiles, xp, G);
    float cif[IPT];
    double fx[IPT], fy[IPT], fz[IPT], eu[IPT];
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        fx[p] = fy[p] = fz[p] = eu[p] = 0.0;
        cif[p] = (float)G.c[p];
    }
    if (it.b0 == it.b1) {
        // diagonal item: the group's own tile b rotates past tiles p <= b
        double eus[IPT];  // energy of the pairs of different tiles (counted twice below)
#pragma unroll
        for (int p = 0; p < IPT; ++p) eus[p] = 0.0;
#pragma unroll
        for (int b = 0; b < IPT; ++b) {
            if (b < it.ng) {
                const bool own = G.gi[b] >= 0;  // past the tile's atoms: the j sentinel
                double xj = own ? G.x[b] : kFar, yj = own ? G.y[b] : kFar, zj = own ? G.z[b] : kFar;
                double pj = own ? -G.c[b] : 0.0;
                double gx = 0.0, gy = 0.0, gz = 0.0;
                // rotation k: lane l meets atom l - k of tile b; k = 0 is the
                // self pair inside tile b
                auto step = [&](bool with_own_tile) {
                    const float pjf = (float)pj;
#pragma unroll
                    for (int p = 0; p < IPT; ++p) {
                        if (p < b) {
                            sym_force_pair<PREC, EN>(G.x[p] - xj, G.y[p] - yj, G.z[p] - zj, G.c[p], pj, cif[p], pjf,
                                                     fx[p], fy[p], fz[p], eus[p], gx, gy, gz, pc, Af);
                        } else if (p == b && with_own_tile) {
                            double hx = 0.0, hy = 0.0, hz = 0.0;  // one-sided: no j sums
                            sym_force_pair<PREC, EN>(G.x[p] - xj, G.y[p] - yj, G.z[p] - zj, G.c[p], pj, cif[p], pjf,
                                                     fx[p], fy[p], fz[p], eu[p], hx, hy, hz, pc, Af);
                        }
                    }
                    xj = ror1(xj);
                    yj = ror1(yj);
                    zj = ror1(zj);
                    pj = ror1(pj);
                    gx = ror1(gx);
                    gy = ror1(gy);
                    gz = ror1(gz);
                };
                step(false);
#pragma unroll 2
                for (int k = 1; k < 64; ++k) step(true);
                // after 64 rotations the j sums are back in their home lanes
                fx[b] += gx;
                fy[b] += gy;
                fz[b] += gz;
            }
        }
#pragma unroll
        for (int p = 0; p < IPT; ++p) eu[p] += 2.0 * eus[p];
    } else {
        for (int b = it.b0; b < it.b1; ++b) {
            const SymTile t = tiles[b];
            double xj = kFar, yj = kFar, zj = kFar, pj = 0.0;
            if (lane < t.ni) {
                const double4 q = xp[t.i0 + lane];
                xj = q.x;
                yj = q.y;
                zj = q.z;
                pj = q.w;
            }
            double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll 2
            for (int k = 0; k < 64; ++k) {
                const float pjf = (float)pj;
#pragma unroll
                for (int p = 0; p < IPT; ++p) {
                    sym_force_pair<PREC, EN>(G.x[p] - xj, G.y[p] - yj, G.z[p] - zj, G.c[p], pj, cif[p], pjf, fx[p], fy[p],
                                         fz[p], eu[p], gx, gy, gz, pc, Af);
                }
                xj = ror1(xj);
                yj = ror1(yj);
                zj = ror1(zj);
                pj = ror1(pj);
                gx = ror1(gx);
                gy = ror1(gy);
                gz = ror1(gz);
            }
            double ge = 0.0;
            unscale_force<PREC, false>(gx, gy, gz, ge);
            double *out = jpart + ((size_t)(t.jbase + it.g) * 3) * 64 + lane;
            out[0] = gx;
            out[64] = gy;
            out[128] = gz;
        }
#pragma unroll
        for (int p = 0; p < IPT; ++p) eu[p] *= 2.0;  // each unordered pair once
    }
#pragma unroll
    for (int p = 0; p < IPT; ++p) unscale_force<PREC, false>(fx[p], fy[p], fz[p], eu[p]);
    double *out = ipart + (size_t)it.slot * 4 * 64 * IPT;
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        out[(0 * IPT + p) * 64 + lane] = fx[p];
        out[(1 * IPT + p) * 64 + lane] = fy[p];
        out[(2 * IPT + p) * 64 + lane] = fz[p];
        // steps without the pair energy leave its slot unwritten (the reduce
        // of such a step does not read it)
        if constexpr (EN) out[(3 * IPT + p) * 64 + lane] = eu[p];
    }
}

// ---------------------------------------------------------------------------
// Density sweep
// ---------------------------------------------------------------------------
// (a/r)^m / a^m = u^6 of one pair ((n, m) = (9, 6)).
template <int PREC>
__device__ __forceinline__ double sym_density_term(double dx, double dy, double dz) {
    if constexpr (PREC == SCMD_FP64) {
        const double w = rcp_nr(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
        return w * w * w;
    } else {
        const float w = __builtin_amdgcn_rcpf((float)__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
        return (double)(w * w * w);
    }
}

template <int IPT, int PREC>
__global__ __launch_bounds__(64) void k_sym_density(const SymItem *__restrict__ items,
                                                    const int32_t *__restrict__ order,
                                                    const SymTile *__restrict__ tiles, const double4 *__restrict__ rp,
                                                    double *__restrict__ ipart, double *__restrict__ jpart,
                                                    PotConst pc) {
    const SymItem it = items[order[blockIdx.x]];
    const int lane = threadIdx.x & 63;
    IGroup<IPT> G;
    load_group<IPT>(it, tiles, rp, G);
    double acc[IPT];
#pragma unroll
    for (int p = 0; p < IPT; ++p) acc[p] = 0.0;
    if (it.b0 == it.b1) {
        // diagonal item (as in the force sweep): tile b rotates past tiles p <= b
#pragma unroll
        for (int b = 0; b < IPT; ++b) {
            if (b < it.ng) {
                const bool own = G.gi[b] >= 0;
                double xj = own ? G.x[b] : kFar, yj = own ? G.y[b] : kFar, zj = own ? G.z[b] : kFar;
                double rj = 0.0;
                auto step = [&](bool with_own_tile) {
#pragma unroll
                    for (int p = 0; p < IPT; ++p) {
                        if (p < b) {
                            const double t6 = sym_density_term<PREC>(G.x[p] - xj, G.y[p] - yj, G.z[p] - zj);
                            acc[p] += t6;
                            rj += t6;
                        } else if (p == b && with_own_tile) {
                            acc[p] += sym_density_term<PREC>(G.x[p] - xj, G.y[p] - yj, G.z[p] - zj);
                        }
                    }
                    xj = ror1(xj);
                    yj = ror1(yj);
                    zj = ror1(zj);
                    rj = ror1(rj);
                };
                step(false);
#pragma unroll 2
                for (int k = 1; k < 64; ++k) step(true);
                acc[b] += rj;
            }
        }
    } else {
        for (int b = it.b0; b < it.b1; ++b) {
            const SymTile t = tiles[b];
            double xj = kFar, yj = kFar, zj = kFar;
            if (lane < t.ni) {
                const double4 q = rp[t.i0 + lane];
                xj = q.x;
                yj = q.y;
                zj = q.z;
            }
            double rj = 0.0;
#pragma unroll 2
            for (int k = 0; k < 64; ++k) {
#pragma unroll
                for (int p = 0; p < IPT; ++p) {
                    const double t6 = sym_density_term<PREC>(G.x[p] - xj, G.y[p] - yj, G.z[p] - zj);
                    acc[p] += t6;
                    rj += t6;
                }
                xj = ror1(xj);
                yj = ror1(yj);
                zj = ror1(zj);
                rj = ror1(rj);
            }
            jpart[(size_t)(t.jbase + it.g) * 64 + lane] = rj;
        }
    }
    double *out = ipart + (size_t)it.slot * 64 * IPT;
#pragma unroll
    for (int p = 0; p < IPT; ++p) out[p * 64 + lane] = acc[p];
}

// ---------------------------------------------------------------------------
// Reduce + finish: one workgroup of 512 threads per 64-atom tile.  Thread
// (g8, lane), g8 = 0..7, adds the tile's i-side items k and j-side partials
// g with k, g = g8 (mod 8) (items first, each run in increasing order); the
// eight sums are combined in g8 order, so the result is deterministic.
// Q = 1: density; Q = 4: force and pair energy (the energy only when the
// sweep accumulated it, EN; otherwise it is zero and was not stored).
// ---------------------------------------------------------------------------
constexpr int kSymRed = 512;
constexpr int kSymRedGroups = kSymRed / 64;

template <int IPT, int Q, bool EN>
__device__ __forceinline__ void sym_sums(const SymTile &t, const double *__restrict__ ipart,
                                         const double *__restrict__ jpart, double *sh) {
    const int lane = threadIdx.x & 63, g8 = threadIdx.x >> 6;
    constexpr int QI = (Q == 4 && !EN) ? 3 : Q;  // i-side values read
    constexpr int QJ = Q == 4 ? 3 : 1;           // the j side carries no energy
    double s[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] = 0.0;
    if (lane < t.ni) {
        for (int k = g8; k < t.nitems; k += kSymRedGroups) {
            const double *p = ipart + (size_t)(t.item0 + k) * Q * 64 * IPT + t.p * 64 + lane;
#pragma unroll
            for (int q = 0; q < QI; ++q) s[q] += p[(size_t)q * IPT * 64];
        }
        for (int g = g8; g < t.nj; g += kSymRedGroups) {
            const double *p = jpart + ((size_t)(t.jbase + g) * QJ) * 64 + lane;
#pragma unroll
            for (int q = 0; q < QJ; ++q) s[q] += p[q * 64];
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) sh[(g8 * Q + q) * 64 + lane] = s[q];
    __syncthreads();
    if (g8 == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double v = sh[q * 64 + lane];
            for (int gg = 1; gg < kSymRedGroups; ++gg) v += sh[(gg * Q + q) * 64 + lane];
            sh[q * 64 + lane] = v;
        }
    }
    __syncthreads();
}

template <int IPT>
__global__ __launch_bounds__(kSymRed) void k_sym_density_reduce(const SymTile *__restrict__ tiles,
                                                                const double *__restrict__ ipart,
                                                                const double *__restrict__ jpart, DensityOut o,
                                                                PotConst pc) {
    __shared__ double sh[kSymRedGroups * 64];
    __shared__ double sh_red[kSymRed];
    const SymTile t = tiles[blockIdx.x];
    sym_sums<IPT, 1, false>(t, ipart, jpart, sh);
    double emb = 0.0;
    if (threadIdx.x < t.ni) emb = density_atom(t.i0 + threadIdx.x, sh[threadIdx.x], o, pc);
    emb = block_sum<kSymRed>(emb, sh_red);
    if (threadIdx.x == 0) o.tile_sums[(size_t)blockIdx.x * kTileSums + 0] = emb;
}

template <int IPT, bool EN>
__global__ __launch_bounds__(kSymRed) void k_sym_force_reduce(const SymTile *__restrict__ tiles,
                                                              const double *__restrict__ ipart,
                                                              const double *__restrict__ jpart, ForceOut o,
                                                              PotConst pc) {
    __shared__ double sh[kSymRedGroups * 4 * 64];
    __shared__ double sh_red[kSymRed];
    const SymTile t = tiles[blockIdx.x];
    sym_sums<IPT, 4, EN>(t, ipart, jpart, sh);
    double epair = 0.0, v2 = 0.0;
    const int l = threadIdx.x;
    if (l < t.ni) force_atom(t.i0 + l, sh[l], sh[64 + l], sh[128 + l], sh[192 + l], o, pc, epair, v2);
    epair = block_sum<kSymRed>(epair, sh_red);
    v2 = block_sum<kSymRed>(v2, sh_red);
    if (threadIdx.x == 0) {
        o.tile_sums[(size_t)blockIdx.x * kTileSums + 1] = epair;
        o.tile_sums[(size_t)blockIdx.x * kTileSums + 2] = v2;
    }
}

template <int IPT, int PREC>
hipError_t launch_ipt(bool force, int stage, bool energy, const SymLaunch &L, const SweepBuffers &B,
                      const ForceOut &fo, const PotConst &pc, hipStream_t s) {
    (void)hipGetLastError();
    if (stage == 0 && L.nitems > 0) {
        if (force && energy)
            hipLaunchKernelGGL((k_sym_force<IPT, PREC, true>), dim3(L.nitems), dim3(64), 0, s, L.items, L.order,
                               L.tiles, B.xp, L.ipart, L.jpart, pc);
        else if (force)
            hipLaunchKernelGGL((k_sym_force<IPT, PREC, false>), dim3(L.nitems), dim3(64), 0, s, L.items, L.order,
                               L.tiles, B.xp, L.ipart, L.jpart, pc);
        else
            hipLaunchKernelGGL((k_sym_density<IPT, PREC>), dim3(L.nitems), dim3(64), 0, s, L.items, L.order, L.tiles,
                               B.rp, L.ipart, L.jpart, pc);
    }
    if (stage == 1 && L.ntiles > 0) {
        if (force) {
            if (energy)
                hipLaunchKernelGGL((k_sym_force_reduce<IPT, true>), dim3(L.ntiles), dim3(kSymRed), 0, s, L.tiles,
                                   L.ipart, L.jpart, fo, pc);
            else
                hipLaunchKernelGGL((k_sym_force_reduce<IPT, false>), dim3(L.ntiles), dim3(kSymRed), 0, s, L.tiles,
                                   L.ipart, L.jpart, fo, pc);
        } else {
            const DensityOut o{B.rp, B.xp, B.rho, B.tile_sums};
            hipLaunchKernelGGL((k_sym_density_reduce<IPT>), dim3(L.ntiles), dim3(kSymRed), 0, s, L.tiles, L.ipart,
                               L.jpart, o, pc);
        }
    }
    return hipGetLastError();
}

template <int PREC>
hipError_t dispatch_ipt(bool force, int stage, bool energy, const SymLaunch &L, const SweepBuffers &B,
                        const ForceOut &fo, const PotConst &pc, hipStream_t s) {
    switch (L.ipt) {
        case 2: return launch_ipt<2, PREC>(force, stage, energy, L, B, fo, pc, s);
        case 4: return launch_ipt<4, PREC>(force, stage, energy, L, B, fo, pc, s);
        case 8: return launch_ipt<8, PREC>(force, stage, energy, L, B, fo, pc, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_sym_density(const SymLaunch &L, const SweepBuffers &B, const PotConst &pc, int precision,
                              int stage, hipStream_t s) {
    if (pc.generic || pc.cut) return hipErrorInvalidValue;
    return precision == SCMD_FP64 ? dispatch_ipt<SCMD_FP64>(false, stage, true, L, B, ForceOut{}, pc, s)
                                  : dispatch_ipt<SCMD_MIXED>(false, stage, true, L, B, ForceOut{}, pc, s);
}

hipError_t launch_sym_force(const SymLaunch &L, const SweepBuffers &B, const StepArgs &a, const PotConst &pc,
                            int precision, int stage, hipStream_t s) {
    if (pc.generic || pc.cut) return hipErrorInvalidValue;
    const ForceOut fo{B.f, B.v, B.tile_sums, a.h, a.advance};
    const bool energy = a.energy != 0;
    return precision == SCMD_FP64 ? dispatch_ipt<SCMD_FP64>(true, stage, energy, L, B, fo, pc, s)
                                  : dispatch_ipt<SCMD_MIXED>(true, stage, energy, L, B, fo, pc, s);
}

}  // namespace scmd
