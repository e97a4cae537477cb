// All-pairs Sutton-Chen sweeps for gfx950 (one-sided: every atom owns its sums).
//
// The paper reduces the many-body force to two successive two-body sweeps:
// first every density rho_i (Sec. 2.1 Eq. (rho)), then the forces, which need
// psi_j = rho_j^(-1/2) of every partner (Sec. 2 "Computational approach").
//
// Work decomposition: an item is an atom tile (BLOCK*IPT atoms, IPT per
// lane) against a contiguous j chunk of the same cluster.  The j index is
// uniform across the wavefront, so partner data (x, y, z, P_j packed in one
// 32-byte double4) is fetched with scalar loads into SGPRs and read directly
// as a VALU operand: no LDS traffic and no barriers in the inner loop, and
// each partner fetched once per wave serves 64*IPT pairs from registers.
// Partial sums go to per-item slots and are reduced in a fixed order by the
// reduce kernels, so results are deterministic.
//
// Self pairs: the j range is split into the part that overlaps the tile's own
// atoms (where j == i is masked by pushing r^2 to a huge value, which makes
// every power term exactly zero) and the parts that do not (no mask at all).
#include "scmd_internal.h"
#include "../../include/scmd.h"

namespace scmd {
namespace {

constexpr double kSelfR2 = 1.0e300;
constexpr float kSelfR2f = 1.0e30f;

// 1/x in double: hardware estimate (about 2^-23 relative) refined by one
// Newton-Raphson step e = 1 - x y, y += y e (relative error ~ e^2).
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}

// 1/sqrt(x) in double: hardware estimate refined by one Newton-Raphson step
// y <- y (3/2 - (x/2) y^2) (relative error ~ 1.5 e^2).
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double hx = 0.5 * x;
    double e = __builtin_fma(-hx, y * y, 1.5);
    return y * e;
}

template <typename T>
__device__ __forceinline__ T powi(T x, int k) {
    T r = T(1);
    T b = x;
    while (k > 0) {
        if (k & 1) r *= b;
        b *= b;
        k >>= 1;
    }
    return r;
}

// ---------------------------------------------------------------------------
// Density term u^m = (1/r)^m for one pair.
// ---------------------------------------------------------------------------
template <int PREC, bool GEN, bool MASK>
__device__ __forceinline__ void density_pair(double dx, double dy, double dz, bool self, double &acc,
                                             const PotConst &pc) {
    if constexpr (PREC == SCMD_FP64) {
        double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        if constexpr (MASK) r2 = self ? kSelfR2 : r2;
        if constexpr (!GEN) {
            double w = rcp_nr(r2);           // u^2
            acc = __builtin_fma(w * w, w, acc);  // + u^6
        } else {
            if ((pc.m & 1) == 0) {
                acc += powi(rcp_nr(r2), pc.m >> 1);
            } else {
                acc += powi(rsq_nr(r2), pc.m);
            }
        }
    } else {
        float fx = (float)dx, fy = (float)dy, fz = (float)dz;
        float r2 = __builtin_fmaf(fx, fx, __builtin_fmaf(fy, fy, fz * fz));
        if constexpr (MASK) r2 = self ? kSelfR2f : r2;
        if constexpr (!GEN) {
            float w = __builtin_amdgcn_rcpf(r2);
            acc += (double)(w * w * w);
        } else {
            if ((pc.m & 1) == 0) {
                acc += (double)powi(__builtin_amdgcn_rcpf(r2), pc.m >> 1);
            } else {
                acc += (double)powi(__builtin_amdgcn_rsqf(r2), pc.m);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Force and pair-energy terms for one pair:
//   F_i += u^(m+2) [A u^(n-m) - P_i - P_j] (r_i - r_j),  eu += u^n.
// ci = -P_i, pj = P_j.
// ---------------------------------------------------------------------------
template <int PREC, bool GEN, bool MASK>
__device__ __forceinline__ void force_pair(double dx, double dy, double dz, bool self, double ci, double pj,
                                           float cif, float pjf, double &fx, double &fy, double &fz, double &eu,
                                           const PotConst &pc, float Af) {
    if constexpr (PREC == SCMD_FP64) {
        double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        if constexpr (MASK) r2 = self ? kSelfR2 : r2;
        double u = rsq_nr(r2);
        double f, un;
        if constexpr (!GEN) {
            double u2 = u * u;
            double u3 = u2 * u;
            double u4 = u2 * u2;
            double u8 = u4 * u4;
            double q = __builtin_fma(pc.A, u3, ci) - pj;
            f = u8 * q;
            un = u8 * u;
        } else {
            double um2 = powi(u, pc.m + 2);
            double und = powi(u, pc.n - pc.m);
            double q = __builtin_fma(pc.A, und, ci) - pj;
            f = um2 * q;
            un = powi(u, pc.n);
        }
        fx = __builtin_fma(f, dx, fx);
        fy = __builtin_fma(f, dy, fy);
        fz = __builtin_fma(f, dz, fz);
        eu += un;
    } else {
        float sx = (float)dx, sy = (float)dy, sz = (float)dz;
        float r2 = __builtin_fmaf(sx, sx, __builtin_fmaf(sy, sy, sz * sz));
        if constexpr (MASK) r2 = self ? kSelfR2f : r2;
        float u = __builtin_amdgcn_rsqf(r2);
        float f, un;
        if constexpr (!GEN) {
            float u2 = u * u;
            float u3 = u2 * u;
            float u4 = u2 * u2;
            float u8 = u4 * u4;
            float q = __builtin_fmaf(Af, u3, cif) - pjf;
            f = u8 * q;
            un = u8 * u;
        } else {
            float um2 = powi(u, pc.m + 2);
            float und = powi(u, pc.n - pc.m);
            float q = __builtin_fmaf(Af, und, cif) - pjf;
            f = um2 * q;
            un = powi(u, pc.n);
        }
        double fd = (double)f;
        fx = __builtin_fma(fd, dx, fx);
        fy = __builtin_fma(fd, dy, fy);
        fz = __builtin_fma(fd, dz, fz);
        eu += (double)un;
    }
}

// ---------------------------------------------------------------------------
// j loops (uniform j: partner data comes through scalar loads)
// ---------------------------------------------------------------------------
template <int IPT, int PREC, bool GEN, bool MASK>
__device__ __forceinline__ void density_range(const double4 *__restrict__ rp, int ja, int jb, const double *xi,
                                              const double *yi, const double *zi, const int *gi, double *acc,
                                              const PotConst &pc) {
#pragma unroll 4
    for (int j = ja; j < jb; ++j) {
        const double4 q = rp[j];
#pragma unroll
        for (int p = 0; p < IPT; ++p) {
            density_pair<PREC, GEN, MASK>(xi[p] - q.x, yi[p] - q.y, zi[p] - q.z, MASK && gi[p] == j, acc[p], pc);
        }
    }
}

template <int IPT, int PREC, bool GEN, bool MASK>
__device__ __forceinline__ void force_range(const double4 *__restrict__ rp, int ja, int jb, const double *xi,
                                            const double *yi, const double *zi, const double *ci, const float *cif,
                                            const int *gi, double *fx, double *fy, double *fz, double *eu,
                                            const PotConst &pc, float Af) {
#pragma unroll 2
    for (int j = ja; j < jb; ++j) {
        const double4 q = rp[j];
        const float pjf = PREC == SCMD_FP64 ? 0.0f : (float)q.w;
#pragma unroll
        for (int p = 0; p < IPT; ++p) {
            force_pair<PREC, GEN, MASK>(xi[p] - q.x, yi[p] - q.y, zi[p] - q.z, MASK && gi[p] == j, ci[p], q.w,
                                        cif[p], pjf, fx[p], fy[p], fz[p], eu[p], pc, Af);
        }
    }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
template <int BLOCK, int IPT, int PREC, bool GEN>
__global__ __launch_bounds__(BLOCK) void k_density(const SweepItem *__restrict__ items,
                                                   const int32_t *__restrict__ order,
                                                   const double4 *__restrict__ rp, double *__restrict__ part,
                                                   PotConst pc) {
    constexpr int TILE = BLOCK * IPT;
    const SweepItem it = items[order[blockIdx.x]];
    double xi[IPT], yi[IPT], zi[IPT], acc[IPT];
    int gi[IPT];
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        const int li = p * BLOCK + (int)threadIdx.x;
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
    const int lo = max(it.j0, it.i0);
    const int hi = min(it.j1, it.i0 + it.ni);
    if (lo < hi) {
        density_range<IPT, PREC, GEN, false>(rp, it.j0, lo, xi, yi, zi, gi, acc, pc);
        density_range<IPT, PREC, GEN, true>(rp, lo, hi, xi, yi, zi, gi, acc, pc);
        density_range<IPT, PREC, GEN, false>(rp, hi, it.j1, xi, yi, zi, gi, acc, pc);
    } else {
        density_range<IPT, PREC, GEN, false>(rp, it.j0, it.j1, xi, yi, zi, gi, acc, pc);
    }
    double *out = part + (size_t)it.slot * TILE;
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        const int li = p * BLOCK + (int)threadIdx.x;
        if (li < it.ni) out[li] = acc[p];
    }
}

template <int BLOCK, int IPT, int PREC, bool GEN>
__global__ __launch_bounds__(BLOCK) void k_force(const SweepItem *__restrict__ items,
                                                 const int32_t *__restrict__ order,
                                                 const double4 *__restrict__ rp, double *__restrict__ part,
                                                 PotConst pc) {
    constexpr int TILE = BLOCK * IPT;
    const SweepItem it = items[order[blockIdx.x]];
    const float Af = (float)pc.A;
    double xi[IPT], yi[IPT], zi[IPT], ci[IPT], fx[IPT], fy[IPT], fz[IPT], eu[IPT];
    float cif[IPT];
    int gi[IPT];
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        const int li = p * BLOCK + (int)threadIdx.x;
        fx[p] = fy[p] = fz[p] = eu[p] = 0.0;
        if (li < it.ni) {
            gi[p] = it.i0 + li;
            const double4 q = rp[gi[p]];
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
    const int lo = max(it.j0, it.i0);
    const int hi = min(it.j1, it.i0 + it.ni);
    if (lo < hi) {
        force_range<IPT, PREC, GEN, false>(rp, it.j0, lo, xi, yi, zi, ci, cif, gi, fx, fy, fz, eu, pc, Af);
        force_range<IPT, PREC, GEN, true>(rp, lo, hi, xi, yi, zi, ci, cif, gi, fx, fy, fz, eu, pc, Af);
        force_range<IPT, PREC, GEN, false>(rp, hi, it.j1, xi, yi, zi, ci, cif, gi, fx, fy, fz, eu, pc, Af);
    } else {
        force_range<IPT, PREC, GEN, false>(rp, it.j0, it.j1, xi, yi, zi, ci, cif, gi, fx, fy, fz, eu, pc, Af);
    }
    double *out = part + (size_t)it.slot * 4 * TILE;
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
        const int li = p * BLOCK + (int)threadIdx.x;
        if (li < it.ni) {
            out[li] = fx[p];
            out[TILE + li] = fy[p];
            out[2 * TILE + li] = fz[p];
            out[3 * TILE + li] = eu[p];
        }
    }
}

template <int BLOCK, int IPT, int PREC, bool GEN>
hipError_t launch_shape(bool force, const SweepLaunch &L, const double4 *rp, double *part, const PotConst &pc,
                        hipStream_t s) {
    if (L.nitems <= 0) return hipSuccess;
    if (force) {
        hipLaunchKernelGGL((k_force<BLOCK, IPT, PREC, GEN>), dim3(L.nitems), dim3(BLOCK), 0, s, L.items, L.order,
                           rp, part, pc);
    } else {
        hipLaunchKernelGGL((k_density<BLOCK, IPT, PREC, GEN>), dim3(L.nitems), dim3(BLOCK), 0, s, L.items,
                           L.order, rp, part, pc);
    }
    return hipGetLastError();
}

template <int PREC, bool GEN>
hipError_t dispatch_shape(bool force, const SweepLaunch &L, const double4 *rp, double *part, const PotConst &pc,
                          hipStream_t s) {
    if constexpr (GEN) {
        // the generic-exponent path exists in one launch shape only
        if (L.block == 256 && L.ipt == 1) return launch_shape<256, 1, PREC, true>(force, L, rp, part, pc, s);
        return hipErrorInvalidValue;
    } else {
#define SCMD_SHAPE(B, I) \
    if (L.block == B && L.ipt == I) return launch_shape<B, I, PREC, false>(force, L, rp, part, pc, s);
        SCMD_SHAPE(64, 1)
        SCMD_SHAPE(64, 2)
        SCMD_SHAPE(64, 4)
        SCMD_SHAPE(128, 1)
        SCMD_SHAPE(128, 2)
        SCMD_SHAPE(128, 4)
        SCMD_SHAPE(256, 1)
        SCMD_SHAPE(256, 2)
        SCMD_SHAPE(256, 4)
#undef SCMD_SHAPE
        return hipErrorInvalidValue;
    }
}

hipError_t dispatch(bool force, const SweepLaunch &L, const double4 *rp, double *part, const PotConst &pc,
                    int precision, hipStream_t s) {
    if (precision == SCMD_FP64) {
        return pc.generic ? dispatch_shape<SCMD_FP64, true>(force, L, rp, part, pc, s)
                          : dispatch_shape<SCMD_FP64, false>(force, L, rp, part, pc, s);
    }
    return pc.generic ? dispatch_shape<SCMD_MIXED, true>(force, L, rp, part, pc, s)
                      : dispatch_shape<SCMD_MIXED, false>(force, L, rp, part, pc, s);
}

}  // namespace

hipError_t launch_density(const SweepLaunch &L, const double4 *rp, double *part, const PotConst &pc, int precision,
                          hipStream_t s) {
    return dispatch(false, L, rp, part, pc, precision, s);
}

hipError_t launch_force(const SweepLaunch &L, const double4 *rp, double *part, const PotConst &pc, int precision,
                        hipStream_t s) {
    return dispatch(true, L, rp, part, pc, precision, s);
}

}  // namespace scmd
