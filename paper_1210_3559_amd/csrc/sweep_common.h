// Device code shared by the pair-sweep kernels (all-pairs and cell list):
// pair arithmetic, fixed-order workgroup reductions and the per-tile and
// per-cluster epilogues that finish a sweep once every partial sum of a tile
// (or every tile of a cluster) has arrived.
#pragma once

#include "../../include/scmd.h"
#include "scmd_internal.h"

namespace scmd {
namespace dev {

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
// Density term: acc += u^m (minus rc^-m inside the cutoff when CUT), u = 1/r.
// MASK: the pair is void (self pair or outside the cutoff) when `off`.
// ---------------------------------------------------------------------------
template <int PREC, bool GEN, bool MASK, bool CUT>
__device__ __forceinline__ void density_pair(double dx, double dy, double dz, bool self, double &acc,
                                             const PotConst &pc) {
    if constexpr (PREC == SCMD_FP64) {
        double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        bool off = false;
        if constexpr (CUT) off = !(r2 < pc.rc2);
        if constexpr (MASK) off = off || self;
        if constexpr (MASK || CUT) r2 = off ? kSelfR2 : r2;
        double t;
        if constexpr (!GEN) {
            double w = rcp_nr(r2);  // u^2
            t = w * w * w;
        } else {
            t = (pc.m & 1) == 0 ? powi(rcp_nr(r2), pc.m >> 1) : powi(rsq_nr(r2), pc.m);
        }
        if constexpr (CUT) {
            acc += off ? 0.0 : t - pc.inv_rc_m;
        } else {
            acc += t;
        }
    } else {
        // mixed: r_i - r_j and r^2 in double (the cutoff decision matches the
        // double path), the powers in single precision, the sum in double
        const double r2d = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        bool off = false;
        if constexpr (CUT) off = !(r2d < pc.rc2);
        if constexpr (MASK) off = off || self;
        float r2 = (float)r2d;
        if constexpr (MASK || CUT) r2 = off ? kSelfR2f : r2;
        float t;
        if constexpr (!GEN) {
            float w = __builtin_amdgcn_rcpf(r2);
            t = w * w * w;
        } else {
            t = (pc.m & 1) == 0 ? powi(__builtin_amdgcn_rcpf(r2), pc.m >> 1) : powi(__builtin_amdgcn_rsqf(r2), pc.m);
        }
        if constexpr (CUT) {
            acc += off ? 0.0 : (double)t - pc.inv_rc_m;
        } else {
            acc += (double)t;
        }
    }
}

// ---------------------------------------------------------------------------
// Force and pair-energy terms:
//   F_i += u^(m+2) [A u^(n-m) - P_i - P_j] (r_i - r_j),  eu += u^n (- rc^-n).
// ci = -P_i, pj = P_j (single-precision copies for the mixed form).
// ---------------------------------------------------------------------------
template <int PREC, bool GEN, bool MASK, bool CUT>
__device__ __forceinline__ void force_pair(double dx, double dy, double dz, bool self, double ci, double pj,
                                           float cif, float pjf, double &fx, double &fy, double &fz, double &eu,
                                           const PotConst &pc, float Af) {
    if constexpr (PREC == SCMD_FP64) {
        double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        bool off = false;
        if constexpr (CUT) off = !(r2 < pc.rc2);
        if constexpr (MASK) off = off || self;
        if constexpr (MASK || CUT) r2 = off ? kSelfR2 : r2;
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
        if constexpr (CUT) {
            eu += off ? 0.0 : un - pc.inv_rc_n;
        } else {
            eu += un;
        }
    } else {
        const double r2d = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        bool off = false;
        if constexpr (CUT) off = !(r2d < pc.rc2);
        if constexpr (MASK) off = off || self;
        float r2 = (float)r2d;
        if constexpr (MASK || CUT) r2 = off ? kSelfR2f : r2;
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
        if constexpr (CUT) {
            eu += off ? 0.0 : (double)un - pc.inv_rc_n;
        } else {
            eu += (double)un;
        }
    }
}

// ---------------------------------------------------------------------------
// Workgroup helpers
// ---------------------------------------------------------------------------
// Fixed-shape tree sum over a workgroup of BLOCK threads (deterministic).
// sh needs BLOCK doubles.  Every thread of the workgroup must call it.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Sum of `n` consecutive slots of a partial array (fixed order, loads issued
// ahead of the adds).
__device__ __forceinline__ double sum_slots(const double *__restrict__ p, int n, size_t stride) {
    double s = 0.0;
    int k = 0;
    for (; k + 4 <= n; k += 4) {
        const double a = p[(size_t)k * stride];
        const double b = p[(size_t)(k + 1) * stride];
        const double c = p[(size_t)(k + 2) * stride];
        const double d = p[(size_t)(k + 3) * stride];
        s += a;
        s += b;
        s += c;
        s += d;
    }
    for (; k < n; ++k) s += p[(size_t)k * stride];
    return s;
}

// ---------------------------------------------------------------------------
// Epilogues
// ---------------------------------------------------------------------------
struct DensityOut {
    const double4 *rp;  // positions
    double4 *xp;        // positions + P, read by the force sweep
    double *rho;
    double *tile_sums;
};

// Finish one atom of the density sweep from its complete sum of u^m.
__device__ __forceinline__ double density_atom(int i, double s, const DensityOut &o, const PotConst &pc) {
    const double r = pc.am * s;
    const double sq = sqrt(r);
    const double psi = r > 0.0 ? 1.0 / sq : 0.0;
    const double4 q = o.rp[i];
    o.rho[i] = r;
    o.xp[i] = make_double4(q.x, q.y, q.z, pc.Pscale * psi);
    return -pc.eps_c * sq;  // embedding energy of atom i
}

struct ForceOut {
    double4 *f;
    double4 *v;
    double *tile_sums;
    double h;
    int advance;
};

struct FinalizeArgs {
    const ClusterDesc *cd;
    ClusterState *st;
    const double *tile_sums;
    int *flag;
    double mass_u, dt;
    int advance;
};

// Finish one atom of the force sweep: store F and the site pair energy,
// second half-kick when advancing; returns (pair energy, v^2) through refs.
__device__ __forceinline__ void force_atom(int i, double fx, double fy, double fz, double eu, const ForceOut &o,
                                           const PotConst &pc, double &epair, double &v2) {
#pragma clang fp contract(off)
    const double ei = pc.half_eps_an * eu;
    o.f[i] = make_double4(fx, fy, fz, ei);
    double4 vi = o.v[i];
    if (o.advance) {
        vi.x = vi.x + o.h * fx;
        vi.y = vi.y + o.h * fy;
        vi.z = vi.z + o.h * fz;
        o.v[i] = vi;
    }
    epair += ei;
    v2 += vi.x * vi.x + vi.y * vi.y + vi.z * vi.z;
}

// Per-cluster finish, run by one whole workgroup per cluster: fixed-order
// sums of the tile sums, then temperature and the Berendsen factor.
// Returns the cluster's current thermostat factor to thread 0.
template <int BLOCK>
__device__ double cluster_finalize(int c, const FinalizeArgs &o, double *sh) {
    const ClusterDesc d = o.cd[c];
    double emb = 0.0, epair = 0.0, v2 = 0.0;
    for (int t = threadIdx.x; t < d.ntiles; t += BLOCK) {
        const double *ts = o.tile_sums + (size_t)(d.tile0 + t) * kTileSums;
        emb += ts[0];
        epair += ts[1];
        v2 += ts[2];
    }
    emb = block_sum<BLOCK>(emb, sh);
    epair = block_sum<BLOCK>(epair, sh);
    v2 = block_sum<BLOCK>(v2, sh);
    if (threadIdx.x != 0) return 1.0;
    ClusterState s = o.st[c];
    const double ke = 0.5 * o.mass_u * v2 * kEvPerUA2Fs2;
    const double T = d.ndof > 0 ? 2.0 * ke / ((double)d.ndof * kBoltzmannEv) : 0.0;
    double lam = s.lambda;
    if (o.advance) {
        s.step += 1;
        lam = 1.0;
        s.ttarget = 0.0;
        if (d.kind == SCMD_BERENDSEN) {
            double tt = d.T_end;
            if (d.ramp > 0) {
                const int64_t k = s.step < d.ramp ? s.step : d.ramp;
                tt = d.T_start + (d.T_end - d.T_start) * (double)k / (double)d.ramp;
            }
            s.ttarget = tt;
            if (T > 0.0) {
                const double x = 1.0 + (o.dt / d.tau) * (tt / T - 1.0);
                lam = x > 0.0 ? sqrt(x) : 0.0;
            }
        }
        s.lambda = lam;
    }
    s.epot = emb + epair;
    s.ekin = lam * lam * ke;
    s.temp = lam * lam * T;
    if (!isfinite(s.epot) || !isfinite(s.ekin)) {
        s.nonfinite = 1;
        atomicOr(o.flag, 1);
    }
    o.st[c] = s;
    return s.lambda;
}

}  // namespace dev
}  // namespace scmd
