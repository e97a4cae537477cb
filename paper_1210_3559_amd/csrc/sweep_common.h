// Device code shared by the pair-sweep kernels (all-pairs and cell list):
// pair arithmetic, fixed-order workgroup reductions and the per-tile and
// per-cluster epilogues that finish a sweep once every partial sum of a tile
// (or every tile of a cluster) has arrived.
#pragma once

#include "../../include/scmd.h"
#include "bath.h"
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
//
// The FP64 (n, m) = (9, 6) form works with w = 2u: the Newton step for
// 1/sqrt(r^2) written without its factor 1/2, w = y (3 - r^2 y^2), is exactly
// twice y (3/2 - (r^2/2) y^2) (scaling by 2 commutes with rounding), so one
// multiply per pair drops out.  With A/8 in place of A every later product
// is an exact power-of-two multiple of the unscaled one: the force sums come
// out 2^8 and the u^n sums 2^9 times too large, and unscale_force() divides
// them out once per sum.  The results are bitwise those of the form with u.
// ---------------------------------------------------------------------------
template <int PREC, bool GEN>
struct ForceScale {
    static constexpr double f = 1.0, e = 1.0;
};
template <>
struct ForceScale<SCMD_FP64, false> {
    static constexpr double f = 1.0 / 256.0, e = 1.0 / 512.0;
};

template <int PREC, bool GEN>
__device__ __forceinline__ void unscale_force(double &fx, double &fy, double &fz, double &eu) {
    if constexpr (ForceScale<PREC, GEN>::f != 1.0) {
        fx *= ForceScale<PREC, GEN>::f;
        fy *= ForceScale<PREC, GEN>::f;
        fz *= ForceScale<PREC, GEN>::f;
        eu *= ForceScale<PREC, GEN>::e;
    }
}

// 2/sqrt(x) from the hardware estimate and one Newton step (see above).
__device__ __forceinline__ double rsq2_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * __builtin_fma(-x, y * y, 3.0);
}

template <int PREC, bool GEN, bool MASK, bool CUT, bool EN = true>
__device__ __forceinline__ void force_pair(double dx, double dy, double dz, bool self, double ci, double pj,
                                           float cif, float pjf, double &fx, double &fy, double &fz, double &eu,
                                           const PotConst &pc, float Af) {
    if constexpr (PREC == SCMD_FP64) {
        double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        bool off = false;
        if constexpr (CUT) off = !(r2 < pc.rc2);
        if constexpr (MASK) off = off || self;
        if constexpr (MASK || CUT) r2 = off ? kSelfR2 : r2;
        double f, un;
        if constexpr (!GEN) {
            const double w = rsq2_nr(r2);  // 2u
            const double w2 = w * w;
            const double w3 = w2 * w;
            const double w4 = w2 * w2;
            const double w8 = w4 * w4;
            const double q = __builtin_fma(pc.A8, w3, ci) - pj;
            f = w8 * q;   // 2^8 x the force coefficient
            if constexpr (EN) un = w8 * w;  // 2^9 u^n
        } else {
            double u = rsq_nr(r2);
            double um2 = powi(u, pc.m + 2);
            double und = powi(u, pc.n - pc.m);
            double q = __builtin_fma(pc.A, und, ci) - pj;
            f = um2 * q;
            un = powi(u, pc.n);
        }
        fx = __builtin_fma(f, dx, fx);
        fy = __builtin_fma(f, dy, fy);
        fz = __builtin_fma(f, dz, fz);
        if constexpr (!EN) {
        } else if constexpr (CUT) {
            eu += off ? 0.0 : un - (GEN ? pc.inv_rc_n : pc.inv_rc_n512);
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
            if constexpr (EN) un = u8 * u;
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
        if constexpr (!EN) {
        } else if constexpr (CUT) {
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

// Finish one atom of the density sweep from its complete sum of u^m; q is
// its position.
__device__ __forceinline__ double density_atom_at(int i, double s, const double4 &q, const DensityOut &o,
                                                  const PotConst &pc) {
    const double r = pc.am * s;
    const double sq = sqrt(r);
    const double psi = r > 0.0 ? 1.0 / sq : 0.0;
    o.rho[i] = r;
    o.xp[i] = make_double4(q.x, q.y, q.z, pc.Pscale * psi);
    return -pc.eps_c * sq;  // embedding energy of atom i
}

__device__ __forceinline__ double density_atom(int i, double s, const DensityOut &o, const PotConst &pc) {
    return density_atom_at(i, s, o.rp[i], o, pc);
}

struct ForceOut {
    double4 *f;
    double4 *v;
    double *tile_sums;
    double h;
    int advance;
    // row sweeps of a single cluster whose drift ran inside the density
    // sweep: the force epilogue also applies the thermostat factor st->lambda
    // and the first half-kick, and stores the drifted positions in rp
    int fused;
    const ClusterState *st;
    double4 *rp;
    double2 *dpv;  // drift inputs of the next step (p, v); Langevin: the drifted (r, v)
    double dth;    // dt h
    // bath epilogue of clusters in a Langevin bath: their baths, the run's step index
    const ClusterDesc *cd;
    int local;
    double dt, mass_u;
    int bath;  // clusters in a Langevin bath: 0 none, 1 all, 2 some (read per cluster)
};

struct FinalizeArgs {
    const ClusterDesc *cd;
    ClusterState *st;
    const double *tile_sums;
    int *flag;
    double mass_u, dt;
    int advance;
    int step_add;    // completed steps since st.step was last stored (ramp index = st.step + step_add)
    int store_step;  // 1: store st.step + step_add
};

// Finish one atom of the force sweep: store F and the site pair energy,
// second half-kick when advancing; returns (pair energy, v^2) through refs.
// vi is the atom's current velocity.
__device__ __forceinline__ void force_atom_v(int i, double fx, double fy, double fz, double eu, double4 vi,
                                             const ForceOut &o, const PotConst &pc, double &epair, double &v2) {
#pragma clang fp contract(off)
    const double ei = pc.half_eps_an * eu;
    o.f[i] = make_double4(fx, fy, fz, ei);
    if (o.advance) {
        vi.x = vi.x + o.h * fx;
        vi.y = vi.y + o.h * fy;
        vi.z = vi.z + o.h * fz;
        o.v[i] = vi;
    }
    epair += ei;
    v2 += vi.x * vi.x + vi.y * vi.y + vi.z * vi.z;
}

__device__ __forceinline__ void force_atom(int i, double fx, double fy, double fz, double eu, const ForceOut &o,
                                           const PotConst &pc, double &epair, double &v2) {
    force_atom_v(i, fx, fy, fz, eu, o.v[i], o, pc, epair, v2);
}

// Kinetic energy (eV) and temperature of a cluster from its sum of v^2.
struct KinT {
    double ke, T;
};
__device__ __forceinline__ KinT kinetic_temperature(const ClusterDesc &d, double mass_u, double v2) {
#pragma clang fp contract(off)
    const double ke = 0.5 * mass_u * v2 * kEvPerUA2Fs2;
    const double T = d.ndof > 0 ? 2.0 * ke / ((double)d.ndof * kBoltzmannEv) : 0.0;
    return KinT{ke, T};
}

// Thermostat factor after a step whose ramp index is step_now, at
// temperature T; *ttarget receives the target (0 without thermostat).  The
// Langevin bath acts inside the drift: its factor is 1.
__device__ __forceinline__ double thermostat_lambda(const ClusterDesc &d, double dt, double T, int64_t step_now,
                                                    double *ttarget) {
#pragma clang fp contract(off)
    double lam = 1.0;
    *ttarget = 0.0;
    if (d.kind == SCMD_LANGEVIN) *ttarget = ramp_target(d, step_now);
    if (d.kind == SCMD_BERENDSEN) {
        const double tt = ramp_target(d, step_now);
        *ttarget = tt;
        if (T > 0.0) {
            const double x = 1.0 + (dt / d.tau) * (tt / T - 1.0);
            lam = x > 0.0 ? sqrt(x) : 0.0;
        }
    }
    return lam;
}

// Fixed-order totals of a cluster's tile sums: threads 0..255 add every
// 256th tile, each of the four wavefronts folds its lanes with wave_total,
// and the four wavefront sums are added as (w0 + w1) + (w2 + w3).  Any
// workgroup of >= 256 threads gets the same bits; every thread must call it.
// sh needs 12 doubles.  With V2_ONLY only the v^2 column is read (the others
// come back as 0).
// Sum of a double over the 64 lanes of a fully active wavefront with DPP
// moves, in one fixed order: pairs and quads (quad_perm), 8 and 16 lanes
// (row_half_mirror, row_mirror), then the four rows of 16 (row_bcast15 into
// rows 1 and 3, row_bcast31 into rows 2 and 3); lane 63 ends with
// (r0 + r1) + (r2 + r3) and its value is returned to every lane.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add_src(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_total(double x) {
    x += dpp_add_src<0xB1, 0xF>(x);
    x += dpp_add_src<0x4E, 0xF>(x);
    x += dpp_add_src<0x141, 0xF>(x);
    x += dpp_add_src<0x140, 0xF>(x);
    x += dpp_add_src<0x142, 0xA>(x);
    x += dpp_add_src<0x143, 0xC>(x);
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), 63);
    return __hiloint2double(hi, lo);
}

constexpr int kTotBlock = 256;
template <bool V2_ONLY>
__device__ __forceinline__ void cluster_totals(const ClusterDesc &d, const double *tile_sums, double *sh,
                                               double &emb, double &epair, double &v2) {
    emb = epair = v2 = 0.0;
    const int t = threadIdx.x;
    if (t < kTotBlock) {
        // thread t adds slots t, t + kTotBlock, ... in that order; the loads
        // of kTotU of them are issued together (the cell list has thousands
        // of slots per cluster)
        constexpr int kTotU = 8;
        for (int k0 = t; k0 < d.ntiles; k0 += kTotU * kTotBlock) {
            double e[kTotU], p[kTotU], w[kTotU];
#pragma unroll
            for (int u = 0; u < kTotU; ++u) {
                const int k = k0 + u * kTotBlock;
                e[u] = p[u] = w[u] = 0.0;
                if (k < d.ntiles) {
                    const double *ts = tile_sums + (size_t)(d.tile0 + k) * kTileSums;
                    if constexpr (!V2_ONLY) {
                        e[u] = ts[0];
                        p[u] = ts[1];
                    }
                    w[u] = ts[2];
                }
            }
#pragma unroll
            for (int u = 0; u < kTotU; ++u) {
                if (k0 + u * kTotBlock < d.ntiles) {
                    if constexpr (!V2_ONLY) {
                        emb += e[u];
                        epair += p[u];
                    }
                    v2 += w[u];
                }
            }
        }
    }
    if constexpr (!V2_ONLY) {
        emb = wave_total(emb);
        epair = wave_total(epair);
    }
    v2 = wave_total(v2);
    if (t < kTotBlock && (t & 63) == 0) {
        const int w = t >> 6;
        sh[w] = emb;
        sh[4 + w] = epair;
        sh[8 + w] = v2;
    }
    __syncthreads();
    emb = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    epair = (sh[4] + sh[5]) + (sh[6] + sh[7]);
    v2 = (sh[8] + sh[9]) + (sh[10] + sh[11]);
    __syncthreads();
}

// Per-cluster finish, run by one whole workgroup (>= 256 threads): the
// totals of the tile sums, then temperature and the Berendsen factor.  Every
// workgroup that runs it for the same cluster and arguments gets the same
// result bit for bit; only a `writer` stores the cluster state (st.step only
// with store_step).  Returns the cluster's current thermostat factor to
// thread 0.  sh needs 12 doubles.
__device__ inline double cluster_finalize(int c, const FinalizeArgs &o, double *sh, bool writer) {
    // no contraction: the same rounding in every kernel that inlines this
#pragma clang fp contract(off)
    const ClusterDesc d = o.cd[c];
    double emb, epair, v2;
    cluster_totals<false>(d, o.tile_sums, sh, emb, epair, v2);
    if (threadIdx.x != 0) return 1.0;
    ClusterState s = o.st[c];
    const KinT kt = kinetic_temperature(d, o.mass_u, v2);
    double lam = s.lambda;
    const int64_t step_now = s.step + o.step_add;
    if (o.store_step) s.step = step_now;
    if (o.advance) {
        lam = thermostat_lambda(d, o.dt, kt.T, step_now, &s.ttarget);
        s.lambda = lam;
    }
    s.epot = emb + epair;
    s.ekin = lam * lam * kt.ke;
    s.temp = lam * lam * kt.T;
    if (!isfinite(s.epot) || !isfinite(s.ekin)) {
        s.nonfinite = 1;
        if (writer) atomicOr(o.flag, 1);
    }
    if (writer) o.st[c] = s;
    return s.lambda;
}

// ---------------------------------------------------------------------------
// Cell-list check (see CellCheck): per atom, then merged per workgroup.
// ---------------------------------------------------------------------------
// Doubles compared as signed 64-bit integers: flip the magnitude bits of
// negative values (an involution, so the same map decodes).
__device__ __forceinline__ long long ord_encode(double d) {
    const long long b = __double_as_longlong(d);
    return b >= 0 ? b : b ^ 0x7FFFFFFFFFFFFFFFLL;
}
__device__ __forceinline__ double ord_decode(long long b) {
    return __longlong_as_double(b >= 0 ? b : b ^ 0x7FFFFFFFFFFFFFFFLL);
}

struct CellBox {
    double m[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    bool moved = false;
};

__device__ __forceinline__ void cell_check_atom(const CellCheck &cc, int i, const double4 &q, CellBox &b) {
    const double4 o = cc.ref[i];
    const double ex = q.x - o.x, ey = q.y - o.y, ez = q.z - o.z;
    b.moved = b.moved || !(ex * ex + ey * ey + ez * ez <= cc.thr2);
    cc.rs[cc.slot_of[i]] = q;
    b.m[0] = fmin(b.m[0], q.x);
    b.m[1] = fmin(b.m[1], q.y);
    b.m[2] = fmin(b.m[2], q.z);
    b.m[3] = fmax(b.m[3], q.x);
    b.m[4] = fmax(b.m[4], q.y);
    b.m[5] = fmax(b.m[5], q.z);
}

// Every thread of the workgroup (BLOCK threads) calls this once with its
// accumulated box; min/max are exact, so neither the reduction order nor
// the atomic merge order matters.  sh: 6 x BLOCK/64 doubles.
template <int BLOCK>
__device__ __forceinline__ void cell_check_merge(const CellCheck &cc, int cluster, CellBox &b, double *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            b.m[d] = fmin(b.m[d], __shfl_xor(b.m[d], o, 64));
            b.m[3 + d] = fmax(b.m[3 + d], __shfl_xor(b.m[3 + d], o, 64));
        }
    }
    if (__ballot(b.moved) != 0ull && lane == 0) atomicOr(cc.flag, 1);
    if (lane == 0)
        for (int d = 0; d < 6; ++d) sh[d * (BLOCK / 64) + w] = b.m[d];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int d = threadIdx.x;
        double v = sh[d * (BLOCK / 64)];
        for (int k = 1; k < BLOCK / 64; ++k)
            v = d < 3 ? fmin(v, sh[d * (BLOCK / 64) + k]) : fmax(v, sh[d * (BLOCK / 64) + k]);
        if (d < 3) atomicMin(&cc.box[6 * cluster + d], ord_encode(v));
        else atomicMax(&cc.box[6 * cluster + d], ord_encode(v));
    }
}

}  // namespace dev
}  // namespace scmd
