// Row sweeps for small clusters: one workgroup holds every partner of a
// short run of atoms, so that a sweep finishes in one launch with no partial
// slots and no reduce kernel.
//
// The two sweeps are those of the paper's scheme (Sec. 2 "Computational
// approach": the density sums of Eq. (rho), then the forces of Eq. (SC)),
// evaluated one-sidedly: every atom accumulates its own sums.  A workgroup
// of 64*W threads owns atoms [i0, i0 + ni) of one cluster, ni <= 8 W.
//
// Threads form groups of 8 consecutive lanes; group g works for atom
// il = g % ni, and its lanes run the partner streams s = 8 (g / ni) + lane8,
// s < S = 8 floor(8 W / ni).  Stream s visits j = off + s, off + s + S, ...,
// so the S streams of an atom interleave over the whole cluster and the 8
// lanes of a group read 8 neighbouring partners.  The partner window
// [i0, i0 + ni), which holds the self pairs, and the last, partly filled
// round of each wavefront are the only masked iterations.
//
// When the cluster fits (at most kRowStageMax atoms), the workgroup first
// copies the cluster's positions into LDS (each thread issues all of its
// loads before storing any), so the pair loop reads LDS only.  Stream sums are added across
// the 8 lanes of a group with DPP (quad_perm, row_half_mirror), then across
// groups through LDS in a fixed order: the result is deterministic.  The
// workgroup then finishes its atoms: psi and the embedding energy after the
// density sweep, F, the second half-kick and the energy / v^2 sums after the
// force sweep.
#include "sweep_common.h"

namespace scmd {
namespace {

using namespace dev;

// floor(a / b) for b > 0 and any sign of a.
__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Thread layout of a row workgroup and the wave-uniform round ranges.
struct RowLayout {
    int ni, G, S;      // atoms, groups per atom, streams per atom (8 G)
    int il, s, i;      // this thread's atom (local, global) and stream
    bool active;       // this thread's group works for an atom
    int k_mask0, k_mask1;  // rounds [k_mask0, k_mask1) may meet the self window
    int k_full, k_end;     // rounds [0, k_full) are full for the whole wavefront; k_end: last round + 1
};

template <int W>
__device__ __forceinline__ RowLayout row_layout(int i0, int ni, int off, int n) {
    constexpr int NG = 8 * W;  // groups in the workgroup
    RowLayout L;
    L.ni = ni;
    L.G = NG / ni;
    L.S = 8 * L.G;
    const int tid = threadIdx.x;
    const int grp = tid >> 3, lane8 = tid & 7;
    const int nact = ni * L.G;  // active groups
    L.active = grp < nact;
    // idle groups shadow the last active group (valid addresses, results dropped)
    const int gg = L.active ? grp : nact - 1;
    L.il = gg % ni;
    L.s = 8 * (gg / ni) + lane8;
    L.i = i0 + L.il;
    // stream range of this wavefront (wave-uniform): groups 8w .. 8w+7
    const int wave = tid >> 6;
    const int g_lo = min(8 * wave, nact - 1), g_hi = min(8 * wave + 7, nact - 1);
    const int s_min = 8 * (g_lo / ni), s_max = 8 * (g_hi / ni) + 7;
    // rounds in which some thread of the wavefront meets j in [i0, i0 + ni)
    const int w0 = i0 - off, w1 = i0 + ni - 1 - off;
    const int klo = max(0, floor_div(w0 - s_max + L.S - 1, L.S));
    const int khi = floor_div(w1 - s_min, L.S);  // inclusive
    // rounds: a thread with stream s has ceil((n - s) / S) of them
    L.k_full = n > s_max ? (n - s_max + L.S - 1) / L.S : 0;
    L.k_end = n > s_min ? (n - s_min + L.S - 1) / L.S : 0;
    L.k_mask0 = min(klo, L.k_full);
    L.k_mask1 = max(L.k_mask0, min(khi + 1, L.k_full));
    return L;
}

// Double moved across lanes with a DPP control (all source lanes valid).
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 8 lanes of a group: pairs (quad_perm 1,0,3,2), quads
// (quad_perm 2,3,0,1), then the two quads (row_half_mirror).  Every lane of
// the group ends with the same value (commuted operands only).
__device__ __forceinline__ double group8_sum(double x) {
    x += dpp<0xB1>(x);
    x += dpp<0x4E>(x);
    x += dpp<0x141>(x);
    return x;
}

// Totals of Q values per atom: group sums with DPP, then per atom over its G
// groups in group order.  Returns the totals to threads t < ni (for atom t),
// zeros elsewhere.  sh holds Q * 8 W doubles.
template <int W, int Q>
__device__ __forceinline__ void row_reduce(const RowLayout &L, double (&v)[Q], double *sh) {
    constexpr int NG = 8 * W;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = group8_sum(L.active ? v[q] : 0.0);
    if ((tid & 7) == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) sh[q * NG + (tid >> 3)] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = 0.0;
    if (tid < L.ni) {
        int g = 0;
        for (; g + 4 <= L.G; g += 4) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const double a = sh[q * NG + tid + L.ni * g], b = sh[q * NG + tid + L.ni * (g + 1)];
                const double c = sh[q * NG + tid + L.ni * (g + 2)], d = sh[q * NG + tid + L.ni * (g + 3)];
                v[q] += a;
                v[q] += b;
                v[q] += c;
                v[q] += d;
            }
        }
        for (; g < L.G; ++g) {
#pragma unroll
            for (int q = 0; q < Q; ++q) v[q] += sh[q * NG + tid + L.ni * g];
        }
    }
}

// Wavefront sum (fixed DPP order, deterministic) of lanes 0..63; the whole
// wavefront must be active.
__device__ __forceinline__ double wave_sum(double x) { return wave_total(x); }

// The workgroup's tile: from the arguments for a single cluster with equal
// runs (no table loads), else from the tables in launch order.
struct RowTile {
    int tix, i0, ni, off, n;
    int c;       // cluster
    bool first;  // the cluster's first tile (writes its per-cluster results)
};

struct RowArgs {
    const ITile *tiles;
    const int32_t *order;
    const ClusterDesc *cd;
    int uni_off, uni_n, uni_ni;
};

__device__ __forceinline__ RowTile row_tile(const RowArgs &a) {
    RowTile r;
    if (a.uni_ni > 0) {
        r.tix = blockIdx.x;
        r.off = a.uni_off;
        r.n = a.uni_n;
        r.i0 = a.uni_off + r.tix * a.uni_ni;
        r.ni = min(a.uni_ni, a.uni_n - r.tix * a.uni_ni);
        r.c = 0;
        r.first = r.tix == 0;
    } else {
        r.tix = a.order[blockIdx.x];
        const ITile t = a.tiles[r.tix];
        const ClusterDesc d = a.cd[t.c];
        r.i0 = t.i0;
        r.ni = t.ni;
        r.off = d.off;
        r.n = d.n;
        r.c = t.c;
        r.first = r.tix == d.tile0;
    }
    return r;
}

// LDS of a row workgroup: the staged partners (STAGE) followed by the
// reduce area.
template <int W, int Q, bool STAGE>
constexpr size_t row_lds_bytes(int n) {
    return (STAGE ? (size_t)n * sizeof(double4) : 0) + (size_t)Q * 8 * W * sizeof(double);
}

// The partner loop over rounds k in [ka, kb) of this thread's stream: plain
// rounds in blocks of four through pointers stepped by 4 S, masked rounds
// (self window, end of the cluster) one by one.  src points at the cluster's
// first atom (LDS or global); pair(q, self) adds one partner.
template <typename PAIR>
__device__ __forceinline__ void row_loop(const RowLayout &L, const double4 *__restrict__ src, int n, int i_local,
                                         PAIR &&pair, int ka, int kb) {
    const int S = L.S;
    int k = ka;
    auto plain = [&](int k1) {
        if (k >= k1) return;
        const double4 *p0 = src + (L.s + (size_t)k * S);
        if (k + 4 <= k1) {
            const double4 *p1 = p0 + S, *p2 = p1 + S, *p3 = p2 + S;
            const size_t S4 = 4 * (size_t)S;
            for (; k + 4 <= k1; k += 4, p0 += S4, p1 += S4, p2 += S4, p3 += S4) {
                const double4 a = *p0, b = *p1, c = *p2, e = *p3;
                pair(a, false);
                pair(b, false);
                pair(c, false);
                pair(e, false);
            }
        }
        for (; k < k1; ++k, p0 += S) pair(*p0, false);
    };
    auto masked = [&](int k1) {
        for (int j = L.s + k * S; k < k1; ++k, j += S) {
            const bool valid = j < n;
            const double4 a = src[valid ? j : 0];
            pair(a, !valid || j == i_local);
        }
    };
    plain(min(kb, L.k_mask0));
    masked(min(kb, L.k_mask1));
    plain(min(kb, L.k_full));
    masked(min(kb, L.k_end));
}

// Staged sweeps copy the whole cluster into LDS before the pair loop.
// Every thread issues the loads of four atoms before it stores any of them
// (named registers: an array here would live in scratch), so four atoms per
// thread cost one memory round trip.  All workgroups read the same atoms, so
// the copy is bound by the L2-to-CU bandwidth (bytes per atom x workgroups).
// `mid` runs between the first loads and their stores (in every thread with
// threadIdx.x < n): ALU work placed there overlaps the memory round trip.
template <int W, typename Mid>
__device__ __forceinline__ void stage_copy(double4 *lj, const double4 *__restrict__ g, int n, Mid &&mid) {
    constexpr int T = 64 * W;
    bool first = true;
    for (int a0 = threadIdx.x; a0 < n; a0 += 4 * T) {
        const int a1 = a0 + T, a2 = a1 + T, a3 = a2 + T;
        double4 t0 = g[a0], t1, t2, t3;
        if (a1 < n) t1 = g[a1];
        if (a2 < n) t2 = g[a2];
        if (a3 < n) t3 = g[a3];
        if (first) {
            mid();
            first = false;
        }
        lj[a0] = t0;
        if (a1 < n) lj[a1] = t1;
        if (a2 < n) lj[a2] = t2;
        if (a3 < n) lj[a3] = t3;
    }
    __syncthreads();
}
template <int W>
__device__ __forceinline__ void stage_copy(double4 *lj, const double4 *__restrict__ g, int n) {
    stage_copy<W>(lj, g, n, [] {});
}

// Drift arguments of the density sweep (see RowDrift).
struct RowDriftArgs {
    int mode, local;
    int bath;  // clusters in a Langevin bath: 0 none, 1 all, 2 some (read per cluster)
    const double4 *v, *f;
    const double2 *dpv;
    ClusterState *st;
    const double *tile_sums;
    const ClusterDesc *cd;
    double mass_u, dt, h, dth;
};

// Drifted position p + (dt lambda) v with p = r + (dt h) F (RowDrift).
// Mode 1 reads r, v, F (x, y, z) and forms p; mode 2 reads p, v from the
// three pairs (px, py), (pz, vx), (vy, vz) stored per atom.
struct PV {
    double px, py, pz, vx, vy, vz;
};
__device__ __forceinline__ double4 xyz(const double4 *__restrict__ p, int a) {
    const double *q = reinterpret_cast<const double *>(p + a);
    return make_double4(q[0], q[1], q[2], 0.0);
}
__device__ __forceinline__ double pcomp(double r, double f, double dth) {
#pragma clang fp contract(off)
    return r + dth * f;
}
__device__ __forceinline__ PV pv_from_rvf(const double4 *__restrict__ r, const double4 *__restrict__ v,
                                          const double4 *__restrict__ f, int a, double dth) {
    const double4 ra = xyz(r, a), va = xyz(v, a), fa = xyz(f, a);
    return PV{pcomp(ra.x, fa.x, dth), pcomp(ra.y, fa.y, dth), pcomp(ra.z, fa.z, dth), va.x, va.y, va.z};
}
__device__ __forceinline__ PV pv_load(const double2 *__restrict__ d, int a) {
    const double2 q0 = d[3 * a], q1 = d[3 * a + 1], q2 = d[3 * a + 2];
    return PV{q0.x, q0.y, q1.x, q1.y, q2.x, q2.y};
}
__device__ __forceinline__ double4 drifted(const PV &q, double dtl) {
#pragma clang fp contract(off)
    return make_double4(q.px + dtl * q.vx, q.py + dtl * q.vy, q.pz + dtl * q.vz, 0.0);
}

// Force epilogue of a step whose drift ran inside the density sweep: the
// velocity gets the thermostat factor and the first half-kick with the old
// force (as in the drift kernel), then the second half-kick with the new one;
// the drifted position r (x, y, z of the density output) is stored.
__device__ __forceinline__ void force_atom_fused(int i, double fx, double fy, double fz, double eu, const double4 &r,
                                                 const double4 &v_old, const double4 &f_old, double lam,
                                                 const ForceOut &o, const PotConst &pc, double &epair, double &v2) {
#pragma clang fp contract(off)
    const double ei = pc.half_eps_an * eu;
    const double4 fo = f_old;
    double4 vi = v_old;
    vi.x = lam * vi.x;
    vi.y = lam * vi.y;
    vi.z = lam * vi.z;
    vi.x = vi.x + o.h * fo.x;
    vi.y = vi.y + o.h * fo.y;
    vi.z = vi.z + o.h * fo.z;
    o.f[i] = make_double4(fx, fy, fz, ei);
    vi.x = vi.x + o.h * fx;
    vi.y = vi.y + o.h * fy;
    vi.z = vi.z + o.h * fz;
    o.v[i] = vi;
    o.rp[i] = make_double4(r.x, r.y, r.z, 0.0);
    // drift inputs of the next step: p = r + (dt h) F, v
    double2 *d = o.dpv + 3 * (size_t)i;
    d[0] = make_double2(r.x + o.dth * fx, r.y + o.dth * fy);
    d[1] = make_double2(r.z + o.dth * fz, vi.x);
    d[2] = make_double2(vi.y, vi.z);
    epair += ei;
    v2 += vi.x * vi.x + vi.y * vi.y + vi.z * vi.z;
}

// Langevin epilogue (a cluster in a bath): the stored post-bath velocity gets
// the second half-kick; then the first half-kick of the next step with the
// same force and that step's A, O, A (bath.h), whose drifted (r, v) are
// stored for the next density sweep.  The order of operations is the same as
// in the drift kernel.
__device__ __forceinline__ void force_atom_bath(int i, double fx, double fy, double fz, double eu, const double4 &r,
                                                const double4 &v_bath, const double3 &xi_next, double c2_next,
                                                const ClusterDesc &d, const ForceOut &o, const PotConst &pc,
                                                double &epair, double &v2) {
#pragma clang fp contract(off)
    const double ei = pc.half_eps_an * eu;
    double4 vi = v_bath;
    vi.x = vi.x + o.h * fx;
    vi.y = vi.y + o.h * fy;
    vi.z = vi.z + o.h * fz;
    o.f[i] = make_double4(fx, fy, fz, ei);
    o.v[i] = vi;
    o.rp[i] = make_double4(r.x, r.y, r.z, 0.0);
    epair += ei;
    v2 += vi.x * vi.x + vi.y * vi.y + vi.z * vi.z;
    double4 rn = make_double4(r.x, r.y, r.z, 0.0);
    vi.x = vi.x + o.h * fx;
    vi.y = vi.y + o.h * fy;
    vi.z = vi.z + o.h * fz;
    // this is step st->step + local + 1 of the cluster; prepare the next one
    bath_drift_xi(d, c2_next, xi_next, o.dt, rn, vi);
    double2 *q = o.dpv + 3 * (size_t)i;
    q[0] = make_double2(rn.x, rn.y);
    q[1] = make_double2(rn.z, vi.x);
    q[2] = make_double2(vi.y, vi.z);
}

// ---------------------------------------------------------------------------
// Density sweep
// ---------------------------------------------------------------------------
template <int W, int PREC, bool GEN, bool STAGE>
__global__ __launch_bounds__(64 * W) void k_row_density(RowArgs ra, DensityOut o, PotConst pc, RowDriftArgs da) {
    extern __shared__ double4 lds_row[];
    const RowTile rt = row_tile(ra);
    const RowLayout L = row_layout<W>(rt.i0, rt.ni, rt.off, rt.n);
    const int i_local = L.i - rt.off;
    const int tid = threadIdx.x;
    double acc = 0.0;
    double4 qi;
    auto pair = [&](const double4 &a, bool self) {
        if (self)
            density_pair<PREC, GEN, true, false>(qi.x - a.x, qi.y - a.y, qi.z - a.z, true, acc, pc);
        else
            density_pair<PREC, GEN, false, false>(qi.x - a.x, qi.y - a.y, qi.z - a.z, false, acc, pc);
    };
    const double4 *src = o.rp + rt.off;
    double *sh = reinterpret_cast<double *>(lds_row);
    if constexpr (STAGE) {
        double4 *lj = lds_row;
        sh += 4 * (size_t)rt.n;
        if (da.mode == 0) {
            qi = src[i_local];
            stage_copy<W>(lj, src, rt.n);
        } else {
            // drift while staging.  The own atom and the first four atoms of
            // this thread are loaded before the thermostat factor is known
            // (named registers, see stage_copy), so the factor's tile-sum
            // loads overlap them; mode 2 reads the stored (p, v), mode 1
            // forms p.  A cluster in a Langevin bath has its drifted (r, v)
            // stored already (by the previous force epilogue, or before the
            // run's first step): it takes p + 0 v = p.
            ClusterState *sc = da.st + rt.c;
            const bool bath = da.bath == 1 || (da.bath == 2 && da.cd[rt.c].kind == SCMD_LANGEVIN);
            const double4 *gv = da.v + rt.off, *gf = da.f + rt.off;
            const double2 *gd = da.dpv + 3 * (size_t)rt.off;
            const bool stored = da.mode == 2 || bath;
            auto load = [&](int a) { return stored ? pv_load(gd, a) : pv_from_rvf(src, gv, gf, a, da.dth); };
            const PV own = load(i_local);
            constexpr int T = 64 * W;
            const int a0 = tid, a1 = a0 + T, a2 = a1 + T, a3 = a2 + T;
            PV t0, t1, t2, t3;
            if (a0 < rt.n) t0 = load(a0);
            if (a1 < rt.n) t1 = load(a1);
            if (a2 < rt.n) t2 = load(a2);
            if (a3 < rt.n) t3 = load(a3);
            __shared__ double sh_tot[12];
            double lam;
            if (bath) {
                lam = 0.0;
            } else if (da.mode == 2) {
                // finish the previous step's thermostat factor (finalize order)
                const ClusterDesc d = da.cd[rt.c];
                double e0, e1, v2;
                cluster_totals<true>(d, da.tile_sums, sh_tot, e0, e1, v2);
                const KinT kt = kinetic_temperature(d, da.mass_u, v2);
                double tt;
                lam = thermostat_lambda(d, da.dt, kt.T, sc->step + da.local, &tt);
                if (rt.first && tid == 0) sc->lambda = lam;
            } else {
                lam = sc->lambda;
            }
            const double dtl = da.dt * lam;
            qi = drifted(own, dtl);
            if (a0 < rt.n) lj[a0] = drifted(t0, dtl);
            if (a1 < rt.n) lj[a1] = drifted(t1, dtl);
            if (a2 < rt.n) lj[a2] = drifted(t2, dtl);
            if (a3 < rt.n) lj[a3] = drifted(t3, dtl);
            for (int b0 = tid + 4 * T; b0 < rt.n; b0 += 4 * T) {
                const int b1 = b0 + T, b2 = b1 + T, b3 = b2 + T;
                const PV u0 = load(b0);
                PV u1, u2, u3;
                if (b1 < rt.n) u1 = load(b1);
                if (b2 < rt.n) u2 = load(b2);
                if (b3 < rt.n) u3 = load(b3);
                lj[b0] = drifted(u0, dtl);
                if (b1 < rt.n) lj[b1] = drifted(u1, dtl);
                if (b2 < rt.n) lj[b2] = drifted(u2, dtl);
                if (b3 < rt.n) lj[b3] = drifted(u3, dtl);
            }
            __syncthreads();
        }
        row_loop(L, lj, rt.n, i_local, pair, 0, L.k_end);
        src = lj;
    } else {
        qi = src[i_local];
        row_loop(L, src, rt.n, i_local, pair, 0, L.k_end);
    }
    double v[1] = {acc};
    row_reduce<W, 1>(L, v, sh);
    double emb = 0.0;
    if (tid < L.ni) emb = density_atom_at(rt.i0 + tid, v[0], src[rt.i0 - rt.off + tid], o, pc);
    if (tid < 64) {
        emb = wave_sum(emb);
        if (tid == 0) o.tile_sums[(size_t)rt.tix * kTileSums + 0] = emb;
    }
}

// ---------------------------------------------------------------------------
// Force sweep
// ---------------------------------------------------------------------------
// EN: accumulate the pair energy (otherwise the energy sums are zero).
// BATH: some cluster of the launch is in a Langevin bath (the bath epilogue
// and its noise draw are compiled only then).
template <int W, int PREC, bool GEN, bool STAGE, bool EN, bool BATH>
__global__ __launch_bounds__(64 * W) void k_row_force(RowArgs ra, const double4 *__restrict__ xp, ForceOut o,
                                                      PotConst pc) {
    extern __shared__ double4 lds_row[];
    const RowTile rt = row_tile(ra);
    const RowLayout L = row_layout<W>(rt.i0, rt.ni, rt.off, rt.n);
    const int i_local = L.i - rt.off;
    const int tid = threadIdx.x;
    const double4 *src = xp + rt.off;
    const double4 qi = src[i_local];
    const double ci = -qi.w;
    const float cif = (float)ci;
    const float Af = (float)pc.A;
    double fx = 0.0, fy = 0.0, fz = 0.0, eu = 0.0;
    auto pair = [&](const double4 &a, bool self) {
        if (self)
            force_pair<PREC, GEN, true, false, EN>(qi.x - a.x, qi.y - a.y, qi.z - a.z, true, ci, a.w, cif,
                                                   (float)a.w, fx, fy, fz, eu, pc, Af);
        else
            force_pair<PREC, GEN, false, false, EN>(qi.x - a.x, qi.y - a.y, qi.z - a.z, false, ci, a.w, cif,
                                                    (float)a.w, fx, fy, fz, eu, pc, Af);
    };
    // the epilogue's own-atom loads are issued now, off the critical path
    double4 v_own = make_double4(0, 0, 0, 0), f_own = make_double4(0, 0, 0, 0);
    const bool bath = BATH && o.fused && (o.bath == 1 || (o.bath == 2 && o.cd[rt.c].kind == SCMD_LANGEVIN));
    if (tid < L.ni) {
        if (bath) {
            // Langevin: the post-bath velocity stored with the drifted position
            const double2 *q = o.dpv + 3 * (size_t)(rt.i0 + tid);
            const double2 q1 = q[1], q2 = q[2];
            v_own = make_double4(q1.y, q2.x, q2.y, 0.0);
        } else {
            v_own = o.v[rt.i0 + tid];
            if (o.fused) f_own = o.f[rt.i0 + tid];
        }
    }
    // Langevin: the next step's noise does not depend on the forces; it is
    // drawn while the staging loads are in flight
    double3 xi_next = make_double3(0.0, 0.0, 0.0);
    double c2_next = 0.0;
    auto draw = [&] {
        if (bath && tid < L.ni) {
            const int64_t next = o.st[rt.c].step + o.local + 2;
            xi_next = bath_noise(o.cd[rt.c].seed, next, rt.i0 - rt.off + tid);
            c2_next = bath_c2(o.cd[rt.c], next, o.mass_u);
        }
    };
    double *sh = reinterpret_cast<double *>(lds_row);
    if constexpr (STAGE) {
        double4 *lj = lds_row;
        sh += 4 * (size_t)rt.n;
        stage_copy<W>(lj, src, rt.n, draw);
        row_loop(L, lj, rt.n, i_local, pair, 0, L.k_end);
        src = lj;
    } else {
        draw();
        row_loop(L, src, rt.n, i_local, pair, 0, L.k_end);
    }
    unscale_force<PREC, GEN>(fx, fy, fz, eu);
    if constexpr (!EN) eu = 0.0;
    double v[4] = {fx, fy, fz, eu};
    row_reduce<W, 4>(L, v, sh);
    double epair = 0.0, v2 = 0.0;
    if (tid < L.ni) {
        const int i = rt.i0 + tid;
        if (bath)
            force_atom_bath(i, v[0], v[1], v[2], v[3], src[i - rt.off], v_own, xi_next, c2_next, o.cd[rt.c], o, pc,
                            epair, v2);
        else if (o.fused)
            force_atom_fused(i, v[0], v[1], v[2], v[3], src[i - rt.off], v_own, f_own, o.st[rt.c].lambda, o, pc,
                             epair, v2);
        else
            force_atom_v(i, v[0], v[1], v[2], v[3], v_own, o, pc, epair, v2);
    }
    if (tid < 64) {
        epair = wave_sum(epair);
        v2 = wave_sum(v2);
        if (tid == 0) {
            o.tile_sums[(size_t)rt.tix * kTileSums + 1] = epair;
            o.tile_sums[(size_t)rt.tix * kTileSums + 2] = v2;
        }
    }
}

// Allow the kernel the dynamic LDS it needs (above the 64 KiB default).
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <int W, int PREC, bool GEN, bool STAGE>
hipError_t row_launch(bool force, bool energy, const RowLaunch &L, const SweepBuffers &B, const ForceOut &fo,
                      const RowDriftArgs &da, const PotConst &pc, hipStream_t s) {
    const RowArgs ra{L.tiles, L.order, L.cd, L.uni_off, L.uni_n, L.uni_ni};
    hipError_t e;
    if (force) {
        const size_t lds = row_lds_bytes<W, 4, STAGE>(L.nmax);
        // the generic-exponent kernels always accumulate the energy
        // the bath epilogue exists only in fused (staged) launches
        constexpr bool kB = STAGE;
        auto kern = (energy || GEN)
                        ? (fo.bath ? k_row_force<W, PREC, GEN, STAGE, true, kB> : k_row_force<W, PREC, GEN, STAGE, true, false>)
                        : (fo.bath ? k_row_force<W, PREC, GEN, STAGE, GEN, kB> : k_row_force<W, PREC, GEN, STAGE, GEN, false>);
        if ((e = allow_lds(kern, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(L.ntiles), dim3(64 * W), lds, s, ra, (const double4 *)B.xp, fo, pc);
    } else {
        const size_t lds = row_lds_bytes<W, 1, STAGE>(L.nmax);
        auto kern = k_row_density<W, PREC, GEN, STAGE>;
        if ((e = allow_lds(kern, lds)) != hipSuccess) return e;
        const DensityOut dout{B.rp, B.xp, B.rho, B.tile_sums};
        hipLaunchKernelGGL(kern, dim3(L.ntiles), dim3(64 * W), lds, s, ra, dout, pc, da);
    }
    return hipGetLastError();
}

template <int W, bool STAGE>
hipError_t row_dispatch_ws(bool force, bool energy, const RowLaunch &L, const SweepBuffers &B, const ForceOut &fo,
                           const RowDriftArgs &da, const PotConst &pc, int precision, hipStream_t s) {
    if (pc.generic) {
        return precision == SCMD_MIXED ? row_launch<W, SCMD_MIXED, true, STAGE>(force, energy, L, B, fo, da, pc, s)
                                       : row_launch<W, SCMD_FP64, true, STAGE>(force, energy, L, B, fo, da, pc, s);
    }
    return precision == SCMD_MIXED ? row_launch<W, SCMD_MIXED, false, STAGE>(force, energy, L, B, fo, da, pc, s)
                                   : row_launch<W, SCMD_FP64, false, STAGE>(force, energy, L, B, fo, da, pc, s);
}

template <int W>
hipError_t row_dispatch_w(bool force, bool energy, const RowLaunch &L, const SweepBuffers &B, const ForceOut &fo,
                          const RowDriftArgs &da, const PotConst &pc, int precision, hipStream_t s) {
    return L.nmax <= kRowStageMax ? row_dispatch_ws<W, true>(force, energy, L, B, fo, da, pc, precision, s)
                                  : row_dispatch_ws<W, false>(force, energy, L, B, fo, da, pc, precision, s);
}

hipError_t row_dispatch(bool force, bool energy, const RowLaunch &L, const SweepBuffers &B, const ForceOut &fo,
                        const RowDriftArgs &da, const PotConst &pc, int precision, hipStream_t s) {
    if (L.ntiles <= 0) return hipSuccess;
    // the drift and the fused epilogue need staged clusters
    if ((da.mode != 0 || fo.fused) && L.nmax > kRowStageMax) return hipErrorInvalidValue;
    (void)hipGetLastError();
    switch (L.waves) {
        case 4: return row_dispatch_w<4>(force, energy, L, B, fo, da, pc, precision, s);
        case 8: return row_dispatch_w<8>(force, energy, L, B, fo, da, pc, precision, s);
        case 16: return row_dispatch_w<16>(force, energy, L, B, fo, da, pc, precision, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_row_density(const RowLaunch &L, const SweepBuffers &B, const StepArgs &a, const RowDrift &dr,
                              const PotConst &pc, int precision, hipStream_t s) {
    const ForceOut fo{};
    const RowDriftArgs da{dr.mode, dr.local, dr.bath, B.v, B.f, B.dpv, a.st, B.tile_sums, a.cd, a.mass_u, a.dt, a.h,
                          a.dt * a.h};
    return row_dispatch(false, true, L, B, fo, da, pc, precision, s);
}

hipError_t launch_row_force(const RowLaunch &L, const SweepBuffers &B, const StepArgs &a, int fused, int local,
                            int bath, const PotConst &pc, int precision, hipStream_t s) {
    // the fused epilogue stores the drifted positions (rp is the context's
    // writable position array; the sweeps otherwise only read it)
    const ForceOut fo{B.f,  B.v,       B.tile_sums, a.h,  a.advance, fused,    a.st,  const_cast<double4 *>(B.rp),
                      B.dpv, a.dt * a.h, a.cd,       local, a.dt,      a.mass_u, bath};
    const RowDriftArgs da{};
    return row_dispatch(true, a.energy != 0, L, B, fo, da, pc, precision, s);
}

}  // namespace scmd
