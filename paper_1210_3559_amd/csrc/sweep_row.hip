// Row sweeps for small clusters: one workgroup holds every partner of a
// short run of atoms, so that a sweep finishes in one launch with no partial
// slots and no reduce kernel.
//
// The two sweeps are those of the paper's scheme (Sec. 2 "Computational
// approach": the density sums of Eq. (rho), then the forces of Eq. (SC)),
// evaluated one-sidedly: every atom accumulates its own sums.  A workgroup
// of 64*W threads owns atoms [i0, i0 + ni) of one cluster, ni <= 64.
// Thread t works for atom il = t % ni on partner stream s = t / ni; the S =
// floor(64 W / ni) streams of an atom interleave over the cluster (stream s
// visits j = off + s, off + s + S, ...), so almost every thread is busy for
// any ni and consecutive threads load neighbouring partners.  The partner
// window [i0, i0 + ni), which holds the self pairs, and the last, partly
// filled round of each wavefront are the only masked iterations.  Stream
// sums are combined in LDS in a fixed order (deterministic), and the
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
    int ni, S, il, s, i;
    bool active;
    int k_mask0, k_mask1;  // rounds [k_mask0, k_mask1) may meet the self window
    int k_full, k_end;     // rounds [0, k_full) are full for the whole wavefront; k_end: last round + 1
};

template <int W>
__device__ __forceinline__ RowLayout row_layout(const ITile &t, int off, int n) {
    RowLayout L;
    L.ni = t.ni;
    L.S = (64 * W) / L.ni;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    L.active = tid < L.ni * L.S;
    // idle threads shadow the last stream (valid addresses, results dropped)
    const int tt = L.active ? tid : L.ni * L.S - 1;
    L.il = tt % L.ni;
    L.s = tt / L.ni;
    L.i = t.i0 + L.il;
    // stream range of this wavefront (wave-uniform)
    const int t_lo = wave * 64;
    const int t_hi = min(wave * 64 + 63, L.ni * L.S - 1);
    const int s_min = min(t_lo, L.ni * L.S - 1) / L.ni;
    const int s_max = t_hi / L.ni;
    // rounds in which some thread of the wavefront meets j in [i0, i0 + ni)
    const int w0 = t.i0 - off, w1 = t.i0 + L.ni - 1 - off;
    const int klo = max(0, floor_div(w0 - s_max + L.S - 1, L.S));
    const int khi = floor_div(w1 - s_min, L.S);  // inclusive
    // rounds: thread with stream s has ceil((n - s) / S) of them
    L.k_full = n > s_max ? (n - s_max + L.S - 1) / L.S : 0;
    L.k_end = n > s_min ? (n - s_min + L.S - 1) / L.S : 0;
    L.k_mask0 = min(klo, L.k_full);
    L.k_mask1 = max(L.k_mask0, min(khi + 1, L.k_full));
    return L;
}

// Fixed-order sum over the streams of each atom: level 1 adds runs of C
// consecutive streams, level 2 adds the runs.  sh holds 64*W doubles per
// value; v[q] are this thread's partial sums.  Returns the totals to threads
// il < ni (others get 0).
template <int W, int Q>
__device__ __forceinline__ void row_reduce(const RowLayout &L, double (&v)[Q], double *sh) {
    constexpr int T = 64 * W;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < Q; ++q) sh[q * T + tid] = L.active ? v[q] : 0.0;
    __syncthreads();
    // level 1: G1 runs of C streams per atom
    int C = 1;
    while (C * C < L.S) ++C;
    const int G1 = (L.S + C - 1) / C;
    double p[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) p[q] = 0.0;
    const bool lvl1 = tid < L.ni * G1;
    if (lvl1) {
        const int il = tid % L.ni, g = tid / L.ni;
        const int s0 = g * C, s1 = min(L.S, s0 + C);
        for (int s = s0; s < s1; ++s) {
#pragma unroll
            for (int q = 0; q < Q; ++q) p[q] += sh[q * T + il + L.ni * s];
        }
    }
    __syncthreads();
    if (lvl1) {
#pragma unroll
        for (int q = 0; q < Q; ++q) sh[q * T + tid] = p[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = 0.0;
    if (tid < L.ni) {
        for (int g = 0; g < G1; ++g) {
#pragma unroll
            for (int q = 0; q < Q; ++q) v[q] += sh[q * T + tid + L.ni * g];
        }
    }
}

// Wavefront sum (fixed butterfly, deterministic) of lanes 0..63.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// ---------------------------------------------------------------------------
// Density sweep
// ---------------------------------------------------------------------------
template <int W, int PREC, bool GEN>
__global__ __launch_bounds__(64 * W) void k_row_density(const ITile *__restrict__ tiles,
                                                        const int32_t *__restrict__ order,
                                                        const ClusterDesc *__restrict__ cd, DensityOut o,
                                                        PotConst pc) {
    __shared__ double sh[64 * W];
    const int tix = order[blockIdx.x];
    const ITile t = tiles[tix];
    const ClusterDesc d = cd[t.c];
    const RowLayout L = row_layout<W>(t, d.off, d.n);
    const double4 qi = o.rp[L.i];
    const double4 *__restrict__ rp = o.rp;
    double acc = 0.0;
    const int S = L.S;
    const int j0 = d.off + L.s;
    int k = 0;
    // partner rounds without masks; four pointers stepped by 4 S (one
    // 64-bit add per load)
    auto plain = [&](int k1) {
        if (k >= k1) return;
        const double4 *p0 = rp + (j0 + (size_t)k * S);
        const double4 *p1 = p0 + S, *p2 = p1 + S, *p3 = p2 + S;
        const size_t S4 = 4 * (size_t)S;
        for (; k + 4 <= k1; k += 4, p0 += S4, p1 += S4, p2 += S4, p3 += S4) {
            const double4 a = *p0, b = *p1, c = *p2, e = *p3;
            density_pair<PREC, GEN, false, false>(qi.x - a.x, qi.y - a.y, qi.z - a.z, false, acc, pc);
            density_pair<PREC, GEN, false, false>(qi.x - b.x, qi.y - b.y, qi.z - b.z, false, acc, pc);
            density_pair<PREC, GEN, false, false>(qi.x - c.x, qi.y - c.y, qi.z - c.z, false, acc, pc);
            density_pair<PREC, GEN, false, false>(qi.x - e.x, qi.y - e.y, qi.z - e.z, false, acc, pc);
        }
        for (; k < k1; ++k, p0 += S) {
            const double4 a = *p0;
            density_pair<PREC, GEN, false, false>(qi.x - a.x, qi.y - a.y, qi.z - a.z, false, acc, pc);
        }
    };
    auto masked = [&](int k1) {
        const int end = d.off + d.n;
        for (int j = j0 + k * S; k < k1; ++k, j += S) {
            const bool valid = j < end;
            const double4 a = rp[valid ? j : d.off];
            density_pair<PREC, GEN, true, false>(qi.x - a.x, qi.y - a.y, qi.z - a.z, !valid || j == L.i, acc, pc);
        }
    };
    plain(L.k_mask0);
    masked(L.k_mask1);
    plain(L.k_full);
    masked(L.k_end);

    double v[1] = {acc};
    row_reduce<W, 1>(L, v, sh);
    double emb = 0.0;
    if (threadIdx.x < L.ni) emb = density_atom(t.i0 + threadIdx.x, v[0], o, pc);
    if (threadIdx.x < 64) {
        emb = wave_sum(emb);
        if (threadIdx.x == 0) o.tile_sums[(size_t)tix * kTileSums + 0] = emb;
    }
}

// ---------------------------------------------------------------------------
// Force sweep
// ---------------------------------------------------------------------------
template <int W, int PREC, bool GEN>
__global__ __launch_bounds__(64 * W) void k_row_force(const ITile *__restrict__ tiles,
                                                      const int32_t *__restrict__ order,
                                                      const ClusterDesc *__restrict__ cd, const double4 *__restrict__ xp,
                                                      ForceOut o, PotConst pc) {
    __shared__ double sh[4 * 64 * W];
    const int tix = order[blockIdx.x];
    const ITile t = tiles[tix];
    const ClusterDesc d = cd[t.c];
    const RowLayout L = row_layout<W>(t, d.off, d.n);
    const double4 qi = xp[L.i];
    const double ci = -qi.w;
    const float cif = (float)ci;
    const float Af = (float)pc.A;
    double fx = 0.0, fy = 0.0, fz = 0.0, eu = 0.0;
    const int S = L.S;
    const int j0 = d.off + L.s;
    int k = 0;
    auto plain = [&](int k1) {
        if (k >= k1) return;
        const double4 *p0 = xp + (j0 + (size_t)k * S);
        const double4 *p1 = p0 + S, *p2 = p1 + S, *p3 = p2 + S;
        const size_t S4 = 4 * (size_t)S;
        for (; k + 4 <= k1; k += 4, p0 += S4, p1 += S4, p2 += S4, p3 += S4) {
            const double4 a = *p0, b = *p1, c = *p2, e = *p3;
            force_pair<PREC, GEN, false, false>(qi.x - a.x, qi.y - a.y, qi.z - a.z, false, ci, a.w, cif, (float)a.w,
                                                fx, fy, fz, eu, pc, Af);
            force_pair<PREC, GEN, false, false>(qi.x - b.x, qi.y - b.y, qi.z - b.z, false, ci, b.w, cif, (float)b.w,
                                                fx, fy, fz, eu, pc, Af);
            force_pair<PREC, GEN, false, false>(qi.x - c.x, qi.y - c.y, qi.z - c.z, false, ci, c.w, cif, (float)c.w,
                                                fx, fy, fz, eu, pc, Af);
            force_pair<PREC, GEN, false, false>(qi.x - e.x, qi.y - e.y, qi.z - e.z, false, ci, e.w, cif, (float)e.w,
                                                fx, fy, fz, eu, pc, Af);
        }
        for (; k < k1; ++k, p0 += S) {
            const double4 a = *p0;
            force_pair<PREC, GEN, false, false>(qi.x - a.x, qi.y - a.y, qi.z - a.z, false, ci, a.w, cif, (float)a.w,
                                                fx, fy, fz, eu, pc, Af);
        }
    };
    auto masked = [&](int k1) {
        const int end = d.off + d.n;
        for (int j = j0 + k * S; k < k1; ++k, j += S) {
            const bool valid = j < end;
            const double4 a = xp[valid ? j : d.off];
            force_pair<PREC, GEN, true, false>(qi.x - a.x, qi.y - a.y, qi.z - a.z, !valid || j == L.i, ci, a.w, cif,
                                               (float)a.w, fx, fy, fz, eu, pc, Af);
        }
    };
    plain(L.k_mask0);
    masked(L.k_mask1);
    plain(L.k_full);
    masked(L.k_end);

    unscale_force<PREC, GEN>(fx, fy, fz, eu);
    double v[4] = {fx, fy, fz, eu};
    row_reduce<W, 4>(L, v, sh);
    double epair = 0.0, v2 = 0.0;
    if (threadIdx.x < L.ni) force_atom(t.i0 + threadIdx.x, v[0], v[1], v[2], v[3], o, pc, epair, v2);
    if (threadIdx.x < 64) {
        epair = wave_sum(epair);
        v2 = wave_sum(v2);
        if (threadIdx.x == 0) {
            o.tile_sums[(size_t)tix * kTileSums + 1] = epair;
            o.tile_sums[(size_t)tix * kTileSums + 2] = v2;
        }
    }
}

template <int W, int PREC, bool GEN>
hipError_t row_launch(bool force, const RowLaunch &L, const SweepBuffers &B, const ForceOut &fo, const PotConst &pc,
                      hipStream_t s) {
    if (force) {
        hipLaunchKernelGGL((k_row_force<W, PREC, GEN>), dim3(L.ntiles), dim3(64 * W), 0, s, L.tiles, L.order, L.cd,
                           (const double4 *)B.xp, fo, pc);
    } else {
        const DensityOut dout{B.rp, B.xp, B.rho, B.tile_sums};
        hipLaunchKernelGGL((k_row_density<W, PREC, GEN>), dim3(L.ntiles), dim3(64 * W), 0, s, L.tiles, L.order, L.cd,
                           dout, pc);
    }
    return hipGetLastError();
}

template <int W>
hipError_t row_dispatch_w(bool force, const RowLaunch &L, const SweepBuffers &B, const ForceOut &fo,
                          const PotConst &pc, int precision, hipStream_t s) {
    if (pc.generic) {
        return precision == SCMD_MIXED ? row_launch<W, SCMD_MIXED, true>(force, L, B, fo, pc, s)
                                       : row_launch<W, SCMD_FP64, true>(force, L, B, fo, pc, s);
    }
    return precision == SCMD_MIXED ? row_launch<W, SCMD_MIXED, false>(force, L, B, fo, pc, s)
                                   : row_launch<W, SCMD_FP64, false>(force, L, B, fo, pc, s);
}

hipError_t row_dispatch(bool force, const RowLaunch &L, const SweepBuffers &B, const ForceOut &fo,
                        const PotConst &pc, int precision, hipStream_t s) {
    if (L.ntiles <= 0) return hipSuccess;
    (void)hipGetLastError();
    switch (L.waves) {
        case 4: return row_dispatch_w<4>(force, L, B, fo, pc, precision, s);
        case 8: return row_dispatch_w<8>(force, L, B, fo, pc, precision, s);
        case 16: return row_dispatch_w<16>(force, L, B, fo, pc, precision, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_row_density(const RowLaunch &L, const SweepBuffers &B, const PotConst &pc, int precision,
                              hipStream_t s) {
    const ForceOut fo{};
    return row_dispatch(false, L, B, fo, pc, precision, s);
}

hipError_t launch_row_force(const RowLaunch &L, const SweepBuffers &B, const StepArgs &a, const PotConst &pc,
                            int precision, hipStream_t s) {
    const ForceOut fo{B.f, B.v, B.tile_sums, a.h, a.advance};
    return row_dispatch(true, L, B, fo, pc, precision, s);
}

}  // namespace scmd
