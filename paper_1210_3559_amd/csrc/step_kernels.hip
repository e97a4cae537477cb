// Integration, reduction and bookkeeping kernels of one velocity-Verlet step.
//
// Step layout on the device (one launch each, captured into a HIP graph):
//   drift          v <- lambda v + (dt/2m) F;  r <- r + dt v      (per atom)
//   density sweep  partial sums of u^m                           (sweep kernels)
//   density reduce rho = a^m sum partials, psi = rho^-1/2, P = Pscale psi,
//                  embedding energy per tile                     (per tile)
//   force sweep    partial sums of force and u^n                 (sweep kernels)
//   force reduce   F = sum partials, v <- v + (dt/2m) F, pair energy and
//                  v^2 per tile                                  (per tile)
//   finalize       per cluster: E_pot, E_kin, T, Berendsen lambda (per cluster)
// Integration follows velocity-Verlet (the paper's Verlet step, Sec. 2
// "Computational approach"); the thermostat factor of step k is applied at
// the start of step k+1, which gives the same arithmetic as scaling at the
// end of step k.
//
// Every reduction is a fixed-order sum (partials by slot index, tiles by
// index, a fixed tree inside a workgroup), so a run is bitwise reproducible.
#include "scmd_internal.h"
#include "../../include/scmd.h"

namespace scmd {
namespace {

constexpr int kReduceBlock = 256;

// Fixed-shape tree sum over a 256-thread workgroup (deterministic).
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = kReduceBlock / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_drift(const int32_t *__restrict__ atom_cluster,
                                               const ClusterState *__restrict__ st, double4 *__restrict__ rp,
                                               double4 *__restrict__ v, const double4 *__restrict__ f, int natoms,
                                               double dt, double h) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natoms) return;
    const double lam = st[atom_cluster[i]].lambda;
    double4 vi = v[i];
    const double4 fi = f[i];
    double4 ri = rp[i];
    vi.x = lam * vi.x;
    vi.y = lam * vi.y;
    vi.z = lam * vi.z;
    vi.x = vi.x + h * fi.x;
    vi.y = vi.y + h * fi.y;
    vi.z = vi.z + h * fi.z;
    ri.x = ri.x + dt * vi.x;
    ri.y = ri.y + dt * vi.y;
    ri.z = ri.z + dt * vi.z;
    v[i] = vi;
    rp[i] = ri;
}

// One workgroup per atom tile; thread t handles tile atoms t, t+256, ...
__global__ __launch_bounds__(kReduceBlock) void k_density_reduce(const ITile *__restrict__ tiles, int tile,
                                                                 const double *__restrict__ part,
                                                                 double4 *__restrict__ rp, double *__restrict__ rho,
                                                                 double *__restrict__ tile_sums, PotConst pc) {
    __shared__ double sh[kReduceBlock];
    const ITile T = tiles[blockIdx.x];
    double emb = 0.0;
    for (int li = threadIdx.x; li < T.ni; li += kReduceBlock) {
        double s = 0.0;
        for (int k = 0; k < T.nsplit; ++k) s += part[(size_t)(T.first + k) * tile + li];
        const double r = pc.am * s;
        const int i = T.i0 + li;
        const double sq = sqrt(r);
        const double psi = r > 0.0 ? 1.0 / sq : 0.0;
        rho[i] = r;
        rp[i].w = pc.Pscale * psi;
        emb -= pc.eps_c * sq;
    }
    emb = block_sum(emb, sh);
    if (threadIdx.x == 0) tile_sums[(size_t)blockIdx.x * kTileSums + 0] = emb;
}

__global__ __launch_bounds__(kReduceBlock) void k_force_reduce(const ITile *__restrict__ tiles, int tile,
                                                               const double *__restrict__ part,
                                                               double4 *__restrict__ f, double4 *__restrict__ v,
                                                               double *__restrict__ tile_sums, PotConst pc, double h,
                                                               int kick) {
#pragma clang fp contract(off)
    __shared__ double sh[kReduceBlock];
    const ITile T = tiles[blockIdx.x];
    double epair = 0.0, v2 = 0.0;
    for (int li = threadIdx.x; li < T.ni; li += kReduceBlock) {
        double fx = 0.0, fy = 0.0, fz = 0.0, eu = 0.0;
        for (int k = 0; k < T.nsplit; ++k) {
            const double *p = part + (size_t)(T.first + k) * 4 * tile + li;
            fx += p[0];
            fy += p[tile];
            fz += p[2 * tile];
            eu += p[3 * tile];
        }
        const int i = T.i0 + li;
        const double ei = pc.half_eps_an * eu;
        f[i] = make_double4(fx, fy, fz, ei);
        double4 vi = v[i];
        if (kick) {
            vi.x = vi.x + h * fx;
            vi.y = vi.y + h * fy;
            vi.z = vi.z + h * fz;
            v[i] = vi;
        }
        epair += ei;
        v2 += vi.x * vi.x + vi.y * vi.y + vi.z * vi.z;
    }
    epair = block_sum(epair, sh);
    v2 = block_sum(v2, sh);
    if (threadIdx.x == 0) {
        tile_sums[(size_t)blockIdx.x * kTileSums + 1] = epair;
        tile_sums[(size_t)blockIdx.x * kTileSums + 2] = v2;
    }
}

// One thread per cluster: fixed-order sums over the cluster's tiles, then the
// thermostat.  advance = 1 after a step (step count and lambda are updated),
// 0 for a plain evaluation (the pending lambda is kept).
__global__ __launch_bounds__(64) void k_finalize(const ClusterDesc *__restrict__ cd, ClusterState *__restrict__ st,
                                                 int nclusters, const double *__restrict__ tile_sums, double mass_u,
                                                 double dt, int advance, int *__restrict__ flag) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nclusters) return;
    const ClusterDesc d = cd[c];
    ClusterState s = st[c];
    double emb = 0.0, epair = 0.0, v2 = 0.0;
    for (int t = 0; t < d.ntiles; ++t) {
        const double *ts = tile_sums + (size_t)(d.tile0 + t) * kTileSums;
        emb += ts[0];
        epair += ts[1];
        v2 += ts[2];
    }
    const double ke = 0.5 * mass_u * v2 * kEvPerUA2Fs2;
    const double T = d.ndof > 0 ? 2.0 * ke / ((double)d.ndof * kBoltzmannEv) : 0.0;
    double lam = s.lambda;
    if (advance) {
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
                const double x = 1.0 + (dt / d.tau) * (tt / T - 1.0);
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
        atomicOr(flag, 1);
    }
    st[c] = s;
}

__global__ __launch_bounds__(256) void k_aos_from4(const double4 *__restrict__ src, double *__restrict__ dst,
                                                   int natoms) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natoms) return;
    const double4 q = src[i];
    dst[3 * (size_t)i + 0] = q.x;
    dst[3 * (size_t)i + 1] = q.y;
    dst[3 * (size_t)i + 2] = q.z;
}

}  // namespace

hipError_t launch_drift(const int32_t *atom_cluster, const ClusterState *st, double4 *rp, double4 *v,
                        const double4 *f, int natoms, double dt, double h, hipStream_t s) {
    if (natoms <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_drift, dim3((natoms + 255) / 256), dim3(256), 0, s, atom_cluster, st, rp, v, f, natoms,
                       dt, h);
    return hipGetLastError();
}

hipError_t launch_density_reduce(const ITile *tiles, int ntiles, int tile, const double *part, double4 *rp,
                                 double *rho, double *tile_sums, const PotConst &pc, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_density_reduce, dim3(ntiles), dim3(kReduceBlock), 0, s, tiles, tile, part, rp, rho,
                       tile_sums, pc);
    return hipGetLastError();
}

hipError_t launch_force_reduce(const ITile *tiles, int ntiles, int tile, const double *part, double4 *f, double4 *v,
                               double *tile_sums, const PotConst &pc, double h, int kick, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_force_reduce, dim3(ntiles), dim3(kReduceBlock), 0, s, tiles, tile, part, f, v, tile_sums,
                       pc, h, kick);
    return hipGetLastError();
}

hipError_t launch_finalize(const ClusterDesc *cd, ClusterState *st, int nclusters, const double *tile_sums,
                           double mass_u, double dt, int advance, int *flag, hipStream_t s) {
    if (nclusters <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3((nclusters + 63) / 64), dim3(64), 0, s, cd, st, nclusters, tile_sums, mass_u,
                       dt, advance, flag);
    return hipGetLastError();
}

hipError_t launch_aos_from4(const double4 *src, double *dst, int natoms, hipStream_t s) {
    if (natoms <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_aos_from4, dim3((natoms + 255) / 256), dim3(256), 0, s, src, dst, natoms);
    return hipGetLastError();
}

}  // namespace scmd
