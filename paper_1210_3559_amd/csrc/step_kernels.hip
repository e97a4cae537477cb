// Per-atom kernels of one velocity-Verlet step.
//
// Step layout on the device (captured into a HIP graph):
//   drift          v <- lambda v + (dt/2m) F;  r <- r + dt v      (this file)
//                  (Langevin bath: r, v <- A, O, A of bath.h)
//   density sweep  rho, psi, embedding energy                    (sweep kernels)
//   force sweep    F, second half-kick, energies, thermostat     (sweep kernels)
// Integration follows velocity-Verlet (the paper's Verlet step, Sec. 2
// "Computational approach"); the thermostat factor of step k is applied at
// the start of step k+1, which gives the same arithmetic as scaling the
// velocities at the end of step k.
#include "sweep_common.h"

namespace scmd {
namespace {

// First half-kick (after the pending thermostat factor) and the move of one
// atom: r + dt v, or the bath's A, O, A of step `step` (atom index a in its
// cluster).
__device__ __forceinline__ void drift_atom(const ClusterDesc &d, int64_t step, int a, double lam, double mass_u,
                                           double dt, double h, double4 &ri, double4 &vi, const double4 &fi) {
#pragma clang fp contract(off)
    vi.x = lam * vi.x;
    vi.y = lam * vi.y;
    vi.z = lam * vi.z;
    vi.x = vi.x + h * fi.x;
    vi.y = vi.y + h * fi.y;
    vi.z = vi.z + h * fi.z;
    if (d.kind == SCMD_LANGEVIN) {
        dev::bath_drift(d, step, a, mass_u, dt, ri, vi);
    } else {
        ri.x = ri.x + dt * vi.x;
        ri.y = ri.y + dt * vi.y;
        ri.z = ri.z + dt * vi.z;
    }
}

__global__ __launch_bounds__(256) void k_drift(const int32_t *__restrict__ atom_cluster,
                                               const ClusterDesc *__restrict__ cd,
                                               const ClusterState *__restrict__ st, double4 *__restrict__ rp,
                                               double4 *__restrict__ v, const double4 *__restrict__ f, int natoms,
                                               double mass_u, double dt, double h, int local) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natoms) return;
    const int c = atom_cluster[i];
    const ClusterState &sc = st[c];
    const ClusterDesc &d = cd[c];
    double4 vi = v[i];
    const double4 fi = f[i];
    double4 ri = rp[i];
    drift_atom(d, sc.step + local + 1, i - d.off, sc.lambda, mass_u, dt, h, ri, vi, fi);
    v[i] = vi;
    rp[i] = ri;
}

// Atoms of clusters in a Langevin bath, before the first step of a run on
// the fused row path: the drifted (r, v) of that step, stored as the pairs
// (x, y), (z, vx), (vy, vz) that the row density sweep reads.
__global__ __launch_bounds__(256) void k_bath_prep(const int32_t *__restrict__ atom_cluster,
                                                   const ClusterDesc *__restrict__ cd,
                                                   const ClusterState *__restrict__ st,
                                                   const double4 *__restrict__ rp, const double4 *__restrict__ v,
                                                   const double4 *__restrict__ f, double2 *__restrict__ dpv,
                                                   int natoms, double mass_u, double dt, double h) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natoms) return;
    const int c = atom_cluster[i];
    const ClusterDesc &d = cd[c];
    if (d.kind != SCMD_LANGEVIN) return;
    double4 vi = v[i];
    const double4 fi = f[i];
    double4 ri = rp[i];
    drift_atom(d, st[c].step + 1, i - d.off, st[c].lambda, mass_u, dt, h, ri, vi, fi);
    double2 *o = dpv + 3 * (size_t)i;
    o[0] = make_double2(ri.x, ri.y);
    o[1] = make_double2(ri.z, vi.x);
    o[2] = make_double2(vi.y, vi.z);
}

// Drift fused with the finish of the previous step of a single cluster:
// every workgroup reduces the cluster's tile sums itself (same order, so the
// same thermostat factor in every workgroup) and workgroup 0 stores the
// cluster state, which saves a launch per step.  CELL: the cell list's
// check on the drifted positions as well (another launch saved).
template <bool CELL>
__global__ __launch_bounds__(256) void k_drift_fin(dev::FinalizeArgs fa, double4 *__restrict__ rp,
                                                   double4 *__restrict__ v, const double4 *__restrict__ f,
                                                   int natoms, double dt, double h, CellCheck cc) {
    __shared__ double sh[12];
    __shared__ double sh_box[6 * (256 / 64)];
    __shared__ double lam_sh;
    const double l0 = dev::cluster_finalize(0, fa, sh, blockIdx.x == 0);
    if (threadIdx.x == 0) lam_sh = l0;
    __syncthreads();
    const double lam = lam_sh;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    dev::CellBox b;
    if (i < natoms) {
        const ClusterDesc &d = fa.cd[0];
        double4 vi = v[i];
        const double4 fi = f[i];
        double4 ri = rp[i];
        // this drift starts step fa.step_add + 1 of the run
        drift_atom(d, fa.st[0].step + fa.step_add + 1, i - d.off, lam, fa.mass_u, dt, h, ri, vi, fi);
        v[i] = vi;
        rp[i] = ri;
        if constexpr (CELL) dev::cell_check_atom(cc, i, ri, b);
    }
    if constexpr (CELL) dev::cell_check_merge<256>(cc, 0, b, sh_box);
}

__global__ __launch_bounds__(256) void k_sample(const ClusterState *__restrict__ st, int nclusters,
                                                double *__restrict__ ring, int slot, double step) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nclusters) return;
    const ClusterState s = st[c];
    double *o = ring + ((size_t)slot * nclusters + c) * 5;
    o[0] = step;
    o[1] = s.epot;
    o[2] = s.ekin;
    o[3] = s.temp;
    o[4] = s.ttarget;
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

hipError_t launch_drift(const int32_t *atom_cluster, const ClusterDesc *cd, const ClusterState *st, double4 *rp,
                        double4 *v, const double4 *f, int natoms, double mass_u, double dt, double h, int local,
                        hipStream_t s) {
    if (natoms <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_drift, dim3((natoms + 255) / 256), dim3(256), 0, s, atom_cluster, cd, st, rp, v, f, natoms,
                       mass_u, dt, h, local);
    return hipGetLastError();
}

hipError_t launch_bath_prep(const StepArgs &a, const int32_t *atom_cluster, const double4 *rp, const double4 *v,
                            const double4 *f, double2 *dpv, int natoms, hipStream_t s) {
    if (natoms <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_bath_prep, dim3((natoms + 255) / 256), dim3(256), 0, s, atom_cluster, a.cd, a.st, rp, v, f,
                       dpv, natoms, a.mass_u, a.dt, a.h);
    return hipGetLastError();
}

hipError_t launch_drift_fin(const StepArgs &a, const double *tile_sums, int local, double4 *rp, double4 *v,
                            const double4 *f, int natoms, const CellCheck *cc, hipStream_t s) {
    if (natoms <= 0) return hipSuccess;
    const dev::FinalizeArgs fa{a.cd, a.st, tile_sums, a.flag, a.mass_u, a.dt, 1, local, 0};
    (void)hipGetLastError();
    if (cc)
        hipLaunchKernelGGL(k_drift_fin<true>, dim3((natoms + 255) / 256), dim3(256), 0, s, fa, rp, v, f, natoms, a.dt,
                           a.h, *cc);
    else
        hipLaunchKernelGGL(k_drift_fin<false>, dim3((natoms + 255) / 256), dim3(256), 0, s, fa, rp, v, f, natoms,
                           a.dt, a.h, CellCheck{});
    return hipGetLastError();
}

hipError_t launch_sample(const ClusterState *st, int nclusters, double *ring, int slot, int64_t step, hipStream_t s) {
    if (nclusters <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_sample, dim3((nclusters + 255) / 256), dim3(256), 0, s, st, nclusters, ring, slot,
                       (double)step);
    return hipGetLastError();
}

hipError_t launch_aos_from4(const double4 *src, double *dst, int natoms, hipStream_t s) {
    if (natoms <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_aos_from4, dim3((natoms + 255) / 256), dim3(256), 0, s, src, dst, natoms);
    return hipGetLastError();
}

}  // namespace scmd
