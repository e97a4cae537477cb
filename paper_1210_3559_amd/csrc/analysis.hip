// On-device analysis of a cluster's current positions.
//
// Pair-distance histogram of the radial distribution function g(r) =
// rho(r) / rho_bar (Sec. 3, "Radial distribution function as an indicator of
// the phase transition", Eq. (Rdist)): reference atoms are those closer than
// r_select to the cluster's centre of mass (every atom when r_select <= 0);
// each (reference, other atom) pair is counted in bin floor(r / dr), with
// r = sqrt(dx*dx + dy*dy + dz*dz) evaluated in that order without
// contraction, so that the bin decision is the one of any IEEE double
// evaluation of the same expression.  Counts are integers added with atomics
// (order-independent), so the histogram is exact.
#include "scmd_internal.h"

namespace scmd {
namespace {

constexpr int kSelBlock = 256;

// One workgroup: centre of mass (fixed-order sums), then the indices of the
// reference atoms in increasing order (compaction by wavefront ballots).
__global__ __launch_bounds__(kSelBlock) void k_rdf_select(const double4 *__restrict__ rp, int off, int n,
                                                         double r_select, int32_t *__restrict__ refs,
                                                         int *__restrict__ nref) {
#pragma clang fp contract(off)
    __shared__ double sh[3 * (kSelBlock / 64)];
    __shared__ int wave_cnt[kSelBlock / 64];
    __shared__ int base_sh;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int i = t; i < n; i += kSelBlock) {
        const double4 q = rp[off + i];
        sx += q.x;
        sy += q.y;
        sz += q.z;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
        sz += __shfl_xor(sz, o, 64);
    }
    if (lane == 0) {
        sh[3 * w] = sx;
        sh[3 * w + 1] = sy;
        sh[3 * w + 2] = sz;
    }
    if (t == 0) base_sh = 0;
    __syncthreads();
    const double inv = n > 0 ? 1.0 / (double)n : 0.0;
    const double cx = ((sh[0] + sh[3]) + (sh[6] + sh[9])) * inv;
    const double cy = ((sh[1] + sh[4]) + (sh[7] + sh[10])) * inv;
    const double cz = ((sh[2] + sh[5]) + (sh[8] + sh[11])) * inv;
    const double rs2 = r_select * r_select;
    for (int i0 = 0; i0 < n; i0 += kSelBlock) {
        const int i = i0 + t;
        bool sel = false;
        if (i < n) {
            const double4 q = rp[off + i];
            const double ex = q.x - cx, ey = q.y - cy, ez = q.z - cz;
            sel = !(r_select > 0.0) || (ex * ex + ey * ey + ez * ez < rs2);
        }
        const unsigned long long m = __ballot(sel);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wave_cnt[w] = __popcll(m);
        __syncthreads();
        int wbase = base_sh;
        for (int k = 0; k < w; ++k) wbase += wave_cnt[k];
        if (sel) refs[wbase + before] = i;
        __syncthreads();
        if (t == 0) base_sh += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
        __syncthreads();
    }
    if (t == 0) *nref = base_sh;
}

constexpr int kHistBlock = 256;
constexpr int kRefsPerBlock = 8;

// Workgroup b takes reference atoms [8b, 8b + 8) against every atom of the
// cluster; counts go to a workgroup histogram in LDS, then to the device
// histogram with 64-bit atomics (nonzero bins only).
__global__ __launch_bounds__(kHistBlock) void k_rdf_hist(const double4 *__restrict__ rp, int off, int n,
                                                        const int32_t *__restrict__ refs,
                                                        const int *__restrict__ nref, double dr, int nbins,
                                                        unsigned long long *__restrict__ counts) {
#pragma clang fp contract(off)
    extern __shared__ unsigned int hist[];
    const int t = threadIdx.x;
    const int nr = *nref;
    const int r0 = blockIdx.x * kRefsPerBlock;
    if (r0 >= nr) return;  // uniform per workgroup
    for (int b = t; b < nbins; b += kHistBlock) hist[b] = 0u;
    __syncthreads();
    const int r1 = min(nr, r0 + kRefsPerBlock);
    for (int r = r0; r < r1; ++r) {
        const int i = refs[r];
        const double4 qi = rp[off + i];
        for (int j = t; j < n; j += kHistBlock) {
            if (j == i) continue;
            const double4 qj = rp[off + j];
            const double dx = qi.x - qj.x, dy = qi.y - qj.y, dz = qi.z - qj.z;
            const double d = sqrt(dx * dx + dy * dy + dz * dz);
            const double b = floor(d / dr);
            if (b < (double)nbins) atomicAdd(&hist[(int)b], 1u);
        }
    }
    __syncthreads();
    for (int b = t; b < nbins; b += kHistBlock) {
        const unsigned int c = hist[b];
        if (c) atomicAdd(&counts[b], (unsigned long long)c);
    }
}

__global__ void k_fill_u64(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace

hipError_t launch_rdf(const double4 *rp, int off, int n, double r_select, double dr, int nbins, int32_t *refs,
                      int *nref, unsigned long long *counts, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_fill_u64, dim3((nbins + 255) / 256), dim3(256), 0, s, counts, nbins);
    hipLaunchKernelGGL(k_rdf_select, dim3(1), dim3(kSelBlock), 0, s, rp, off, n, r_select, refs, nref);
    if (n > 0) {
        const size_t lds = (size_t)nbins * sizeof(unsigned int);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_rdf_hist),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        // enough workgroups for every atom to be a reference; the surplus
        // ones return at once
        hipLaunchKernelGGL(k_rdf_hist, dim3((n + kRefsPerBlock - 1) / kRefsPerBlock), dim3(kHistBlock), lds, s, rp,
                           off, n, refs, nref, dr, nbins, counts);
    }
    return hipGetLastError();
}

}  // namespace scmd
