// On-device analysis of a cluster's positions: the pair-distance histogram
// of its current positions and the diffusion coefficient of stored frames.
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

// Adds the number of reference atoms to a 64-bit device total.
__global__ void k_add_nref(const int *__restrict__ nref, long long *__restrict__ total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) total[0] += (long long)nref[0];
}


// ---------------------------------------------------------------------------
// Self-diffusion coefficient of the central atoms (Sec. 3, "Diffusion
// coefficient as a fingerprint of solidification phase transition",
// Eq. (diffusion): D = <dr^2> / (2 z dt), z = 3).  A window of frames is cut
// into segments; each frame at a segment end is superimposed on the window's
// first frame by the proper rigid motion of least mean-square displacement,
// and dr is the displacement of a central atom (closer than `radius` to the
// first frame's centre of mass) between the two ends of its segment.
//
// The optimal rotation is found as a unit quaternion (Horn, J. Opt. Soc.
// Am. A 4 (1987) 629): the eigenvector of the largest eigenvalue of a
// symmetric 4x4 matrix built from the 3x3 cross-covariance
// S_ab = sum_i (p_i - p_c)_a (q_i - q_c)_b of the moving frame p and the
// reference q.  The eigenproblem is solved by cyclic Jacobi rotations; a
// quaternion always gives a proper rotation, so no reflection can appear.
// ---------------------------------------------------------------------------
constexpr int kDiffBlock = 256;

// Sum of K per-thread values over the workgroup in a fixed order (xor
// butterfly in each wavefront, then the wavefronts in index order); every
// thread receives the totals.
template <int K>
__device__ void block_sum(double (&v)[K], double *sh) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    constexpr int W = kDiffBlock / 64;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        v[k] = x;
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = sh[k];
        for (int q = 1; q < W; ++q) x += sh[q * K + k];
        v[k] = x;
    }
}

// Rotation matrix (row-major) of the proper rigid motion taking the centred
// moving frame onto the centred reference, from the cross-covariance S.
__device__ void horn_rotation(const double S[9], double R[9]) {
    const double Sxx = S[0], Sxy = S[1], Sxz = S[2];
    const double Syx = S[3], Syy = S[4], Syz = S[5];
    const double Szx = S[6], Szy = S[7], Szz = S[8];
    double A[4][4] = {{Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx},
                      {Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz},
                      {Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy},
                      {Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz}};
    double V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    double scale = 0.0;
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) scale += A[p][q] * A[p][q];
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) off += A[p][q] * A[p][q];
        if (!(off > 1e-34 * scale)) break;
        for (int p = 0; p < 3; ++p) {
            for (int q = p + 1; q < 4; ++q) {
                const double apq = A[p][q];
                if (fabs(apq) <= 1e-300) continue;
                // rotation angle that zeroes A[p][q]: t = tan(phi) is the
                // smaller root of t^2 + 2 theta t - 1 = 0
                const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                double t;
                if (fabs(theta) > 1e150)
                    t = 0.5 / theta;
                else
                    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 4; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 4; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 4; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
        }
    }
    int best = 0;
    for (int k = 1; k < 4; ++k)
        if (A[k][k] > A[best][best]) best = k;
    double a = V[0][best], b = V[1][best], c = V[2][best], d = V[3][best];
    const double inv = 1.0 / sqrt(a * a + b * b + c * c + d * d);
    a *= inv;
    b *= inv;
    c *= inv;
    d *= inv;
    R[0] = a * a + b * b - c * c - d * d;
    R[1] = 2.0 * (b * c - a * d);
    R[2] = 2.0 * (b * d + a * c);
    R[3] = 2.0 * (b * c + a * d);
    R[4] = a * a - b * b + c * c - d * d;
    R[5] = 2.0 * (c * d - a * b);
    R[6] = 2.0 * (b * d - a * c);
    R[7] = 2.0 * (c * d + a * b);
    R[8] = a * a - b * b - c * c + d * d;
}

// Workgroup s: segment s of the window of frames [first, first + S seg)
// (frame f sits at ring slot f % cap, n atoms each).  Writes the segment's
// <dr^2> / (6 (seg - 1) dt) to seg_d[s] and the number of central atoms to
// *ncentral (segment 0).
__global__ __launch_bounds__(kDiffBlock) void k_diffusion_segments(const double4 *__restrict__ frames, int n,
                                                                  int cap, int64_t first, int seg, double radius,
                                                                  double dt_ps, double *__restrict__ seg_d,
                                                                  int *__restrict__ ncentral) {
    __shared__ double sh[(kDiffBlock / 64) * 18];
    __shared__ double rot[18];
    const int t = threadIdx.x;
    const int64_t fa = first + (int64_t)blockIdx.x * seg, fb = fa + seg - 1;
    const double4 *q = frames + (size_t)(first % cap) * n;
    const double4 *pa = frames + (size_t)(fa % cap) * n;
    const double4 *pb = frames + (size_t)(fb % cap) * n;
    // centres of the reference and of both segment ends
    double c9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = t; i < n; i += kDiffBlock) {
        const double4 x = q[i], y = pa[i], z = pb[i];
        c9[0] += x.x;
        c9[1] += x.y;
        c9[2] += x.z;
        c9[3] += y.x;
        c9[4] += y.y;
        c9[5] += y.z;
        c9[6] += z.x;
        c9[7] += z.y;
        c9[8] += z.z;
    }
    block_sum<9>(c9, sh);
    const double inv_n = 1.0 / (double)n;
    const double qx = c9[0] * inv_n, qy = c9[1] * inv_n, qz = c9[2] * inv_n;
    const double ax = c9[3] * inv_n, ay = c9[4] * inv_n, az = c9[5] * inv_n;
    const double bx = c9[6] * inv_n, by = c9[7] * inv_n, bz = c9[8] * inv_n;
    // cross-covariances of both ends with the reference
    double s18[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) s18[k] = 0.0;
    for (int i = t; i < n; i += kDiffBlock) {
        const double4 x = q[i], y = pa[i], z = pb[i];
        const double r0 = x.x - qx, r1 = x.y - qy, r2 = x.z - qz;
        const double a0 = y.x - ax, a1 = y.y - ay, a2 = y.z - az;
        const double b0 = z.x - bx, b1 = z.y - by, b2 = z.z - bz;
        s18[0] += a0 * r0; s18[1] += a0 * r1; s18[2] += a0 * r2;
        s18[3] += a1 * r0; s18[4] += a1 * r1; s18[5] += a1 * r2;
        s18[6] += a2 * r0; s18[7] += a2 * r1; s18[8] += a2 * r2;
        s18[9] += b0 * r0; s18[10] += b0 * r1; s18[11] += b0 * r2;
        s18[12] += b1 * r0; s18[13] += b1 * r1; s18[14] += b1 * r2;
        s18[15] += b2 * r0; s18[16] += b2 * r1; s18[17] += b2 * r2;
    }
    block_sum<18>(s18, sh);
    if (t == 0) {
        horn_rotation(s18, rot);
        horn_rotation(s18 + 9, rot + 9);
    }
    __syncthreads();
    double Ra[9], Rb[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Ra[k] = rot[k];
        Rb[k] = rot[9 + k];
    }
    // squared displacement of the central atoms between the superimposed ends
    const double r2max = radius * radius;
    double acc[2] = {0.0, 0.0};
    for (int i = t; i < n; i += kDiffBlock) {
        const double4 x = q[i];
        const double e0 = x.x - qx, e1 = x.y - qy, e2 = x.z - qz;
        if (!(e0 * e0 + e1 * e1 + e2 * e2 < r2max)) continue;
        const double4 y = pa[i], z = pb[i];
        const double a0 = y.x - ax, a1 = y.y - ay, a2 = y.z - az;
        const double b0 = z.x - bx, b1 = z.y - by, b2 = z.z - bz;
        const double d0 = (Rb[0] * b0 + Rb[1] * b1 + Rb[2] * b2) - (Ra[0] * a0 + Ra[1] * a1 + Ra[2] * a2);
        const double d1 = (Rb[3] * b0 + Rb[4] * b1 + Rb[5] * b2) - (Ra[3] * a0 + Ra[4] * a1 + Ra[5] * a2);
        const double d2 = (Rb[6] * b0 + Rb[7] * b1 + Rb[8] * b2) - (Ra[6] * a0 + Ra[7] * a1 + Ra[8] * a2);
        acc[0] += d0 * d0 + d1 * d1 + d2 * d2;
        acc[1] += 1.0;
    }
    block_sum<2>(acc, sh);
    if (t == 0) {
        const double cnt = acc[1];
        seg_d[blockIdx.x] = cnt > 0.0 ? acc[0] / cnt / (6.0 * (double)(seg - 1) * dt_ps) : 0.0;
        if (blockIdx.x == 0) *ncentral = (int)cnt;
    }
}

// Mean of the per-segment coefficients in segment order.
__global__ void k_diffusion_finish(const double *__restrict__ seg_d, int segments, double *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < segments; ++k) s += seg_d[k];
    out[0] = s / (double)segments;
}

// Frame store: cluster atoms [off, off + n) into ring slot `slot`.
__global__ void k_store_frame(const double4 *__restrict__ rp, int off, int n, double4 *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = rp[off + i];
}

}  // namespace

hipError_t launch_rdf(const double4 *rp, int off, int n, double r_select, double dr, int nbins, int32_t *refs,
                      int *nref, unsigned long long *counts, bool clear, long long *nref_total, hipStream_t s) {
    (void)hipGetLastError();
    if (clear) hipLaunchKernelGGL(k_fill_u64, dim3((nbins + 255) / 256), dim3(256), 0, s, counts, nbins);
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
    if (nref_total) hipLaunchKernelGGL(k_add_nref, dim3(1), dim3(64), 0, s, nref, nref_total);
    return hipGetLastError();
}

hipError_t launch_store_frame(const double4 *rp, int off, int n, double4 *dst, hipStream_t s) {
    (void)hipGetLastError();
    if (n > 0) hipLaunchKernelGGL(k_store_frame, dim3((n + 255) / 256), dim3(256), 0, s, rp, off, n, dst);
    return hipGetLastError();
}

hipError_t launch_diffusion(const double4 *frames, int n, int cap, int64_t first, int seg, int segments,
                            double radius, double dt_ps, double *seg_d, int *ncentral, double *d_out,
                            hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_diffusion_segments, dim3(segments), dim3(kDiffBlock), 0, s, frames, n, cap, first, seg,
                       radius, dt_ps, seg_d, ncentral);
    hipLaunchKernelGGL(k_diffusion_finish, dim3(1), dim3(64), 0, s, seg_d, segments, d_out);
    return hipGetLastError();
}

}  // namespace scmd
