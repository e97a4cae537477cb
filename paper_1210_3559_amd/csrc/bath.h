// Langevin bath of the cluster (the thermostat of the paper, Sec. 2
// "Computational approach": friction with a damping constant gamma),
// integrated with the BAOAB splitting of Leimkuhler and Matthews.  For the
// step numbered s (steps of a cluster count from 1) and an atom whose
// velocity after the first half-kick is v1:
//   r <- r + (dt/2) v1
//   v <- c1 v1 + c2 xi,   c1 = exp(-gamma dt),
//                         c2 = sqrt((1 - c1^2) k_B T_target(s) / m)
//   r <- r + (dt/2) v
// then the force sweep and the second half-kick.  The noise xi is three
// standard normal deviates drawn from the counter-based generator
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) through the
// Box-Muller transform: key (seed low word, seed high word), counter
// (atom index in its cluster, 0, s low word, s high word), the four output
// words w become uniforms (w + 1/2) 2^-32, and
//   xi = sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1),  sqrt(-2 ln u2) cos 2 pi u3.
// Keying by (seed, step, atom) makes the noise independent of the launch
// shape and of how a run is split into calls.
#pragma once

#include "scmd_internal.h"

namespace scmd {
namespace dev {

struct Words4 {
    uint32_t a, b, c, d;
};

// Ten Philox rounds: words a and c are multiplied by the two round
// multipliers; the high halves are mixed with the other two words and the
// key, and the key advances by the two Weyl increments between rounds.
__device__ __forceinline__ Words4 philox4x32_10(Words4 x, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = kM0 * x.a, hi0 = __umulhi(kM0, x.a);
        const uint32_t lo1 = kM1 * x.c, hi1 = __umulhi(kM1, x.c);
        x = Words4{hi1 ^ x.b ^ k0, lo1, hi0 ^ x.d ^ k1, lo0};
        k0 += kW0;
        k1 += kW1;
    }
    return x;
}

__device__ __forceinline__ double unit_open(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

// The three deviates of atom `atom` at step `step` (see the file comment).
__device__ __forceinline__ double3 bath_noise(uint64_t seed, int64_t step, int atom) {
#pragma clang fp contract(off)
    const uint64_t s = (uint64_t)step;
    const Words4 w = philox4x32_10(Words4{(uint32_t)atom, 0u, (uint32_t)s, (uint32_t)(s >> 32)}, (uint32_t)seed,
                                   (uint32_t)(seed >> 32));
    const double ra = sqrt(-2.0 * log(unit_open(w.a)));
    const double rb = sqrt(-2.0 * log(unit_open(w.c)));
    double sa, ca;
    sincospi(2.0 * unit_open(w.b), &sa, &ca);
    return make_double3(ra * ca, ra * sa, rb * cospi(2.0 * unit_open(w.d)));
}

// Target temperature of the ramp at step index k (both thermostats); the
// ramp starts at step count d.ramp_origin and holds T_start before it.
__device__ __forceinline__ double ramp_target(const ClusterDesc &d, int64_t k) {
#pragma clang fp contract(off)
    if (d.ramp <= 0) return d.T_end;
    int64_t kr = k - d.ramp_origin;
    if (kr < 0) kr = 0;
    const int64_t kk = kr < d.ramp ? kr : d.ramp;
    return d.T_start + (d.T_end - d.T_start) * (double)kk / (double)d.ramp;
}

// Noise amplitude c2 of step `step`.
__device__ __forceinline__ double bath_c2(const ClusterDesc &d, int64_t step, double mass_u) {
#pragma clang fp contract(off)
    const double c1 = d.bath_c1;
    const double tt = ramp_target(d, step);
    return sqrt((1.0 - c1 * c1) * kBoltzmannEv * tt / (mass_u * kEvPerUA2Fs2));
}

// A, O, A for one atom whose velocity v has had the first half-kick, with
// its noise xi and the step's amplitude c2 given: updates r and v in place.
__device__ __forceinline__ void bath_drift_xi(const ClusterDesc &d, double c2, const double3 &xi, double dt,
                                              double4 &r, double4 &v) {
#pragma clang fp contract(off)
    const double hdt = 0.5 * dt;
    const double c1 = d.bath_c1;
    r.x = r.x + hdt * v.x;
    r.y = r.y + hdt * v.y;
    r.z = r.z + hdt * v.z;
    v.x = c1 * v.x + c2 * xi.x;
    v.y = c1 * v.y + c2 * xi.y;
    v.z = c1 * v.z + c2 * xi.z;
    r.x = r.x + hdt * v.x;
    r.y = r.y + hdt * v.y;
    r.z = r.z + hdt * v.z;
}

__device__ __forceinline__ void bath_drift(const ClusterDesc &d, int64_t step, int atom, double mass_u, double dt,
                                           double4 &r, double4 &v) {
    bath_drift_xi(d, bath_c2(d, step, mass_u), bath_noise(d.seed, step, atom), dt, r, v);
}

}  // namespace dev
}  // namespace scmd
