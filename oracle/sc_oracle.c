/*
 * Sutton-Chen oracle: a plain, slow, double-precision CPU implementation of
 * what the cluster-MD hot path computes.  TEST INFRASTRUCTURE ONLY: it is
 * called by the test suite, by the smoke check and by the CPU-baseline leg of
 * the benchmark, never by the product library, and it shares no code with it.
 *
 * Every sum below is the literal definition: a double loop over ordered pairs
 * (i, j != i) in index order, no blocking, no Newton-3 halving, no fusion.
 * Floating point is IEEE double with round-to-nearest; build without
 * -ffast-math.  OpenMP (when enabled) only splits the outer i loop; each
 * per-atom sum is still taken over j in increasing order.
 *
 * Paper: Yakubovich, Sushko, Schramm, Solov'yov, "Kinetics of liquid-solid
 * phase transition in large nickel clusters" (arXiv:1210.3559).
 *   - potential energy:       Sec. 2.1 "Interaction potential for nickel
 *                             atoms", Eq. (SC)
 *   - per-atom density:       Sec. 2.1, Eq. (rho)
 *   - Ni parameter set:       Sec. 2.1, text after Eq. (rho)
 *   - forces:                 -grad U of Eq. (SC); the paper states only that
 *                             the density sweep precedes the force sweep
 *                             (Sec. 2, "Computational approach").  The
 *                             closed form is derived at sco_forces below.
 *   - Verlet integrator, 1 fs (Sec. 2, "Computational approach", last
 *     paragraph);
 *     read as velocity-Verlet.
 *   - Berendsen thermostat with a linear target ramp: not in the paper (the
 *     paper uses Langevin); it is the deterministic thermostat of the
 *     cooling workloads this library runs.
 *   - Langevin thermostat (Sec. 2, "Computational approach": damping
 *     constant 10 1/ps), integrated with the BAOAB splitting; the noise is
 *     Philox4x32-10 with a Box-Muller transform, keyed by (seed, step, atom)
 *     so that any implementation of the same definition draws the same
 *     numbers (see sco_gauss3).
 *   - Shifted cutoff: not in the paper (which runs all-pairs and calls a
 *     cutoff future work); both power sums are shifted to zero at rc and the
 *     forces are the exact gradient of that shifted energy.
 */
#include "sc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* 1 u*A^2/fs^2 in eV (CODATA 2018: e = 1.602176634e-19 J, u = 1.66053906660e-27 kg). */
#define SCO_KE_EV_PER_U_A2_FS2 103.64269652680505
/* Boltzmann constant in eV/K (SI 2019 exact k_B divided by e). */
#define SCO_KB_EV_PER_K 8.617333262145179e-05

double sco_ke_conversion(void) { return SCO_KE_EV_PER_U_A2_FS2; }
double sco_kb(void) { return SCO_KB_EV_PER_K; }

static void set_threads(int nthreads) {
#ifdef _OPENMP
    omp_set_num_threads(nthreads > 0 ? nthreads : 1);
#else
    (void)nthreads;
#endif
}

int sco_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static double dist(const double *pos, int64_t i, int64_t j, double d[3]) {
    d[0] = pos[3 * i + 0] - pos[3 * j + 0];
    d[1] = pos[3 * i + 1] - pos[3 * j + 1];
    d[2] = pos[3 * i + 2] - pos[3 * j + 2];
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* A pair (i, j) contributes iff there is no cutoff or r < rc. */
static int inside(const sco_params *p, double r) { return !(p->rc > 0.0) || r < p->rc; }

/* (a/r)^k, shifted by (a/rc)^k when a cutoff is set (zero at r = rc). */
static double power_term(const sco_params *p, double r, int k) {
    double v = pow(p->a / r, (double)k);
    if (p->rc > 0.0) v -= pow(p->a / p->rc, (double)k);
    return v;
}

/* Eq. (rho): rho_i = sum_{j != i} (a / r_ij)^m. */
void sco_density(int64_t n, const double *pos, const sco_params *p, double *rho, int nthreads) {
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            double r = dist(pos, i, j, d);
            if (!inside(p, r)) continue;
            s += power_term(p, r, p->m);
        }
        rho[i] = s;
    }
}

/*
 * Forces F_i = -dU/dr_i of Eq. (SC).  With psi_k = rho_k^(-1/2):
 *   F_i = eps * sum_{j != i} [ n (a/r)^n - (c m / 2)(psi_i + psi_j)(a/r)^m ] (r_i - r_j) / r^2
 * The pair part comes from both the i and the j site terms (each holds half
 * of the pair sum); the embedding part from d sqrt(rho_k)/d r_i for k = i
 * and for every k = j.  Shifting by constants does not change a derivative,
 * so the cutoff form is the same bracket restricted to r < rc, with the
 * shifted densities inside psi.
 *
 * site_energy (optional) receives eps * [ 1/2 sum_j (a/r)^n - c sqrt(rho_i) ].
 * An atom with rho_i = 0 has no neighbour; its psi is taken as 0 and is
 * never multiplied by a non-zero term.
 */
void sco_forces(int64_t n, const double *pos, const sco_params *p, double *force, double *rho_out,
                double *site_energy, int nthreads) {
    double *rho = rho_out ? rho_out : (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *psi = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    sco_density(n, pos, p, rho, nthreads);
    for (int64_t i = 0; i < n; ++i) psi[i] = rho[i] > 0.0 ? 1.0 / sqrt(rho[i]) : 0.0;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double f[3] = {0.0, 0.0, 0.0};
        double pair_sum = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            double r = dist(pos, i, j, d);
            if (!inside(p, r)) continue;
            double an = pow(p->a / r, (double)p->n);
            double am = pow(p->a / r, (double)p->m);
            double coef = p->eps * ((double)p->n * an - 0.5 * p->c * (double)p->m * (psi[i] + psi[j]) * am) / (r * r);
            f[0] += coef * d[0];
            f[1] += coef * d[1];
            f[2] += coef * d[2];
            pair_sum += power_term(p, r, p->n);
        }
        force[3 * i + 0] = f[0];
        force[3 * i + 1] = f[1];
        force[3 * i + 2] = f[2];
        if (site_energy) site_energy[i] = p->eps * (0.5 * pair_sum - p->c * sqrt(rho[i]));
    }
    free(psi);
    if (!rho_out) free(rho);
}

/*
 * The same force definition evaluated only for the k atoms listed in idx
 * (for spot checks of large systems): the density sweep still covers every
 * atom, because F_i needs psi_j of every partner j.  force receives k x 3.
 */
void sco_forces_subset(int64_t n, const double *pos, const sco_params *p, const int64_t *idx, int64_t k,
                       double *force, double *rho_out, int nthreads) {
    double *rho = rho_out ? rho_out : (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *psi = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    sco_density(n, pos, p, rho, nthreads);
    for (int64_t i = 0; i < n; ++i) psi[i] = rho[i] > 0.0 ? 1.0 / sqrt(rho[i]) : 0.0;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < k; ++q) {
        const int64_t i = idx[q];
        double f[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            double r = dist(pos, i, j, d);
            if (!inside(p, r)) continue;
            double an = pow(p->a / r, (double)p->n);
            double am = pow(p->a / r, (double)p->m);
            double coef = p->eps * ((double)p->n * an - 0.5 * p->c * (double)p->m * (psi[i] + psi[j]) * am) / (r * r);
            f[0] += coef * d[0];
            f[1] += coef * d[1];
            f[2] += coef * d[2];
        }
        force[3 * q + 0] = f[0];
        force[3 * q + 1] = f[1];
        force[3 * q + 2] = f[2];
    }
    free(psi);
    if (!rho_out) free(rho);
}

/* Eq. (SC): U = eps * sum_i [ 1/2 sum_{j != i} (a/r)^n - c sqrt(rho_i) ]. */
double sco_energy(int64_t n, const double *pos, const sco_params *p, double *site_energy, int nthreads) {
    double *rho = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *site = site_energy ? site_energy : (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    sco_density(n, pos, p, rho, nthreads);
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double pair_sum = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            double r = dist(pos, i, j, d);
            if (!inside(p, r)) continue;
            pair_sum += power_term(p, r, p->n);
        }
        site[i] = p->eps * (0.5 * pair_sum - p->c * sqrt(rho[i]));
    }
    double u = 0.0;
    for (int64_t i = 0; i < n; ++i) u += site[i];
    free(rho);
    if (!site_energy) free(site);
    return u;
}

/* Degrees of freedom of a free cluster with zero linear and angular momentum. */
int64_t sco_ndof(int64_t n) {
    if (n >= 3) return 3 * n - 6;
    if (n == 2) return 1;
    return 0;
}

double sco_kinetic(int64_t n, const double *vel, double mass_u) {
    double s = 0.0;
    for (int64_t i = 0; i < 3 * n; ++i) s += vel[i] * vel[i];
    return 0.5 * mass_u * s * SCO_KE_EV_PER_U_A2_FS2;
}

double sco_temperature(int64_t n, const double *vel, double mass_u) {
    int64_t dof = sco_ndof(n);
    if (dof <= 0) return 0.0;
    return 2.0 * sco_kinetic(n, vel, mass_u) / ((double)dof * SCO_KB_EV_PER_K);
}

/* Linear target ramp begun at step count k0 (ramp_origin):
 * T_s + (T_e - T_s) * min(k - k0, K) / K for k >= k0, T_s before (K <= 0:
 * T_e at once).  A temperature programme of several legs (heating, then
 * cooling) is a sequence of ramps, each begun where the previous one ends. */
double sco_target_temperature(const sco_thermostat *t, int64_t k) {
    if (t->ramp_steps <= 0) return t->T_end;
    int64_t kr = k - t->ramp_origin;
    if (kr < 0) kr = 0;
    int64_t kk = kr < t->ramp_steps ? kr : t->ramp_steps;
    return t->T_start + (t->T_end - t->T_start) * (double)kk / (double)t->ramp_steps;
}

/* Berendsen factor lambda = sqrt(1 + (dt/tau)(T_target/T - 1)); 1 when T = 0. */
double sco_berendsen_lambda(double T, double T_target, double dt, double tau) {
    if (!(T > 0.0)) return 1.0;
    double x = 1.0 + (dt / tau) * (T_target / T - 1.0);
    return x > 0.0 ? sqrt(x) : 0.0;
}

/* Degrees of freedom by thermostat: the Langevin bath exchanges momentum and
 * angular momentum with the cluster, so all 3N are thermal; the
 * deterministic kinds conserve both (3N - 6). */
int64_t sco_ndof_kind(int64_t n, int kind) {
    if (kind == SCO_LANGEVIN) return 3 * n;
    return sco_ndof(n);
}

double sco_temperature_dof(int64_t n, const double *vel, double mass_u, int64_t dof) {
    if (dof <= 0) return 0.0;
    return 2.0 * sco_kinetic(n, vel, mass_u) / ((double)dof * SCO_KB_EV_PER_K);
}

/*
 * Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): a 128-bit counter (four 32-bit words) is passed
 * ten times through the Philox round under a 64-bit key.  A round multiplies
 * words 0 and 2 by the two Philox multipliers into 64-bit products and
 * rebuilds the block as
 *   (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0));
 * between rounds the key words are advanced by the two Weyl increments
 * (the golden ratio and sqrt(3) - 1, as 32-bit fractions).
 */
#define SCO_PHILOX_M0 0xD2511F53u
#define SCO_PHILOX_M1 0xCD9E8D57u
#define SCO_PHILOX_W0 0x9E3779B9u
#define SCO_PHILOX_W1 0xBB67AE85u

void sco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += SCO_PHILOX_W0;
            k1 += SCO_PHILOX_W1;
        }
        const uint64_t p0 = (uint64_t)SCO_PHILOX_M0 * (uint64_t)c[0];
        const uint64_t p1 = (uint64_t)SCO_PHILOX_M1 * (uint64_t)c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        const uint32_t n3 = (uint32_t)p0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
    }
    memcpy(out, c, sizeof(c));
}

/*
 * Langevin noise of one atom at one step: three independent standard normal
 * deviates.  One Philox4x32-10 block, key (seed mod 2^32, seed div 2^32),
 * counter (atom, 0, step mod 2^32, step div 2^32); each word w becomes the
 * uniform u = (w + 1/2) / 2^32 in (0, 1), and the Box-Muller transform turns
 * (u0, u1) into sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1) and u2, u3 into
 * sqrt(-2 ln u2) cos 2 pi u3.
 */
void sco_gauss3(uint64_t seed, int64_t step, int64_t atom, double out[3]) {
    const uint64_t st = (uint64_t)step;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {(uint32_t)atom, 0u, (uint32_t)st, (uint32_t)(st >> 32)};
    uint32_t w[4];
    sco_philox4x32_10(ctr, key, w);
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((double)w[k] + 0.5) / 4294967296.0;
    const double two_pi = 6.283185307179586476925286766559;
    const double ra = sqrt(-2.0 * log(u[0]));
    const double rb = sqrt(-2.0 * log(u[2]));
    out[0] = ra * cos(two_pi * u[1]);
    out[1] = ra * sin(two_pi * u[1]);
    out[2] = rb * cos(two_pi * u[3]);
}

/*
 * Pair-distance histogram behind the radial distribution function g(r) =
 * rho(r) / rho_bar (Sec. 3, "Radial distribution function as an indicator of
 * the phase transition", Eq. (Rdist)): the reference atoms are those closer
 * than r_select to the centre of mass (x_c = (sum_i x_i) / n in index order;
 * r_select <= 0 takes every atom); for each reference atom i and every other
 * atom j, r = sqrt(dx*dx + dy*dy + dz*dz) with d = r_i - r_j, and the pair
 * is counted in bin floor(r / dr) when that is below nbins.  counts[nbins]
 * and *n_ref are added to (the caller clears them), so frames accumulate.
 * Returns 0, or -1 on bad arguments.
 */
int sco_rdf(int64_t n, const double *pos, double r_select, double dr, int nbins, uint64_t *counts,
            int64_t *n_ref) {
    if (n < 0 || !(dr > 0.0) || nbins <= 0) return -1;
    double c[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) c[d] += pos[3 * i + d];
    if (n > 0)
        for (int d = 0; d < 3; ++d) c[d] /= (double)n;
    const double rs2 = r_select * r_select;
    for (int64_t i = 0; i < n; ++i) {
        const double ex = pos[3 * i] - c[0], ey = pos[3 * i + 1] - c[1], ez = pos[3 * i + 2] - c[2];
        if (r_select > 0.0 && !(ex * ex + ey * ey + ez * ez < rs2)) continue;
        *n_ref += 1;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = pos[3 * i] - pos[3 * j];
            const double dy = pos[3 * i + 1] - pos[3 * j + 1];
            const double dz = pos[3 * i + 2] - pos[3 * j + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double b = floor(r / dr);
            if (b < (double)nbins) counts[(int64_t)b] += 1;
        }
    }
    return 0;
}

/*
 * Velocity-Verlet trajectory.  On entry pos/vel hold r(t0), v(t0) (n x 3,
 * row-major); force holds F(r(t0)) when have_force is set, else it is
 * computed first.  Each step:
 *   v += (dt/2m) F;  r += dt v;  F = F(r);  v += (dt/2m) F;
 *   then, for the Berendsen kind, T from v, the target of the completed
 *   step index (step0 + k), and v *= lambda.
 * The Langevin kind (the paper's thermostat, Sec. 2 "Computational
 * approach": damping constant gamma) replaces the drift by the BAOAB
 * splitting of Leimkuhler and Matthews: for the step numbered s (the steps
 * of a trajectory count from 1, s = step0 + k + 1)
 *   v += (dt/2m) F;  r += (dt/2) v;
 *   v = c1 v + c2 xi_s  with c1 = exp(-gamma dt),
 *                       c2 = sqrt((1 - c1^2) k_B T_target(s) / m),
 *                       xi_s from sco_gauss3(seed, s, atom);
 *   r += (dt/2) v;  F = F(r);  v += (dt/2m) F;
 * and T counts 3N degrees of freedom.
 * Per step k (0-based in this call) the log receives, when not NULL,
 *   log[4k + 0] = E_pot, [1] = E_kin, [2] = T, [3] = T_target,
 * all of the state after the thermostat has acted.
 */
int sco_vv_run(int64_t n, double *pos, double *vel, double *force, int have_force, const sco_params *p,
               double mass_u, double dt, int64_t nsteps, const sco_thermostat *thermo, int64_t step0,
               double *log, int nthreads) {
    if (n < 0 || nsteps < 0 || !(dt > 0.0) || !(mass_u > 0.0)) return -1;
    const int langevin = thermo && thermo->kind == SCO_LANGEVIN;
    if (langevin && !(thermo->gamma >= 0.0)) return -1;
    double h = 0.5 * dt / (mass_u * SCO_KE_EV_PER_U_A2_FS2);
    const int64_t dof = sco_ndof_kind(n, thermo ? thermo->kind : SCO_NVE);
    double *site = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!have_force) sco_forces(n, pos, p, force, NULL, NULL, nthreads);
    for (int64_t k = 0; k < nsteps; ++k) {
        double Tt = 0.0;
        for (int64_t i = 0; i < 3 * n; ++i) vel[i] += h * force[i];
        if (langevin) {
            const int64_t s = step0 + k + 1;
            Tt = sco_target_temperature(thermo, s);
            const double c1 = exp(-thermo->gamma * 1e-3 * dt); /* gamma in 1/ps, dt in fs */
            const double c2 = sqrt((1.0 - c1 * c1) * SCO_KB_EV_PER_K * Tt / (mass_u * SCO_KE_EV_PER_U_A2_FS2));
            for (int64_t i = 0; i < 3 * n; ++i) pos[i] += 0.5 * dt * vel[i];
            for (int64_t i = 0; i < n; ++i) {
                double xi[3];
                sco_gauss3(thermo->seed, s, i, xi);
                for (int d = 0; d < 3; ++d) vel[3 * i + d] = c1 * vel[3 * i + d] + c2 * xi[d];
            }
            for (int64_t i = 0; i < 3 * n; ++i) pos[i] += 0.5 * dt * vel[i];
        } else {
            for (int64_t i = 0; i < 3 * n; ++i) pos[i] += dt * vel[i];
        }
        sco_forces(n, pos, p, force, NULL, site, nthreads);
        for (int64_t i = 0; i < 3 * n; ++i) vel[i] += h * force[i];
        double T = sco_temperature_dof(n, vel, mass_u, dof);
        if (thermo && thermo->kind == SCO_BERENDSEN) {
            Tt = sco_target_temperature(thermo, step0 + k + 1);
            double lam = sco_berendsen_lambda(T, Tt, dt, thermo->tau);
            for (int64_t i = 0; i < 3 * n; ++i) vel[i] *= lam;
            T = sco_temperature_dof(n, vel, mass_u, dof);
        }
        if (log) {
            double u = 0.0;
            for (int64_t i = 0; i < n; ++i) u += site[i];
            log[4 * k + 0] = u;
            log[4 * k + 1] = sco_kinetic(n, vel, mass_u);
            log[4 * k + 2] = T;
            log[4 * k + 3] = Tt;
        }
    }
    free(site);
    return 0;
}
