/*
 * Sutton-Chen oracle (test infrastructure; see sc_oracle.c).
 *
 * Positions, velocities and forces are n x 3 row-major double arrays
 * (atom-major, x y z).  Units: Angstrom, fs, eV, atomic mass unit u, Kelvin.
 *
 * Parity pins live in the test suite; every function here is pinned against
 * closed forms, lattice sums, finite differences, invariants or statistical
 * laws, except where the oracle module header says "parity unpinned".
 */
#ifndef SC_ORACLE_H
#define SC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double eps; /* energy scale, eV */
    double a;   /* length scale (fcc lattice constant), Angstrom */
    double c;   /* embedding strength, dimensionless */
    int n;      /* repulsive exponent */
    int m;      /* density exponent, n > m */
    double rc;  /* cutoff radius; <= 0 means all pairs, no cutoff */
} sco_params;

enum { SCO_NVE = 0, SCO_BERENDSEN = 1, SCO_LANGEVIN = 2 };

typedef struct {
    int kind;           /* SCO_NVE, SCO_BERENDSEN or SCO_LANGEVIN */
    double T_start;     /* K */
    double T_end;       /* K */
    int64_t ramp_steps; /* linear ramp length in steps */
    double tau;         /* Berendsen coupling time, fs */
    double gamma;       /* Langevin damping constant, 1/ps */
    uint64_t seed;      /* Langevin noise key */
    int64_t ramp_origin; /* step count at which the ramp starts */
} sco_thermostat;

double sco_ke_conversion(void);
double sco_kb(void);
int sco_max_threads(void);

void sco_density(int64_t n, const double *pos, const sco_params *p, double *rho, int nthreads);
void sco_forces(int64_t n, const double *pos, const sco_params *p, double *force, double *rho_out,
                double *site_energy, int nthreads);
void sco_forces_subset(int64_t n, const double *pos, const sco_params *p, const int64_t *idx, int64_t k,
                       double *force, double *rho_out, int nthreads);
double sco_energy(int64_t n, const double *pos, const sco_params *p, double *site_energy, int nthreads);

int64_t sco_ndof(int64_t n);
int64_t sco_ndof_kind(int64_t n, int kind);
double sco_temperature_dof(int64_t n, const double *vel, double mass_u, int64_t dof);

void sco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void sco_gauss3(uint64_t seed, int64_t step, int64_t atom, double out[3]);
double sco_kinetic(int64_t n, const double *vel, double mass_u);
double sco_temperature(int64_t n, const double *vel, double mass_u);
double sco_target_temperature(const sco_thermostat *t, int64_t k);
double sco_berendsen_lambda(double T, double T_target, double dt, double tau);

int sco_rdf(int64_t n, const double *pos, double r_select, double dr, int nbins, uint64_t *counts,
            int64_t *n_ref);

int sco_vv_run(int64_t n, double *pos, double *vel, double *force, int have_force, const sco_params *p,
               double mass_u, double dt, int64_t nsteps, const sco_thermostat *thermo, int64_t step0,
               double *log, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
