/*
 * scmd.h -- C ABI of an MI355X (gfx950) molecular-dynamics library for free
 * nickel clusters with the Sutton-Chen many-body potential.
 *
 * What the library computes (Yakubovich, Sushko, Schramm, Solov'yov,
 * "Kinetics of liquid-solid phase transition in large nickel clusters",
 * arXiv:1210.3559):
 *   - potential energy U = eps sum_i [ 1/2 sum_{j!=i} (a/r_ij)^n - c sqrt(rho_i) ]
 *     (Sec. 2.1, Eq. (SC)) with rho_i = sum_{j!=i} (a/r_ij)^m (Eq. (rho));
 *   - the forces -grad U, evaluated as two all-pairs sweeps: first every
 *     rho_i, then the forces (Sec. 2, "Computational approach");
 *   - Verlet time stepping, read as velocity-Verlet (same section, last
 *     paragraph), with an optional thermostat following a linear
 *     temperature ramp: the paper's Langevin bath (same paragraph: damping
 *     constant gamma), integrated with the BAOAB splitting, or a
 *     deterministic Berendsen rescaling (the cooling runs of the benchmark
 *     workloads are driven this way);
 *   - optionally the potential truncated at rc with both power sums shifted
 *     to zero there (not in the paper, which calls a cutoff future work),
 *     evaluated with a cell list.
 *
 * Several independent clusters ("a batch") can live in one context; they
 * are stored back to back (CSR offsets) and advanced together.
 *
 * Units: Angstrom, fs, eV, atomic mass unit u, Kelvin.
 * Host arrays of positions, velocities and forces are n x 3 row-major double
 * (x y z per atom, atoms in the order given at init).
 *
 * Errors: every call returns SCMD_OK (0) or a negative SCMD_E* code; on
 * error no output argument is written and scmd_last_error() describes the
 * failure.  No C++ exception crosses this interface.
 *
 * Ownership: the caller owns every buffer it passes; the library copies
 * inputs during the call and never keeps a caller pointer.  The library
 * owns its device memory and graph objects; scmd_destroy releases them.
 *
 * Threading and streams: a context is not thread-safe.  All device work of
 * a context is ordered on one HIP stream (the one given to scmd_create, or
 * a non-blocking stream the library creates).
 *
 * Call order: scmd_create -> scmd_init_clusters -> scmd_set_potential ->
 * scmd_set_integrator -> [scmd_set_thermostat ...] -> scmd_compute /
 * scmd_step -> scmd_get_*.  A call before its prerequisites returns
 * SCMD_ESTATE.  Re-initialising clusters or changing the potential or the
 * integrator discards the step count, forces and captured graphs.
 */
#ifndef SCMD_H
#define SCMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCMD_ABI_VERSION 1

typedef struct scmd_ctx scmd_ctx;

/* Status codes. */
enum {
    SCMD_OK = 0,
    SCMD_EINVAL = -1,       /* bad argument (null pointer, size, range)            */
    SCMD_ENOMEM = -2,       /* device or host allocation failed                     */
    SCMD_EDEVICE = -3,      /* no usable gfx950 device or a HIP runtime error       */
    SCMD_ENONFINITE = -4,   /* a non-finite energy appeared (e.g. coincident atoms) */
    SCMD_ESTATE = -5,       /* call out of order                                    */
    SCMD_EBOX = -6,         /* reserved: the cell list coarsens its cells instead   */
    SCMD_EUNSUPPORTED = -7  /* valid request this build does not implement          */
};

/* Arithmetic of the pair sweeps. */
enum {
    SCMD_FP64 = 0,  /* every operation in double precision                          */
    SCMD_MIXED = 1  /* r_i - r_j and r^2 in double, then 1/r, the powers and the
                       pair coefficient in single precision; each term added to
                       double accumulators (force terms as f * (r_i - r_j) in
                       double); positions, velocities and integration double    */
};

/* Neighbour handling. */
enum {
    SCMD_ALLPAIRS = 0, /* every pair (i, j != i); requires rc == 0                 */
    SCMD_CELLLIST = 1  /* pairs with r < rc found through a cell list; rc > 0      */
};

/* Thermostats. */
enum {
    SCMD_NVE = 0,       /* no thermostat                                             */
    SCMD_BERENDSEN = 1, /* velocity rescaling towards a linear ramp T_start -> T_end */
    SCMD_LANGEVIN = 2   /* the paper's Langevin bath (set with scmd_set_langevin)     */
};

/* Sutton-Chen parameters (Sec. 2.1).  Ni: eps = 1.5707e-2 eV, a = 3.52 A,
 * c = 39.432, n = 9, m = 6.  Integer exponents with 1 <= m < n <= 24.
 * rc > 0 truncates at rc and shifts (a/r)^n and (a/r)^m to zero there. */
typedef struct {
    double eps;
    double a;
    double c;
    int n;
    int m;
    double rc;
} scmd_sc_params;

/* Launch shape of the all-pairs sweeps (all zero = library defaults).
 * An atom tile holds 64 * ipt * waves_i atoms (ipt atoms per lane, waves_i
 * wavefronts along i); waves_j wavefronts split each tile's partner range
 * inside a workgroup of 64 * waves_i * waves_j threads.  Supported
 * (ipt, waves_i, waves_j): (1,4,1) (2,4,1) (1,2,2) (2,2,2) (1,1,4) (2,1,4)
 * (1,2,4) (2,2,4) (1,4,4) (1,1,8) (2,1,8) (1,2,8) (1,1,16) (4,1,2) (4,1,4)
 * (4,2,2).  target_items:
 * aim for about this many workgroups per sweep when splitting partner
 * ranges across workgroups (0 = default).  Results may differ in the last
 * bits between shapes (summation order); a given shape is deterministic. */
typedef struct {
    int ipt;
    int waves_i;
    int waves_j;
    int target_items;
    int pairs; /* 0 = library choice; 1 = one-sided sweeps (every atom owns its
                  sums, shapes above); 2 = symmetric sweeps (each unordered
                  pair evaluated once, j tiles rotated through the wavefront;
                  ipt 2, 4 or 8, waves_i and waves_j ignored; (n, m) = (9, 6) and
                  all-pairs only); 3 = row sweeps (one workgroup of
                  64 * waves_j threads per run of at most 8 * waves_j atoms
                  against all of its partners, finished in the same launch;
                  waves_j 4, 8 or 16 (0 = 8), target_items = workgroups per
                  sweep (0 = 256), ipt and waves_i ignored; all-pairs only) */
} scmd_tuning;

/* Kernel classes timed by scmd_get_kernel_time (device time per launch). */
enum {
    SCMD_KERNEL_DENSITY = 0, /* density sweep (rho partial sums)          */
    SCMD_KERNEL_FORCE = 1,   /* force sweep (force and pair-energy sums)   */
    SCMD_KERNEL_COUNT = 2
};

/* Returns SCMD_ABI_VERSION. */
int scmd_abi_version(void);

/* Human-readable name of a status code (static string). */
const char *scmd_status_string(int status);

/* Create a context on HIP device `device` (must be gfx950).  `hip_stream`
 * is a hipStream_t the caller keeps alive for the context's lifetime, or NULL
 * for a library-owned non-blocking stream.  *out receives the context.
 * Returns SCMD_EDEVICE when there is no such device. */
int scmd_create(scmd_ctx **out, int device, void *hip_stream);

/* Wait for outstanding work and free everything the context owns.  NULL is
 * accepted and ignored. */
int scmd_destroy(scmd_ctx *ctx);

/* Load n_clusters independent clusters.  offsets[n_clusters + 1] (host,
 * int64, offsets[0] = 0, non-decreasing; empty clusters allowed) delimit the
 * atoms of each cluster inside pos and vel (host, offsets[n_clusters] x 3
 * doubles, A and A/fs).  vel may be NULL (all zero).  mass_u > 0 is the atomic
 * mass (58.6934 for Ni).  The total atom count must be below 2^30.  Copies the
 * data to the device; the caller's arrays may be reused at return.  A batch
 * holds the paper's ensembles of independent runs of one cluster (Sec. 3,
 * "Kinetics of the solidification phase transition", Table LT). */
int scmd_init_clusters(scmd_ctx *ctx, int n_clusters, const int64_t *offsets, const double *pos,
                       const double *vel, double mass_u);

/* Set the potential (Sec. 2.1).  Requires eps > 0, a > 0, c >= 0,
 * 1 <= m < n <= 24 and rc >= 0. */
int scmd_set_potential(scmd_ctx *ctx, const scmd_sc_params *params);

/* Time step dt_fs > 0 (the paper uses 1 fs), precision SCMD_FP64 or
 * SCMD_MIXED, neighbour SCMD_ALLPAIRS (needs rc == 0) or SCMD_CELLLIST
 * (needs rc > 0; the cell list keeps about 1 KiB of device memory per atom
 * for the neighbours each atom's density sweep finds, plus O(cells) for the
 * grid). */
int scmd_set_integrator(scmd_ctx *ctx, double dt_fs, int precision, int neighbour);

/* Thermostat of one cluster (cluster = -1: every cluster).  Berendsen: after
 * the second half-kick of step k (k counts completed steps of that cluster
 * since init, from 1), T_k = 2 E_kin / (ndof k_B) with ndof = 3N - 6 (1 for a
 * dimer, 0 below), target T_start + (T_end - T_start) min(k - k0, K)/K for
 * k >= k0, where k0 is the cluster's step count when this call was made
 * (the ramp starts now: a programme of several legs is one call per leg;
 * K = ramp_steps; K <= 0 means T_end at once), lambda =
 * sqrt(1 + (dt/tau)(target/T_k - 1)) (1 when T_k = 0, 0 when the radicand is
 * negative), v <- lambda v.  tau_fs > 0; temperatures >= 0.  SCMD_NVE
 * ignores the other arguments.  SCMD_LANGEVIN returns SCMD_EINVAL (its
 * parameters differ: use scmd_set_langevin). */
int scmd_set_thermostat(scmd_ctx *ctx, int cluster, int kind, double T_start_K, double T_end_K,
                        int64_t ramp_steps, double tau_fs);

/* Langevin bath of one cluster (cluster = -1: every cluster), the paper's
 * thermostat (Sec. 2, "Computational approach": damping constant 10 1/ps at
 * a 1 fs step).  Each step, numbered s = k + 1 when k steps of the cluster
 * are complete (counted since init, carried by checkpoints), is BAOAB:
 *   v += (dt/2m) F;  r += (dt/2) v;
 *   v = c1 v + c2 xi,  c1 = exp(-gamma dt),
 *                      c2 = sqrt((1 - c1^2) k_B T_target(s) / m);
 *   r += (dt/2) v;  F = F(r);  v += (dt/2m) F;
 * with T_target(s) = T_start + (T_end - T_start) min(s - k0, K)/K, k0 the
 * cluster's step count when this call was made (K = ramp_steps; K <= 0:
 * T_end).  xi is three standard normal deviates per
 * atom: the Philox4x32-10 block (Salmon et al., SC'11) of key (seed mod 2^32,
 * seed div 2^32) and counter (atom index within its cluster, 0, s mod 2^32,
 * s div 2^32), its words w mapped to u = (w + 1/2) 2^-32 and through the
 * Box-Muller transform: sqrt(-2 ln u0)(cos 2 pi u1, sin 2 pi u1),
 * sqrt(-2 ln u2) cos 2 pi u3.  The noise therefore depends only on (seed,
 * s, atom): not on the launch shape, the precision form or how steps are
 * split into calls; give clusters different seeds for independent baths.
 * The temperature of such a cluster counts ndof = 3N.  gamma_per_ps >= 0
 * (0 gives velocity-Verlet with the BAOAB rounding), temperatures finite
 * and >= 0. */
int scmd_set_langevin(scmd_ctx *ctx, int cluster, double T_start_K, double T_end_K, int64_t ramp_steps,
                      double gamma_per_ps, uint64_t seed);

/* Margin of the cell list (neighbour SCMD_CELLLIST), A (default 0.4):
 * cells of edge >= rc + skin, and per-atom lists of the candidates within
 * rc + skin, are rebuilt only once an atom has moved more than skin / 2
 * since the last rebuild, and reused in between (every pair closer than rc
 * is then still listed; the pair terms apply rc themselves).  skin = 0
 * rebuilds every step.  Results are the same up to summation order (the
 * order of a list's entries).  SCMD_EINVAL for a negative or non-finite
 * skin; takes effect at the next evaluation.  The paper sums over all pairs
 * and leaves a cutoff to later work (Sec. 2, "Computational approach"): the
 * cell list and its skin are this library's. */
int scmd_set_cell_skin(scmd_ctx *ctx, double skin_A);

/* Rebuilds of the cell list's cells and lists since it was planned (the
 * first evaluation, a change of potential, integrator or skin, or new
 * clusters plan it afresh); 0 without a cell list.  Synchronises the
 * context stream. */
int scmd_get_cell_rebuilds(scmd_ctx *ctx, int64_t *rebuilds);

/* Override the sweep launch shape (NULL restores defaults).  These shapes
 * replace the paper's one-atom-per-thread GPU scheme (Sec. 2, "Computational
 * approach"); every shape computes the same sums up to summation order. */
int scmd_set_tuning(scmd_ctx *ctx, const scmd_tuning *tuning);

/* Evaluate rho_i (Sec. 2.1, Eq. (rho)), the forces -grad U of Eq. (SC) and
 * the energies, by the paper's two sweeps over all pairs (Sec. 2,
 * "Computational approach": every density first, then the forces), and the
 * temperature, at the current positions, without moving atoms.  Enqueued on
 * the context stream; synchronises and returns SCMD_ENONFINITE when an energy
 * is not finite. */
int scmd_compute(scmd_ctx *ctx);

/* Advance every cluster by nsteps >= 0 velocity-Verlet steps (Sec. 2,
 * "Computational approach": per step a density sweep and a force sweep over
 * all pairs, integrated with velocity-Verlet; forces at the initial
 * positions are computed first if needed).  Steps are replayed from captured
 * HIP graphs: a 32-step graph and a graph of the remainder (nsteps mod 32),
 * each kept for later calls.  Waits for completion and returns SCMD_ENONFINITE
 * if an energy became non-finite during these steps (the state is then
 * undefined). */
int scmd_step(scmd_ctx *ctx, int64_t nsteps);

/* As scmd_step, but only enqueues the work: returns without waiting; errors
 * from the device surface at the next scmd_synchronize or getter. */
int scmd_step_async(scmd_ctx *ctx, int64_t nsteps);

/* Wait for the context stream; returns SCMD_ENONFINITE if flagged. */
int scmd_synchronize(scmd_ctx *ctx);

/* Completed steps of the context (all clusters advance together). */
int scmd_get_step(scmd_ctx *ctx, int64_t *step);

/* Energies of the current state of one cluster (cluster = -1: sum over all):
 * out3[0] = E_pot = U of Sec. 2.1, Eq. (SC) (with the shifted powers when
 * rc > 0), out3[1] = E_kin = sum m v^2 / 2, out3[2] = E_pot + E_kin, eV (the
 * paper follows the total energy per atom of its runs, Sec. 3).  Valid after
 * scmd_compute or scmd_step; out3 is host memory of 3 doubles. */
int scmd_get_energy(scmd_ctx *ctx, int cluster, double out3[3]);

/* Temperature T = 2 E_kin / (ndof k_B) (K) of one cluster's current state
 * and its degrees of freedom (3N - 6 for a free cluster, 3N in a Langevin
 * bath); the paper plots its runs' energy against this temperature (Sec. 3).
 * T_K (host) required, ndof may be NULL. */
int scmd_get_temperature(scmd_ctx *ctx, int cluster, double *T_K, int64_t *ndof);

/* Observables along a trajectory (the paper follows the energy per atom and
 * the temperature of its runs, Sec. 3).  With every > 0, after each step k
 * of the context step counter with k % every == 0, the state of every
 * cluster is appended to a device ring buffer that keeps the last
 * `capacity` samples; scmd_step splits its run at these steps (graph
 * replays in between).  every = 0 stops sampling.  Any call clears the
 * buffer.  SCMD_ESTATE before scmd_init_clusters; SCMD_EINVAL for
 * every < 0, or capacity < 1 with every > 0; SCMD_ENOMEM if the buffer
 * (capacity x n_clusters x 5 doubles) cannot be allocated.  scmd_init_clusters
 * turns sampling off. */
int scmd_set_sampling(scmd_ctx *ctx, int64_t every, int capacity);

/* Samples of one cluster held in the buffer, oldest first: *n_out = number
 * written (<= max_samples and <= capacity), out[5 s + 0..4] = { step,
 * E_pot (eV), E_kin (eV), T (K), T_target (K, 0 without a thermostat) }.
 * *recorded (may be NULL) = samples taken since the last
 * scmd_set_sampling.  When more are held than max_samples, the newest
 * max_samples are written. */
int scmd_get_samples(scmd_ctx *ctx, int cluster, double *out, int max_samples, int *n_out, int64_t *recorded);

/* Copy current state to host arrays of offsets[n_clusters] x 3 doubles
 * (density: offsets[n_clusters] doubles), caller-owned, row-major x y z.
 * Velocities include any pending thermostat factor.  Forces (eV/A, -grad U of
 * Sec. 2.1 Eq. (SC)) and density (rho_i of Eq. (rho), dimensionless) are
 * those of the current positions (valid after scmd_compute or scmd_step,
 * else SCMD_ESTATE). */
int scmd_get_positions(scmd_ctx *ctx, double *out);
int scmd_get_velocities(scmd_ctx *ctx, double *out);
int scmd_get_forces(scmd_ctx *ctx, double *out);
int scmd_get_density(scmd_ctx *ctx, double *out);

/* Device variant: write the forces (n x 3 doubles, row-major) into caller
 * device memory dev_out, ordered on the context stream; does not wait. */
int scmd_get_forces_device(scmd_ctx *ctx, double *dev_out);

/* Pair-distance histogram behind the radial distribution function
 * g(r) = rho(r) / rho_bar of one cluster at its current positions (Sec. 3,
 * "Radial distribution function as an indicator of the phase transition",
 * Eq. (Rdist)).  Reference atoms: those closer than r_select (A) to the
 * cluster's centre of mass (every atom when r_select <= 0).  Each pair of a
 * reference atom i and another atom j of the cluster adds 1 to bin
 * floor(r_ij / dr) when that is below nbins, r_ij = sqrt(dx*dx + dy*dy +
 * dz*dz) with d = r_i - r_j evaluated in IEEE double without contraction.
 * counts[nbins] (host) and *n_ref receive the counts and the number of
 * reference atoms by ADDING to what they hold, so that frames accumulate
 * (clear them first).  g of bin b is counts[b] / (n_ref * rho_bar * 4 pi
 * ((b+1)^3 - b^3) dr^3 / 3).  dr > 0, 1 <= nbins <= 32768.  Synchronises
 * the context stream.  The centre of mass is summed in a fixed tree order:
 * an atom within rounding of the r_select sphere may be classed either way. */
int scmd_rdf(scmd_ctx *ctx, int cluster, double r_select, double dr, int nbins, uint64_t *counts,
             int64_t *n_ref);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): scmd_rdf without any allocation and without
 * waiting.  The histogram of the cluster's current positions, defined as for
 * scmd_rdf, is ADDED on the context stream to dev_counts[nbins] (caller
 * device memory, uint64) and the number of reference atoms to *dev_n_ref
 * (caller device memory, int64); the call returns once the work is enqueued
 * and the caller synchronises (e.g. scmd_synchronize) before reading.  The
 * reference-atom list lives in a fixed device array of the library (4 MiB +
 * 256 bytes per GPU, held until the process ends) shared by every context on
 * that GPU: clusters above 1,048,576 atoms return SCMD_EINVAL, and calls that
 * overlap on one GPU (other streams, other threads) race on that array.
 * Other errors as scmd_rdf; device pointers are not checked. */
int scmd_rdf_noalloc(scmd_ctx *ctx, int cluster, double r_select, double dr, int nbins, uint64_t *dev_counts,
                     int64_t *dev_n_ref);

/* Frames for the self-diffusion coefficient (Sec. 3, "Diffusion coefficient
 * as a fingerprint of solidification phase transition").  scmd_set_frames
 * gives cluster `cluster` a device store that keeps its last `capacity`
 * frames (positions; 32 bytes per atom and frame), replacing and clearing any
 * store it had; capacity = 0 removes the store.  SCMD_ENOMEM when the store
 * cannot be allocated.  scmd_init_clusters removes every store. */
int scmd_set_frames(scmd_ctx *ctx, int cluster, int capacity);

/* Append the current positions of every cluster that has a frame store
 * (enqueued on the context stream; does not wait).  Frames are numbered from
 * 0 in the order recorded since the store was set. */
int scmd_record_frame(scmd_ctx *ctx);

/* Frames recorded into the cluster's store since it was set (SCMD_EINVAL if
 * the cluster has no store). */
int scmd_get_frame_count(scmd_ctx *ctx, int cluster, int64_t *recorded);

/* Self-diffusion coefficient D = <dr^2> / (2 z dt), z = 3 (Sec. 3,
 * Eq. (diffusion)), of the atoms of one cluster that lie closer than `radius`
 * (A) to the centre of mass of frame `first`, from the frames [first, first +
 * nframes) recorded frame_dt_ps apart (all still held by the store).  Every
 * frame of the window is first moved onto frame `first` by the proper
 * rotation and translation that minimise the summed squared displacement of
 * all the cluster's atoms (the paper removes the cluster's overall motion
 * this way); the window is cut into `segments` consecutive runs of
 * floor(nframes / segments) >= 2 frames (trailing frames unused), dr is a
 * central atom's displacement between the first and the last frame of a run
 * and dt the time between them; D (A^2/ps; 1 A^2/ps = 1e-4 cm^2/s) is the
 * mean over the central atoms and the runs, *n_central their number.
 * Synchronises the context stream.  SCMD_EINVAL for a bad window, radius or
 * dt, or when no atom is within radius (outputs then untouched).  An atom
 * within rounding of the radius sphere may be classed either way. */
int scmd_diffusion(scmd_ctx *ctx, int cluster, int64_t first, int nframes, double frame_dt_ps, double radius,
                   int segments, double *D_A2_per_ps, int64_t *n_central);

/* Checkpoint: scmd_get_state writes a self-describing blob (positions,
 * velocities, forces, thermostat factors and settings, step counts, and for
 * the cell list the positions of its last rebuild) into buf of *bytes
 * capacity; with buf NULL it only stores the needed size in *bytes.
 * scmd_set_state restores a blob taken from a context with the same cluster
 * layout (for the cell list it also rebuilds the cells and lists from those
 * positions, so the potential and integrator must be set for that); stepping
 * on from it reproduces the uninterrupted run bit for bit. */
int scmd_get_state(scmd_ctx *ctx, void *buf, size_t *bytes);
int scmd_set_state(scmd_ctx *ctx, const void *buf, size_t bytes);

/* Record device time per launch of the pair sweeps during subsequent
 * scmd_step / scmd_compute calls: HIP events on the context stream around
 * every eager launch (scmd_compute, the first force evaluation of a run),
 * and inside each captured graph (the 32-step graph and the graph of a run's
 * remainder) around the sweeps of its second-to-last step (event nodes
 * between graph kernels cost a few microseconds, so a graph is sampled once
 * per replay; the sample of its last replay in each scmd_step call is kept).
 * Changing the setting re-captures the graphs; enable = 0 stops recording;
 * every call resets the averages. */
int scmd_set_profiling(scmd_ctx *ctx, int enable);

/* Average device milliseconds per launch of a kernel class over the launches
 * recorded since profiling was enabled, and how many launches that covers. */
int scmd_get_kernel_time(scmd_ctx *ctx, int kernel, double *avg_ms, int64_t *launches);

/* Last error message of this context (or of the last failed scmd_create when
 * ctx is NULL).  The string stays valid until the next call on the context. */
const char *scmd_last_error(const scmd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* SCMD_H */
