/*
 * gpr.h -- C ABI of the MI355X Generalized Parallel Replica (Gen.ParRep) hot path.
 *
 * The method (Generalized Parallel Replica dynamics as implemented in gen.parRep,
 * arXiv 1807.02431): many replicas of one molecular system follow underdamped Langevin dynamics (Sec. 2.1,
 * Eq. 1); a reference walker first reaches and resides in a metastable state Omega
 * (transient propagation, Sec. 2.4 step 1); a Fleming-Viot particle process dephases the
 * other replicas until the Gelman-Rubin statistic of every observable is below 1+TOL
 * (Sec. 2.4.1, Eqs. 2-4); then all replicas run in parallel until the first exit, whose
 * time is assembled from the check count and replica index (Sec. 2.4.2, Eqs. 5-6).
 *
 * Every entry point is extern "C", takes plain pointers and sizes and returns a
 * gpr_status (except the few documented otherwise).  Nothing aborts or throws across the
 * boundary.  On error the outputs are left untouched and gpr_last_error() describes the
 * failure.  Host pointers are read or written only during the call; the caller keeps
 * ownership of every buffer it passes.  A gpr_system handle is not thread-safe: all calls
 * on one handle are serialised on the HIP stream set with gpr_set_stream (default: the
 * null stream) and return only after that stream has finished the call's work.
 *
 * Units for molecular systems: nm, ps, amu, kJ/mol, elementary charge.  The toy system
 * is dimensionless.  Time is counted in integer steps of dt; the clock t_sim is the
 * integer step count times dt.
 */
#ifndef GPR_H
#define GPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
typedef int32_t gpr_status;
#define GPR_OK          0   /* success */
#define GPR_BUDGET      1   /* step/check budget exhausted; the call is resumable, state kept */
#define GPR_EINVAL    (-1)  /* invalid argument or descriptor */
#define GPR_ENOMEM    (-2)  /* device or host allocation failed */
#define GPR_EDEVICE   (-3)  /* HIP runtime error, missing device, or an in-kernel capacity limit */
#define GPR_EPHASE    (-4)  /* call out of sequence (e.g. gpr_parallel_step before a converged gpr_dephase) */
#define GPR_EUNSTABLE (-5)  /* a non-finite position or velocity, or a force component beyond
                                 2.5e5 kJ/mol/nm, appeared */

/* ---------------------------------------------------------------- system kinds */
#define GPR_KIND_TOY2D      1  /* one particle in U(x,y) = (x^2-1)^2 + 2 y^2; z and v_z held at 0 */
#define GPR_KIND_MOLECULAR  2  /* bonded + Lennard-Jones + Coulomb force field */

/* ---------------------------------------------------------------- state functions (Sec. 2.2)
 * A state function maps a configuration q to an integer state id >= 0, or -1 when q lies
 * in no state (the states need not partition configuration space; Sec. 2.2).  An exit
 * from Omega is observed at a check when state(q) != Omega (Sec. 2.4.2). */
#define GPR_STATE_SIGN_X          1  /* id = (x[atoms[0]] >= 0) ? 1 : 0 */
#define GPR_STATE_DIHEDRAL_BOXES  2  /* phi = dihedral(atoms[0..3]), psi = dihedral(atoms[4..7]);
                                        id = first b with box[b][0] < phi <= box[b][1] and
                                        box[b][2] < psi <= box[b][3]; -1 if none */
#define GPR_STATE_COM_SPHERE      3  /* id = (|COM(group) - center| < radius) ? 1 : 0 (COM mass-weighted) */

#define GPR_MAX_BOXES 8
#define GPR_MAX_OBS   8

typedef struct gpr_state_desc {
    int32_t kind;
    int32_t atoms[8];
    int32_t n_boxes;
    double  box[GPR_MAX_BOXES][4];   /* (phi_lo, phi_hi, psi_lo, psi_hi), radians, half-open (lo, hi] */
    int32_t n_group;
    const int32_t *group;            /* [n_group] atom indices */
    double  center[3];
    double  radius;
} gpr_state_desc;

/* ---------------------------------------------------------------- observables (Sec. 2.4.1, Eq. 2)
 * Real-valued functions of (q, p) whose trajectory averages feed the Gelman-Rubin test. */
#define GPR_OBS_COORD        1  /* coordinate atoms[1] (0=x,1=y,2=z) of atom atoms[0] */
#define GPR_OBS_POTENTIAL    2  /* total potential energy V(q) */
#define GPR_OBS_KINETIC      3  /* kinetic energy K = 1/2 sum_i m_i |v_i|^2 */
#define GPR_OBS_DIHEDRAL     4  /* dihedral angle of atoms[0..3], radians in (-pi, pi] */
#define GPR_OBS_COM_DISTANCE 5  /* |COM(group_a) - COM(group_b)| (a one-atom group is that atom) */
#define GPR_OBS_RMS_VELOCITY 6  /* sqrt(mean over group_a of |v_i|^2) */

typedef struct gpr_obs_desc {
    int32_t kind;
    int32_t atoms[4];
    int32_t n_a;
    const int32_t *group_a;
    int32_t n_b;
    const int32_t *group_b;
} gpr_obs_desc;

/* ---------------------------------------------------------------- system descriptor
 * Force field (molecular kind):
 *   bond      1/2 k (r - r0)^2
 *   angle     1/2 k (theta - theta0)^2
 *   torsion   k (1 + cos(n phi - phi0)), phi the IUPAC dihedral (trans = pi), integer n in [0, 12]
 *   restraint 1/2 k |r - r_ref|^2
 *   nonbonded, every pair that is neither excluded nor listed as a 1-4 pair:
 *     Lennard-Jones 4 eps_ij ((s_ij/r)^12 - (s_ij/r)^6), s_ij = (s_i+s_j)/2, eps_ij = sqrt(eps_i eps_j)
 *     Coulomb f q_i q_j / r                                   (cutoff == 0: all pairs, vacuum)
 *     reaction field f q_i q_j (1/r + k_rf r^2 - c_rf), r < cutoff, zero beyond it, with
 *       k_rf = (eps_rf - 1) / ((2 eps_rf + 1) cutoff^3), c_rf = 1/cutoff + k_rf cutoff^2
 *     f = 138.935458 kJ mol^-1 nm e^-2; Lennard-Jones is truncated at the cutoff without shift
 *   1-4 pairs: scale14 * (Lennard-Jones + vacuum Coulomb), never cut off
 *   excluded pairs contribute nothing.
 * Dynamics: BAOAB splitting of Langevin dynamics (Eq. 1) with friction rate gamma (1/time):
 *   B v += dt/2 F/m; A x += dt/2 v; O v = c1 v + sqrt((1-c1^2) kT/m) xi, c1 = exp(-gamma dt);
 *   A x += dt/2 v; F = F(x); B v += dt/2 F/m.
 * Noise xi: Philox4x32-10 (Salmon et al., SC'11), key = (seed lo, seed hi), counter =
 *   (atom, step lo 32 bits, replica, stream << 24 | step hi 24 bits); uniforms
 *   u_k = (2 (w_k >> 9) + 1) 2^-24; Box-Muller z0,z1 from (u0,u1), z2 from (u2,u3)
 *   (z = sqrt(-2 ln u_a) cos/sin(2 pi u_b)); (xi_x, xi_y, xi_z) = (z0, z1, z2).
 *   Streams: 0 = Langevin noise, 1 = initial velocities, 2 = Fleming-Viot donor draws.
 *   "step" is the system's global step counter s, advanced by one for every BAOAB step
 *   applied to the set of replicas that is running.
 */
typedef struct gpr_system_desc {
    int32_t kind;
    int32_t n_atoms;             /* >= 1; the pair kernels hold a replica's positions and LJ
                                    parameters in LDS (24 bytes per atom), so creation fails with
                                    EINVAL past about 6,500 atoms on a 160 KiB-LDS device; the
                                    persistent path, which also keeps its own atoms' velocities
                                    and forces in LDS, takes up to about 4,600 atoms (8 workgroups
                                    per replica; gpr_set_path reports EINVAL beyond) */
    int32_t n_replicas;          /* 2 <= R <= 4096 (replica 0 is the reference walker); the check kernel
                                    keeps one survivor index per replica in LDS */

    const double *mass;          /* [n_atoms], amu (> 0) */
    const double *pos;           /* [3][n_atoms] SoA, nm: x[0..n), y[0..n), z[0..n) */
    const double *vel;           /* [3][n_atoms] SoA, or NULL: Maxwell-Boltzmann draw (stream 1, replica 0, step 0) */

    const double *sigma;         /* [n_atoms] nm (molecular only) */
    const double *epsilon;       /* [n_atoms] kJ/mol */
    const double *charge;        /* [n_atoms] e */

    double  cutoff;              /* 0 = all pairs with vacuum Coulomb; > 0 = cutoff with reaction field */
    double  eps_rf;              /* reaction-field dielectric (cutoff > 0) */
    double  skin;                /* pair-list skin (nm), cutoff > 0 */
    int32_t nlist_period;        /* pair lists are at most this many steps old (persistent path: per replica;
                                    plain path: on the steps s with s+1 a multiple of it, for all replicas);
                                    rebuilt earlier when an atom has moved more than skin/2 since the last
                                    build.  Results do not depend on when lists are rebuilt. */

    int32_t n_bonds;     const int32_t *bond_atoms;     const double *bond_r0;      const double *bond_k;
    int32_t n_angles;    const int32_t *angle_atoms;    const double *angle_theta0; const double *angle_k;
    int32_t n_torsions;  const int32_t *torsion_atoms;  const int32_t *torsion_n;   const double *torsion_k;
                         const double *torsion_phi0;
    int32_t n_restraints; const int32_t *restraint_atom; const double *restraint_ref; /* [n][3] */
                         const double *restraint_k;
    int32_t n_pairs14;   const int32_t *pair14_atoms;   double scale14;
    int32_t n_exclusions; const int32_t *exclusion_atoms;   /* [n][2]; 1-4 pairs need not be repeated here */

    double  kT;                  /* k_B T (kJ/mol, or 1/beta for the toy) */
    double  gamma;               /* friction rate, 1/time */
    double  dt;                  /* time step */
    uint64_t seed;               /* Philox key */

    int32_t t_gr;                /* observable sampling period (steps), Sec. 2.4.1 */
    int32_t t_check_dephase;     /* exit-test period in transient and convergence steps */
    int32_t t_check_parallel;    /* exit-test period in the parallel step, Eq. 5 */
    double  tol;                 /* Gelman-Rubin tolerance, Eq. 4 */
    int64_t t_min;               /* floor on t_FV in steps (0 = none) */

    gpr_state_desc state;
    int32_t n_obs;               /* <= GPR_MAX_OBS */
    const gpr_obs_desc *obs;
} gpr_system_desc;

typedef struct gpr_system gpr_system;   /* opaque, library-owned */

/* ---------------------------------------------------------------- outputs */
#define GPR_EV_RESIDENT 0
#define GPR_EV_EXITED   1
typedef struct gpr_event {
    int32_t kind;            /* GPR_EV_RESIDENT or GPR_EV_EXITED */
    int32_t from_state;      /* Omega on entry (-1 if the walker started in no state) */
    int32_t to_state;        /* the state now held as Omega */
    int32_t pad;
    int64_t resident_steps;  /* steps spent in from_state during this call, up to the deciding check */
    int64_t steps_taken;     /* steps of replica 0 in this call (all added to t_sim) */
} gpr_event;

#define GPR_DEPHASE_CONVERGED  0
#define GPR_DEPHASE_REF_EXITED 1
typedef struct gpr_dephase_out {
    int32_t outcome;         /* GPR_DEPHASE_CONVERGED or GPR_DEPHASE_REF_EXITED */
    int32_t to_state;        /* reference walker's state at the deciding check */
    int64_t t_steps;         /* t_FV (converged) or t_ref (reference exit), in steps */
    int64_t n_branch;        /* Fleming-Viot branchings (worker kills) in this dephasing */
    int64_t n_samples;       /* observable samples per worker */
    double  rhat[GPR_MAX_OBS];
} gpr_dephase_out;

typedef struct gpr_exit_out {
    int64_t M;               /* number of checks until the first exit (Eq. 5) */
    int32_t k;               /* 1-based index of the exiting replica, smallest among ties */
    int32_t to_state;        /* state of replica k at the exit check */
    int64_t tau_steps;       /* (R (M-1) + k) t_check_parallel */
    double  tau;             /* tau_steps * dt */
} gpr_exit_out;

/* ---------------------------------------------------------------- lifecycle */
/* Validates d, copies every array, uploads to the current HIP device, builds the pair lists
 * and evaluates F(q0) for all replicas (all replicas start as copies of (pos, vel)).
 * On failure *out is set to NULL.  EINVAL for malformed descriptors.  Excluded and 1-4
 * pairs may join any two atoms (rings, branches): those less than 32 indices apart are held
 * as a bit mask per atom, the others in a sorted partner list per atom. */
gpr_status gpr_system_create(const gpr_system_desc *d, gpr_system **out);
void       gpr_system_destroy(gpr_system *sys);
/* Static-lifetime text of the last error on sys, or of the calling thread when sys is NULL. */
const char *gpr_last_error(const gpr_system *sys);

/* Sets the HIP stream (hipStream_t passed as void*) on which all later calls run. */
gpr_status gpr_set_stream(gpr_system *sys, void *hip_stream);

/* Stepping path: GPR_PATH_PLAIN launches separate kernels every step (list build every
 * nlist_period, BAOAB, bonded, nonbonded); GPR_PATH_PERSISTENT advances whole check
 * periods in one launch with the replica state held on chip.  Results are bit-identical.
 * EINVAL for the persistent path when no split of a replica over 1, 2, 4 or 8 workgroups fits
 * the device. */
#define GPR_PATH_PLAIN      0
#define GPR_PATH_PERSISTENT 1
gpr_status gpr_set_path(gpr_system *sys, int32_t path);
/* Launch shape of the persistent path: threads per workgroup (multiple of 64, <= 1024) and
 * workgroups per replica (1, 2, 4 or 8; a replica's atoms are split between its workgroups,
 * which exchange positions every step).  0 keeps the current value.  When the replicas times
 * the workgroups per replica exceed what the device holds at once, sets of workgroups take the
 * replicas in turn.  EINVAL, with nothing changed, if one workgroup's share of a replica does
 * not fit in LDS (large systems need several workgroups per replica) or a workgroup of that
 * size cannot run.  Results do not depend on the shape. */
gpr_status gpr_set_launch(gpr_system *sys, int32_t block_threads, int32_t groups_per_replica);

/* Plain path as replays of a HIP graph: with cycle_steps > 0 the plain path's launches of
 * cycle_steps steps are captured once (per replica count and sampling mode) and replayed;
 * the kernels then take the step counter and the sampling decision from device memory, so
 * every replay continues where the last one stopped, and the steps left over are launched
 * directly.  0 (the default) launches every step from the host.  Results are bit-identical
 * either way.  EINVAL outside [0, 10000]. */
gpr_status gpr_set_graph(gpr_system *sys, int32_t cycle_steps);

/* Autotuner of the persistent path's launch shape: every (threads per workgroup in {256, 512,
 * 768, 1024}, workgroups per replica in {1, 2, 4, 8}) that fits the device is timed over nsteps
 * steps from the same saved state, and the fastest becomes the launch shape (written to
 * *block_threads and *groups when not NULL).  The state is restored afterwards (every pair list
 * is rebuilt at the next step), so later results are those of a run without the call.  Device
 * scratch for one copy of the replicas' state is allocated and freed within the call.  EINVAL
 * if nsteps < 1 or the persistent path does not fit. */
gpr_status gpr_autotune(gpr_system *sys, int32_t nsteps, int32_t *block_threads, int32_t *groups);

/* ---------------------------------------------------------------- force field (Sec. 3.2) */
/* Energy and forces of replicas [r0, r0+nr) at their current positions.
 * energy: [nr] or NULL; forces: [nr][3][n_atoms] (SoA per replica) or NULL; host buffers.
 * Forces are the 64-bit fixed-point accumulators (2^-32 kJ/mol/nm) converted exactly. */
gpr_status gpr_energy_forces(gpr_system *sys, int32_t r0, int32_t nr, double *energy, double *forces);

/* ---------------------------------------------------------------- differentiation
 * The potential energy U_r(x_r; theta) of every replica as a function of its positions and of
 * the force-field parameters theta = (epsilon_i, sigma_i, charge_i per atom, k_t per torsion),
 * with the terms and combination rules of the descriptor (Sec. 3.2 engine requirement: V(q)
 * and its gradient).  dU/dx = -F comes with the forces; the parameter gradient is a second
 * pass over the same terms.  For callers whose tensors live on the GPU (an autograd binding):
 * *_dev pointers are device memory, written on the system's stream, and the call returns once
 * the stream has finished. */

/* Replaces epsilon, sigma, charge ([n_atoms], caller's atom order) and the torsion force
 * constants ([n_torsions], caller's torsion order); a NULL array keeps its current values.
 * Re-evaluates the forces of every replica at its current positions (the integrator carries
 * them from step to step).  Host buffers.  EINVAL for a toy system, epsilon or sigma < 0, or a
 * non-finite value (nothing is changed then).  Meant for use between the Gen.ParRep calls. */
gpr_status gpr_set_params(gpr_system *sys, const double *epsilon, const double *sigma, const double *charge,
                          const double *torsion_k);

/* Sets the positions of all replicas from x_dev (float, [n_replicas][3][n_atoms] SoA, device),
 * rebuilds their pair lists and writes energy_dev (double [n_replicas]) and forces_dev (float
 * [n_replicas][3][n_atoms]); either output may be NULL.  Velocities are kept.  EDEVICE if a pair
 * list overflows its capacity. */
gpr_status gpr_energy_forces_dev(gpr_system *sys, const float *x_dev, double *energy_dev, float *forces_dev);

/* Backward pass at the replicas' current positions, weighted by w_dev (double [n_replicas],
 * device): d_x[r] = w[r] dU_r/dx_r = -w[r] F_r (float [n_replicas][3][n_atoms]) and the
 * parameter gradient sum_r w[r] dU_r/dtheta into d_epsilon, d_sigma, d_charge (double
 * [n_atoms]) and d_torsion_k (double [n_torsions], caller's torsion order); device buffers, each
 * may be NULL.  Parameter sums are taken in 2^-32 fixed point, so they do not depend on the order
 * of the terms.  EINVAL for a toy system (when a parameter output is requested) or when an
 * epsilon is 0 and d_epsilon is requested (sqrt(eps_i eps_j) has no derivative there). */
gpr_status gpr_energy_backward_dev(gpr_system *sys, const double *w_dev, float *d_x, double *d_epsilon,
                                   double *d_sigma, double *d_charge, double *d_torsion_k);

/* ---------------------------------------------------------------- Gen.ParRep steps (Sec. 2.4) */
/* Transient propagation of the reference walker (replica 0), Sec. 2.4 step 1, followed by a
 * residence of t_corr_steps in the state reached.  Steps replica 0 with a state test every
 * t_check_dephase steps.  Returns GPR_OK with ev->kind = RESIDENT once the walker has stayed
 * t_corr_steps in a state (which becomes Omega), or EXITED when a check finds it in another
 * state than the one it was resident in (Omega becomes that state).  Every step taken is
 * added to t_sim.  GPR_BUDGET after max_steps steps without a decision (state kept). */
gpr_status gpr_decorrelate(gpr_system *sys, int64_t t_corr_steps, int64_t max_steps, gpr_event *ev);

/* Convergence step, Sec. 2.4.1: replica 0's (q, v, F) is copied into replicas 1..R-1 and the
 * observable accumulators are cleared; all replicas step; every t_gr steps the observables of
 * the workers (replicas >= 1) are accumulated; every t_check_dephase steps: (i) if replica 0
 * left Omega, t_sim += t_ref and outcome = REF_EXITED (Omega becomes its new state);
 * (ii) each exited worker, in increasing index, is replaced by a copy (q, v, F, accumulators)
 * of a survivor drawn uniformly (stream 2); with no survivor all workers are re-copied from
 * replica 0 and the accumulators cleared; (iii) if t >= t_min, at least 2 samples were taken
 * and every observable has R-hat < 1 + tol (Eq. 3, 4), t_sim += t_FV and outcome = CONVERGED.
 * GPR_BUDGET after max_steps steps in this call (the dephasing resumes on the next call). */
gpr_status gpr_dephase(gpr_system *sys, int64_t max_steps, gpr_dephase_out *o);

/* Dephasing of the original ParRep algorithm (Sec. 2.4.3), the step that Gen.ParRep replaces by
 * the Fleming-Viot process: all R replicas start from the reference walker's configuration and
 * a replica's sample is the state it has at the first check (every t_check_dephase steps) at
 * which it has stayed in Omega for t_phase steps since its last (re)start; a replica found
 * outside Omega at a check restarts from that start configuration.  When every replica has its
 * sample, all are set to their samples and gpr_parallel_step may follow.  The dephasing time
 * is not added to t_sim.  o->t_steps: steps taken, o->n_branch: restarts.  Resumable
 * (GPR_BUDGET after max_steps); EPHASE if the reference walker is in no state, EINVAL for
 * t_phase < 0. */
gpr_status gpr_dephase_fixed(gpr_system *sys, int64_t t_phase, int64_t max_steps, gpr_dephase_out *o);

/* Parallel dynamics step, Sec. 2.4.2: after a converged dephasing, all R replicas step
 * t_check_parallel steps between checks; at the first check M where some replica left Omega,
 * k = 1 + the smallest such index, tau = (R (M-1) + k) t_check_parallel (Eq. 5),
 * t_sim += tau (Eq. 6), replica 0 <- replica k-1 and Omega <- its state.  EPHASE unless the
 * last gpr_dephase converged.  GPR_BUDGET after max_checks checks (resumable). */
gpr_status gpr_parallel_step(gpr_system *sys, int64_t max_checks, gpr_exit_out *o);

/* Simulation clock t_sim = steps * dt (Sec. 2.4, Eq. 6).  NaN for a NULL handle. */
double  gpr_simulated_time(const gpr_system *sys);
/* Integer step count behind the clock; -1 for a NULL handle. */
int64_t gpr_simulated_steps(const gpr_system *sys);
/* Global noise step counter s; -1 for a NULL handle. */
int64_t gpr_global_step(const gpr_system *sys);
/* Current state Omega (-1 = none); INT32_MIN for a NULL handle. */
int32_t gpr_current_state(const gpr_system *sys);

/* Read/write access to X = (q, p) of one replica (Sec. 3.2 engine requirement), as
 * velocities v = p/m.  q, v: [3][n_atoms] host buffers (v may be NULL).  Setting a state
 * recomputes that replica's forces and returns the system to the idle phase; Omega is
 * left unchanged (the next check compares the new configuration with it). */
gpr_status gpr_get_state(const gpr_system *sys, int32_t r, double *q, double *v);
gpr_status gpr_set_state(gpr_system *sys, int32_t r, const double *q, const double *v);

/* Advances all replicas nsteps BAOAB steps, sampling the observables of replicas >= 1 every
 * t_gr steps and testing the state of every replica every t_check_dephase steps, with
 * nothing acted on: no branching, no phase change, clock unchanged.  The sampling and test
 * schedule runs on the steps taken by all gpr_advance / gpr_batch_advance calls on the
 * handle since creation, so that several short calls sample and test as one long call
 * does.  first_exit_check ([R] host int64, or NULL) receives, per replica, the index
 * (1-based, counted over all calls) of the first check within this call at which
 * state != Omega (0 if none); with NULL they are neither recorded nor read back.  The
 * fixed-work stepping loop of the measurement harness. */
gpr_status gpr_advance(gpr_system *sys, int64_t nsteps, int64_t *first_exit_check);

/* Steps taken by gpr_advance / gpr_batch_advance on the handle since creation (the position
 * in their sampling and check schedule); -1 for a NULL handle. */
int64_t gpr_advance_steps(const gpr_system *sys);

/* gpr_advance of several systems (1 to 8, each its own handle, all on one stream and able to
 * use the persistent path) whose persistent steps share launches: each launch advances every
 * system up to the next exit check of any of them (their t_check_dephase may differ), the
 * workgroups shared out in proportion to each system's work per step; sets of workgroups take
 * a system's replicas in turn when they do not all fit at once.  Per system the result is
 * bit-identical to gpr_advance.  first_exit_check: NULL, or nsys pointers (each NULL or
 * [n_replicas]).  EINVAL for a repeated handle, different streams, or more workgroups than
 * the device holds at once. */
gpr_status gpr_batch_advance(gpr_system *const *systems, int32_t nsys, int64_t nsteps,
                             int64_t *const *first_exit_check);

/* The Gen.ParRep calls of several systems with their persistent steps in shared launches.
 * ops[k] names the call to run on systems[k] (GPR_OP_DECORRELATE: gpr_decorrelate with t_corr and
 * max_steps; GPR_OP_DEPHASE: gpr_dephase with max_steps; GPR_OP_PARALLEL_STEP: gpr_parallel_step
 * with max_steps checks) and receives its status (GPR_OK with the result in event, dephase or
 * exit, GPR_BUDGET, or the error) and result.  Every launch advances each system that is still
 * running up to the next exit check of any of them, the systems at a check then take it, and
 * a system whose call is done waits for the others.  Per system every step, check, result and
 * clock reading is bit-identical to the single-system call.  Systems as in gpr_batch_advance
 * (1 to 8 distinct handles on one stream, each able to use the persistent path).  Returns
 * GPR_OK when every call finished with GPR_OK or GPR_BUDGET, else the first error (the other
 * systems' calls stop where they are). */
#define GPR_OP_DECORRELATE   0
#define GPR_OP_DEPHASE       1
#define GPR_OP_PARALLEL_STEP 2
typedef struct gpr_batch_op {
    int32_t op;              /* GPR_OP_* */
    int32_t status;          /* out */
    int64_t t_corr;          /* GPR_OP_DECORRELATE: residence time (steps) */
    int64_t max_steps;       /* budget: steps (decorrelate, dephase) or checks (parallel step) */
    gpr_event event;         /* out: GPR_OP_DECORRELATE */
    gpr_dephase_out dephase; /* out: GPR_OP_DEPHASE */
    gpr_exit_out exit;       /* out: GPR_OP_PARALLEL_STEP */
} gpr_batch_op;
gpr_status gpr_batch_run(gpr_system *const *systems, int32_t nsys, gpr_batch_op *ops);

/* Convergence and parallel steps on the persistent path as replays of a captured HIP graph of
 * `cycles` check cycles (0 = off, the default: one launch and one status read-back per check).
 * A cycle is the persistent launch of one check period, with the state test at its end, then
 * the check launch (Fleming-Viot clone-on-kill, R-hat, the exit vote and the decision whether
 * the call ends there); once a check ends the call, the rest of the replay does nothing.  The
 * host reads the statuses of a replay once and takes the same decisions as after a check it
 * runs itself, so results are bit-identical to cycles = 0.  A replay runs only from a check
 * boundary with room in the call's budget for all its cycles; other steps run as with
 * cycles = 0.  0 <= cycles <= 4096; EINVAL for a system too large for the persistent path.
 * Changing the launch shape (gpr_set_launch, gpr_autotune) discards the captured graphs. */
gpr_status gpr_set_cycles(gpr_system *sys, int32_t cycles);

/* Timing of the dominant stepping kernel (the persistent kernel on the persistent path,
 * the pair-force kernel on the plain path) with HIP events recorded on the system's
 * stream around each launch.  gpr_profile enables (1) or disables (0) recording and
 * clears the totals; gpr_profile_read waits for the stream and returns the summed
 * duration in ms and the number of launches timed since the last clear. */
gpr_status gpr_profile(gpr_system *sys, int32_t enable);
gpr_status gpr_profile_read(gpr_system *sys, double *ms, int64_t *launches);

/* Phase timers of the persistent kernel, for measurement: only the library's timer build
 * (libgpr_hip_probe.so, the same sources built with GPR_PHASE_PROBE) records them; the
 * product build returns GPR_EINVAL.  out ([R][8][11] doubles, host, caller-owned) receives per
 * replica r and workgroup g of its replica (rows g >= G stay 0): the microseconds spent since
 * the last read in the launch prologue (staging), the integrator (B A O A and the position
 * stores), the exchange (the other groups' positions), the pair-list rebuild, the forces
 * (bonded and pair terms), the step's tail (closing B, samples) and the epilogue (write back);
 * the number of steps and of pair-list rebuilds; then the start and the end of the group's
 * last launch, in microseconds after the earliest start among all groups.  The totals are
 * then cleared.  Waits for the system's stream.  Several systems advanced together share the
 * totals. */
gpr_status gpr_phase_read(gpr_system *sys, double *out);

/* Observable accumulators of replicas [0, R): n (samples) and, per replica r and observable
 * j, S1[r][j] = sum (O - c_j), S2[r][j] = sum (O - c_j)^2, shift[j] = c_j = O_j of replica 0
 * at dephasing start.  Host buffers, each may be NULL. */
gpr_status gpr_get_accumulators(const gpr_system *sys, int64_t *n, double *S1, double *S2, double *shift);

/* Current observables and state ids of all replicas: obs [R][n_obs], state [R]. */
gpr_status gpr_observe(gpr_system *sys, double *obs, int32_t *state);

/* ---------------------------------------------------------------- building blocks
 * Stateless device implementations of the reductions inside the steps above, exposed so
 * that their integer and FP64 results can be compared bit for bit.  Host buffers in/out. */

/* Philox4x32-10 words (stream, replicas, step, atoms as in the noise counter): out_words
 * [n_atoms][4] uint32 and out_gauss [n_atoms][3] float for one (replica, step, stream). */
gpr_status gpr_philox_noise(uint64_t seed, int32_t replica, int64_t step, int32_t stream,
                            int32_t n_atoms, uint32_t *out_words, float *out_gauss);

/* Fleming-Viot branching plan (Sec. 2.4.1 item 2): exited[R] flags of workers (entry 0, the
 * reference, is ignored); donor[R] receives for each exited worker the survivor it copies
 * (j = S[(u * |S|) >> 32], S the ascending survivor list, u the first Philox word of
 * counter (0, s lo, r, 2 << 24 | s hi)), -1 for others; -2 everywhere if no survivor. */
gpr_status gpr_fv_plan(uint64_t seed, int64_t step, int32_t R, const uint8_t *exited, int32_t *donor);

/* gpr_fv_plan for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same arguments and results, but
 * the exited flags, the survivor list and the donors are staged through one device array of
 * the library, sized for R <= GPR_NOALLOC_MAX_R, that every device the library runs on holds
 * until the process ends; the call allocates and frees no device memory.  EINVAL (nothing
 * done) for R beyond the limit.  Calls on one device share that array: calls that overlap on
 * a device (several host threads) race and must be serialised by the caller. */
#define GPR_NOALLOC_MAX_R 16384
gpr_status gpr_fv_plan_noalloc(uint64_t seed, int64_t step, int32_t R, const uint8_t *exited, int32_t *donor);

/* Gelman-Rubin statistic (Eq. 3) over nw workers from shifted sums: Ob_k = S1[k]/n,
 * num = mean_k(S2[k]/n) - (mean_k Ob_k)^2, den = mean_k(S2[k]/n - Ob_k^2), rhat = num/den
 * (+inf if den <= 0).  Means are pairwise sums over k on one canonical tree: the nw terms
 * padded with zeros to the next power of two, each node the sum of its lower and its upper
 * half; no FMA contraction.  The routine is the one the dephasing check runs.  S1, S2:
 * [nw][n_obs]; rhat: [n_obs]; 1 <= n_obs <= 64. */
gpr_status gpr_rhat(int32_t nw, int32_t n_obs, int64_t n, const double *S1, const double *S2, double *rhat);

/* Parallel-step vote (Eq. 5): first_exit_check[R] (0 = no exit yet, else 1-based check
 * index); M = min over nonzero entries, k = 1 + smallest r attaining M, tau_steps =
 * (R (M-1) + k) t_check.  GPR_BUDGET (outputs untouched) if no replica exited. */
gpr_status gpr_exit_vote(int32_t R, const int64_t *first_exit_check, int64_t t_check,
                         int64_t *M, int32_t *k, int64_t *tau_steps);

#ifdef __cplusplus
}
#endif
#endif /* GPR_H */
