/*
 * gpr_oracle.h -- FP64 CPU oracle of the Gen.ParRep hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct reference that
 * the GPU library is checked against.  It shares no code with the GPU library (its own
 * declarations, its own arithmetic) and may only be used by the tests, by the smoke check
 * and by the CPU-baseline leg of the benchmark.  The product path never calls it.
 *
 * What it computes (arXiv 1807.02431):
 *   - Langevin dynamics, Sec. 2.1 Eq. 1, discretised with the BAOAB splitting;
 *   - states and exits, Sec. 2.2; the Gen.ParRep loop of Sec. 2.4 (Fig. 1):
 *     transient propagation, Fleming-Viot convergence step with the Gelman-Rubin
 *     diagnostic (Sec. 2.4.1, Eqs. 2-4 and the clock updates that follow them), and the
 *     parallel dynamics step (Sec. 2.4.2, Eqs. 5-6);
 *   - the force field the MD engine must provide (Sec. 3.2): bonds, angles, torsions,
 *     position restraints, Lennard-Jones, Coulomb (vacuum, or reaction field with a cutoff).
 * Every sum over pairs is a brute-force double loop; nothing is cached between steps
 * except the forces at the current positions.
 */
#ifndef GPR_ORACLE_H
#define GPR_ORACLE_H
#include <stdint.h>

#define GRO_OK 0
#define GRO_BUDGET 1
#define GRO_EINVAL (-1)
#define GRO_ENOMEM (-2)
#define GRO_EPHASE (-4)
#define GRO_EUNSTABLE (-5)

#define GRO_TOY2D 1
#define GRO_MOLECULAR 2

#define GRO_STATE_SIGN_X 1
#define GRO_STATE_DIHEDRAL_BOXES 2
#define GRO_STATE_COM_SPHERE 3

#define GRO_OBS_COORD 1
#define GRO_OBS_POTENTIAL 2
#define GRO_OBS_KINETIC 3
#define GRO_OBS_DIHEDRAL 4
#define GRO_OBS_COM_DISTANCE 5
#define GRO_OBS_RMS_VELOCITY 6

#define GRO_NMAXOBS 8
#define GRO_NMAXBOX 8

typedef struct {
    int32_t kind;
    int32_t atoms[8];
    int32_t n_boxes;
    double box[GRO_NMAXBOX][4];
    int32_t n_group;
    const int32_t *group;
    double center[3];
    double radius;
} gro_state_spec;

typedef struct {
    int32_t kind;
    int32_t atoms[4];
    int32_t n_a;
    const int32_t *group_a;
    int32_t n_b;
    const int32_t *group_b;
} gro_obs_spec;

typedef struct {
    int32_t kind, n_atoms, n_replicas;
    const double *mass, *pos, *vel;
    const double *sigma, *epsilon, *charge;
    double cutoff, eps_rf, skin;
    int32_t nlist_period;
    int32_t n_bonds;      const int32_t *bond_atoms;    const double *bond_r0, *bond_k;
    int32_t n_angles;     const int32_t *angle_atoms;   const double *angle_theta0, *angle_k;
    int32_t n_torsions;   const int32_t *torsion_atoms; const int32_t *torsion_n;
                          const double *torsion_k, *torsion_phi0;
    int32_t n_restraints; const int32_t *restraint_atom; const double *restraint_ref, *restraint_k;
    int32_t n_pairs14;    const int32_t *pair14_atoms;  double scale14;
    int32_t n_exclusions; const int32_t *exclusion_atoms;
    double kT, gamma, dt;
    uint64_t seed;
    int32_t t_gr, t_check_dephase, t_check_parallel;
    double tol;
    int64_t t_min;
    gro_state_spec state;
    int32_t n_obs;
    const gro_obs_spec *obs;
} gro_spec;

typedef struct gro_sys gro_sys;

typedef struct { int32_t kind, from_state, to_state, pad; int64_t resident_steps, steps_taken; } gro_event;
typedef struct { int32_t outcome, to_state; int64_t t_steps, n_branch, n_samples; double rhat[GRO_NMAXOBS]; } gro_dephase_result;
typedef struct { int64_t M; int32_t k, to_state; int64_t tau_steps; double tau; } gro_exit_result;

int  gro_create(const gro_spec *spec, gro_sys **out);
void gro_destroy(gro_sys *S);
const char *gro_error(void);

/* potential energy and forces at arbitrary positions q[3][n] (SoA) */
int  gro_eval(const gro_sys *S, const double *q, double *F, double *U);
/* dU/d(eps_i, sigma_i, q_i, torsion k_t) at positions q[3][n] (molecular systems, eps_i > 0) */
int  gro_param_grad(const gro_sys *S, const double *q, double *dU_eps, double *dU_sig, double *dU_q, double *dU_k);
int  gro_energy_forces(const gro_sys *S, int32_t r0, int32_t nr, double *E, double *F);
int  gro_decorrelate(gro_sys *S, int64_t t_corr, int64_t max_steps, gro_event *ev);
int  gro_dephase(gro_sys *S, int64_t max_steps, gro_dephase_result *o);
int  gro_dephase_fixed(gro_sys *S, int64_t t_phase, int64_t max_steps, gro_dephase_result *o);
int  gro_parallel_step(gro_sys *S, int64_t max_checks, gro_exit_result *o);
int  gro_advance(gro_sys *S, int64_t nsteps, int64_t *first_exit_check);
int  gro_step_replicas(gro_sys *S, int64_t nsteps, int32_t r_lo, int32_t r_hi);
double  gro_simulated_time(const gro_sys *S);
int64_t gro_simulated_steps(const gro_sys *S);
int64_t gro_global_step(const gro_sys *S);
int32_t gro_current_state(const gro_sys *S);
int  gro_get_state(const gro_sys *S, int32_t r, double *q, double *v);
int  gro_set_state(gro_sys *S, int32_t r, const double *q, const double *v);
int  gro_get_accumulators(const gro_sys *S, int64_t *n, double *S1, double *S2, double *shift);
int  gro_observe(const gro_sys *S, double *obs, int32_t *state);
/* state id and observables of an arbitrary configuration */
int32_t gro_state_of(const gro_sys *S, const double *q);
int  gro_observables_of(const gro_sys *S, const double *q, const double *v, double U, double *out);

/* building blocks */
void gro_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void gro_noise(uint64_t seed, int32_t replica, int64_t step, int32_t stream, int32_t n_atoms,
               uint32_t *words, double *gauss);
int  gro_fv_plan(uint64_t seed, int64_t step, int32_t R, const uint8_t *exited, int32_t *donor);
int  gro_rhat(int32_t nw, int32_t n_obs, int64_t n, const double *S1, const double *S2, double *rhat);
int  gro_exit_vote(int32_t R, const int64_t *first_exit_check, int64_t t_check,
                   int64_t *M, int32_t *k, int64_t *tau_steps);
#endif
