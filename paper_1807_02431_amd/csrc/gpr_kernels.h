// gpr_kernels.h -- kernel entry points of the Gen.ParRep hot path (launched by gpr_api.hip).
#pragma once
#include "gpr_device.h"

namespace gpr {

enum { CHK_STATE = 0, CHK_DEPHASE = 1, CHK_PARALLEL = 2, CHK_ADVANCE = 3 };

// per-check status word read back by the host
struct Status {
    int mode;
    int ref_exited;     // dephasing: the reference walker left Omega
    int n_exited;       // dephasing: workers that left Omega at this check
    int n_surv;         // dephasing: surviving workers
    int k;              // parallel step: 1-based index of the first exiting replica, 0 if none
    int to_state;       // state of replica 0 (or of replica k-1 in the parallel step)
    int err[4];
    long long M;        // parallel step: check index of the first exit (Eq. 5), 0 if none
    long long tau;      // parallel step: (R (M - 1) + k) t_check steps (Eq. 5)
    double rhat[MAX_OBS];
};

// Device record of a captured run of check cycles (a persistent launch, then the check):
// cycle j of a replay steps from s_start + j nsteps (local step t_start + j nsteps) and takes
// check index M_start + j + 1; the check that ends the call records its cycle in halt_cycle,
// and every later kernel of the replay returns at once.  nsamp: observable samples so far.
struct CycRec {
    long long s_start, t_start, M_start, nsamp;
    int nsteps, halt_cycle;
    int omega;          // the state the checks compare with
    int pad;
};
constexpr int NO_HALT = 0x7FFFFFFF;

// Phase timers of the persistent body (a build with GPR_PHASE_PROBE only): the slots of one
// (replica, group): clock ticks spent in each phase, the counts of steps and rebuilds (all
// summed over launches), then the clock at the start and at the end of its last launch.
enum { PH_PROLOGUE = 0, PH_INTEGRATE, PH_EXCHANGE, PH_REBUILD, PH_FORCES, PH_TAIL, PH_EPILOGUE, PH_NSTEP, PH_NREBUILD,
       PH_START, PH_END, NPHASE };
constexpr int PHASE_MAX_R = 4096, PHASE_MAX_G = 8;
// Host side: copies the slots of replicas [0, R) ([R][PHASE_MAX_G][NPHASE]) to out and clears
// them, on the stream; hipErrorNotSupported in a build without the timers.
hipError_t phase_take(unsigned long long *out, int R, hipStream_t st);

// atom ranges of the workgroups of one replica on the persistent path
struct Split {
    int G;          // workgroups per replica (1, 2, 4 or 8)
    int lmax;       // LDS length of the per-group arrays: the largest range, rounded up to 16
    int bnd[9];     // group g owns atoms [bnd[g], bnd[g + 1]); every bnd[g] < n is a multiple of 16
};

__global__ void k_set_clock(const Dev *__restrict__ Sp, long long s, long long t);
__global__ void k_tick(const Dev *__restrict__ Sp, long long n);
__global__ void k_integrate(const Dev *__restrict__ Sp, long long s, int r_off, int energy);
__global__ void k_bonded(const Dev *__restrict__ Sp, long long s, int r_off, int energy);
__global__ void k_nonbonded(const Dev *__restrict__ Sp, long long s, int r_off, int energy, int apply_b, int force_build);
__global__ void k_obs(const Dev *__restrict__ Sp, int r_off, int mode, double *out, int k);
__global__ void k_state(const Dev *__restrict__ Sp, int r_off);
// one system's share of a persistent launch (see k_persist)
struct PersistItem {
    const Dev *dev;     // device descriptor of the system
    Split sp;           // atom ranges of the workgroups of a replica
    long long s0;       // global step counter at the first step
    int nsteps, t0;     // steps of this launch; steps already taken in the current call
    int sample;         // accumulate worker observables every t_GR steps (t counted from t0)
    int state_end;      // write each replica's state id at the end
    int nrep;           // replicas of the system
    int nsets;          // sets of sp.G workgroups that share the replicas
    int roff;           // k_persist: set k takes replica roff + k
    int boff;           // first workgroup of the item in the grid
    int xcd;            // map a set's workgroups to one XCD (nsets and boff multiples of 8)
    const CycRec *cyc;  // non-null: cycle `cycle` of a captured run (s0 and t0 from the record)
    int cycle;
};
constexpr int MAX_BATCH = 8;
struct PersistBatch {
    int nitems;
    PersistItem it[MAX_BATCH];
};

// Work items of persistent launches: an item is a system whose replicas are shared by nsets
// sets of sp.G workgroups.  Workgroup `local` of the item (counted from boff) is group g of set
// `set`.  With xcd set (nsets a multiple of 8) the workgroups of a set have equal blockIdx mod
// 8, which under the round-robin dispatch of workgroups to XCDs puts them on one XCD, for L2
// locality only: what they exchange is device-coherent.  Host code checks every launch's
// layout with it.
__host__ __device__ inline bool persist_place(const PersistItem &it, int local, int &set, int &g)
{
    const int G = it.sp.G;
    if (local < 0 || local >= it.nsets * G) return false;
    if (G == 1) {
        set = local; g = 0;
    } else if (it.xcd) {
        const int x = local % 8, slot = local / 8;
        set = (slot / G) * 8 + x;
        g = slot % G;
    } else {
        set = local / G; g = local % G;
    }
    return true;
}

__global__ void k_persist(PersistItem it);
__global__ void k_persist_batch(PersistBatch pb);
__global__ void k_grad_nb(const Dev *__restrict__ Sp, const double *w);
__global__ void k_grad_terms(const Dev *__restrict__ Sp, const double *w);
__global__ void k_grad_finish(const Dev *__restrict__ Sp, double *d_eps, double *d_sigma, double *d_charge, double *d_tk);
__global__ void k_unfix_out(const Dev *__restrict__ Sp, double *energy, float *forces);
__global__ void k_weighted_dx(const Dev *__restrict__ Sp, const double *w, float *dx);
__global__ void k_check(const Dev *__restrict__ Sp, int mode, long long s, int omega, int nrep, long long nsamp,
                        long long check_index, long long t_check, Status *st, int *donor, int *surv, long long *fec,
                        CycRec *cyc, int cycle);
__global__ void k_clone(const Dev *__restrict__ Sp, const int *donor, int acc_mode);
__global__ void k_init_vel(const Dev *__restrict__ Sp, float kT);
__global__ void k_noise_test(uint32_t k0, uint32_t k1, int replica, long long step, int stream, int n,
                             uint32_t *words, float *gauss);
__global__ void k_fvplan_test(uint32_t k0, uint32_t k1, long long s, int R, const uint8_t *exited, int *donor, int *surv);
__global__ void k_rhat_test(int nw, int nobs, long long n, const double *S1, const double *S2, double *out);
__global__ void k_vote_test(int R, const long long *fec, long long t_check, long long *out);

} // namespace gpr
