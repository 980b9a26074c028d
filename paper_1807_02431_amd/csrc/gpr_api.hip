// gpr_api.hip -- host runtime behind the C ABI of include/gpr.h.
//
// Owns the device buffers of a system, drives the stepping paths and the per-check
// bookkeeping kernels, and keeps the Gen.ParRep phase machine (transient propagation,
// Fleming-Viot convergence step, parallel step; Sec. 2.4, Fig. 1) on the host: every
// decision is taken from a small status word read back once per check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gpr.h"
#include "gpr_kernels.h"

using namespace gpr;

namespace {

constexpr double COULOMB_F = 138.935458;
enum { PH_IDLE = 0, PH_DECORR = 1, PH_DEPHASE = 2, PH_CONVERGED = 3, PH_PARALLEL = 4, PH_DEPHASE_FIXED = 5 };

thread_local std::string g_thread_err;

} // namespace

struct gpr_system {
    Dev d{};
    Dev *d_dev = nullptr;     // device copy of d, passed to every kernel
    std::vector<void *> bufs;
    hipStream_t stream = nullptr;
    int path = GPR_PATH_PLAIN;
    int bt_persist = 0;
    int groups = 1;            // workgroups per replica on the persistent path
    Split split{};             // their atom ranges
    std::vector<double> work;  // per-atom work estimate that places the ranges
    // force-field parameters as the caller gave them (gpr_set_params rewrites the device copies)
    std::vector<double> mass_h, eps_h, sig_h, q_h, tor_k_h, tor_phi0_h;
    std::vector<int> tor_n_h, tor_order, p14_order;   // sorted term -> caller's index
    std::vector<int2> p14_h;
    double scale14 = 0.0;
    int max_coresident = 0;    // persistent-kernel workgroups that fit on the device at once
    int cap_bt = -1;           // persist_capacity: the launch shape last asked for and its capacity
    size_t cap_lds = 0;
    int cap_blocks = 0;
    int n = 0, R = 0, np = 0, kind = 0, nobs = 0;
    int t_gr = 1, tcd = 1, tcp = 1;
    double tol = 0, dt = 0, kT = 0;
    long long t_min = 0;
    // phase machine
    long long s = 0, tsim = 0;
    int omega = -1, phase = PH_IDLE;
    int dc_from = -1, dc_omega = -1;
    long long dc_resid = 0, dc_steps = 0;
    long long dp_t = 0, nsamp = 0, n_branch = 0;
    long long adv_t = 0;       // steps taken by gpr_advance / gpr_batch_advance: their sampling and check phase
    long long par_M = 0, par_t = 0;   // parallel step: checks done, steps into the current check period
    // original ParRep dephasing: start configuration, samples, per-replica progress
    float *snap_x = nullptr, *snap_v = nullptr, *samp_x = nullptr, *samp_v = nullptr;
    long long *snap_F = nullptr, *samp_F = nullptr;
    std::vector<long long> resid;
    std::vector<int> done;
    // plain path as replays of a captured cycle of steps (0: off)
    int graph_cycle = 0;
    struct Graph { int nrep, code, phase; hipGraphExec_t exec; };
    std::vector<Graph> graphs;
    // persistent convergence and parallel steps as replays of captured check cycles (0: off)
    int cycles = 0;
    struct CGraph { int op; hipGraphExec_t exec; };
    std::vector<CGraph> cgraphs;
    CycRec *cyc_dev = nullptr, *cyc_host = nullptr;
    Status *stc_dev = nullptr, *stc_host = nullptr;   // [cycles] statuses of a replay
    // scratch
    Status *st_dev = nullptr, *st_host = nullptr;
    long long *adv_fec = nullptr;   // page-locked [R]: first exit checks read back by gpr_advance
    int *adv_err = nullptr;         // page-locked [4]: error flags read back by gpr_advance
    double *obs_out = nullptr;
    int *donor = nullptr, *surv = nullptr;
    long long *fec = nullptr;
    size_t lds_persist = 0, lds_nb = 0, lds_stage = 0;
    int maxlds = 0;            // LDS bytes one workgroup may use on this device
    int maxlds_persist = 0;    // of which k_persist may allocate dynamically
    int persist_ok = 0;
    // event timing of the dominant stepping kernel
    bool prof = false;
    std::vector<hipEvent_t> ev_a, ev_b;
    size_t ev_used = 0;
    double prof_ms = 0.0;
    long long prof_n = 0;
    std::string err;
};

namespace {

gpr_status fail(gpr_system *s, gpr_status code, const std::string &msg)
{
    if (s) s->err = msg;
    g_thread_err = msg;
    return code;
}

#define HIPCHK(sys, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((sys), GPR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK(sys)                                                                           \
    do {                                                                                         \
        hipError_t e_ = hipGetLastError();                                                       \
        if (e_ != hipSuccess)                                                                    \
            return fail((sys), GPR_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

template <class T>
hipError_t dalloc(gpr_system *s, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    s->bufs.push_back(q);
    *p = (T *)q;
    return hipMemset(q, 0, std::max<size_t>(count, 1) * sizeof(T));
}

template <class T>
hipError_t upload(gpr_system *s, T **p, const std::vector<T> &h)
{
    hipError_t e = dalloc(s, p, h.size());
    if (e != hipSuccess || h.empty()) return e;
    return hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
}

bool idx_ok(const int32_t *a, long cnt, int n)
{
    if (cnt > 0 && !a) return false;
    for (long k = 0; k < cnt; ++k) if (a[k] < 0 || a[k] >= n) return false;
    return true;
}

// sorts terms of width w by their smallest atom; returns order, start offsets, span
void sort_terms(const int32_t *atoms, int cnt, int w, int n, std::vector<int> &order, std::vector<int> &start, int &span)
{
    order.resize(cnt);
    std::vector<int> mn(cnt);
    span = 0;
    for (int t = 0; t < cnt; ++t) {
        int lo = atoms[t * w], hi = atoms[t * w];
        for (int k = 1; k < w; ++k) { lo = std::min(lo, (int)atoms[t * w + k]); hi = std::max(hi, (int)atoms[t * w + k]); }
        mn[t] = lo;
        span = std::max(span, hi - lo);
        order[t] = t;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mn[a] < mn[b]; });
    start.assign(n + 1, cnt);
    int t = 0;
    for (int a = 0; a <= n; ++a) {
        while (t < cnt && mn[order[t]] < a) ++t;
        start[a] = t;
    }
}

long long count_samples(long long t_old, long long t_new, int t_gr) { return t_new / t_gr - t_old / t_gr; }

} // namespace

static void drop_cycle_graphs(gpr_system *S);

// event pair around the next timed launch (created on first use, reused afterwards)
// one more pair of timing events (created ahead by gpr_profile, so that a timed call does not
// create them; more only when a call launches the kernel more often than that)
static hipError_t prof_add_pair(gpr_system *S)
{
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return e;
    }
    S->ev_a.push_back(a);
    S->ev_b.push_back(b);
    return hipSuccess;
}

static hipError_t prof_begin(gpr_system *S)
{
    if (!S->prof) return hipSuccess;
    if (S->ev_used == S->ev_a.size()) {
        const hipError_t e = prof_add_pair(S);
        if (e != hipSuccess) return e;
    }
    return hipEventRecord(S->ev_a[S->ev_used], S->stream);
}

static hipError_t prof_end(gpr_system *S)
{
    if (!S->prof) return hipSuccess;
    hipError_t e = hipEventRecord(S->ev_b[S->ev_used], S->stream);
    S->ev_used++;
    return e;
}

// after the stream has drained: fold the recorded pairs into the totals
static hipError_t prof_collect(gpr_system *S)
{
    for (size_t k = 0; k < S->ev_used; ++k) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, S->ev_a[k], S->ev_b[k]);
        if (e != hipSuccess) return e;
        S->prof_ms += ms;
        S->prof_n += 1;
    }
    S->ev_used = 0;
    return hipSuccess;
}

// Atom ranges of the G workgroups of a replica (k_persist): contiguous, starting at multiples
// of 16 (so that every wave of the pair loop covers 16 atoms of one group), with boundaries
// placed where the running sum of the per-atom work estimate crosses g/G of the total.
static Split make_split(const std::vector<double> &work, int n, int np, int G)
{
    Split sp{};
    sp.G = G;
    sp.bnd[0] = 0;
    sp.bnd[G] = n;
    if (G == 1) {
        sp.lmax = np;
        return sp;
    }
    std::vector<double> cum(n + 1, 0.0);
    for (int i = 0; i < n; ++i) cum[i + 1] = cum[i] + work[i];
    for (int g = 1; g < G; ++g) {
        const double target = cum[n] * g / G;
        int a = (int)(std::lower_bound(cum.begin(), cum.end(), target) - cum.begin());
        const int lo = a / 16 * 16, hi = std::min(n, lo + 16);
        a = (target - cum[lo] <= cum[hi] - target) ? lo : hi;
        sp.bnd[g] = std::min(n, std::max(a, sp.bnd[g - 1]));
    }
    int lmax = 16;
    for (int g = 0; g < G; ++g) lmax = std::max(lmax, sp.bnd[g + 1] - sp.bnd[g]);
    sp.lmax = (lmax + 15) / 16 * 16;
    return sp;
}

static size_t persist_lds(int n, int np, const Split &sp)
{
    const int lmax = sp.lmax;
    const int nblk = (n + BLK - 1) / BLK;
    return (size_t)3 * lmax * 8 + (MAX_OBS * 8 + 8) * 8 + MAX_OBS * 8 + (size_t)np * 16 + (size_t)np * 8 +
           (size_t)8 * lmax * 4 + (size_t)nblk * 16 + (size_t)16 * WBLK * 4 + (size_t)32 * ((lmax + 15) / 16) +
           (size_t)2 * lmax;
}

// ------------------------------------------------------------------ force-field parameters
// Device copies of the per-atom parameters (sigma/2, 2 sqrt(eps), q sqrt(f), 1/m), the torsion
// parameters (k, cos phi0, sin phi0, n) and the 1-4 pair parameters (sigma_ij, 4 eps_ij s14,
// f q_i q_j s14) in the sorted term order, and 1/(2 eps_i), from the host copies.
static hipError_t write_params(gpr_system *S)
{
    const int n = S->n, np = S->np;
    Dev &d = S->d;
    const bool mol = S->kind == GPR_KIND_MOLECULAR;
    std::vector<float4> prm(np, make_float4(0, 0, 0, 0));
    std::vector<double> inv2eps(n, 0.0);
    for (int i = 0; i < n; ++i) {
        const double sig = mol ? S->sig_h[i] : 0.0, eps = mol ? S->eps_h[i] : 0.0, q = mol ? S->q_h[i] : 0.0;
        prm[i] = make_float4((float)(0.5 * sig), (float)(2.0 * std::sqrt(eps)), (float)(q * std::sqrt(COULOMB_F)),
                             (float)(1.0 / S->mass_h[i]));
        inv2eps[i] = eps > 0 ? 0.5 / eps : INFINITY;
    }
    hipError_t e = hipMemcpyAsync((void *)d.prm, prm.data(), sizeof(float4) * np, hipMemcpyHostToDevice, S->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void *)d.inv2eps, inv2eps.data(), sizeof(double) * n, hipMemcpyHostToDevice, S->stream);
    const Topo &T = d.tp;
    if (e == hipSuccess && mol && T.nt) {
        std::vector<float4> p(T.nt);
        for (int k = 0; k < T.nt; ++k) {
            const int t = S->tor_order[k];
            p[k] = make_float4((float)S->tor_k_h[t], (float)std::cos(S->tor_phi0_h[t]), (float)std::sin(S->tor_phi0_h[t]),
                               (float)S->tor_n_h[t]);
        }
        e = hipMemcpyAsync((void *)T.t_p, p.data(), sizeof(float4) * T.nt, hipMemcpyHostToDevice, S->stream);
    }
    if (e == hipSuccess && mol && T.n14) {
        std::vector<float4> p(T.n14);
        for (int k = 0; k < T.n14; ++k) {
            const int2 ij = S->p14_h[S->p14_order[k]];
            const double sij = 0.5 * (S->sig_h[ij.x] + S->sig_h[ij.y]);
            const double eij = std::sqrt(S->eps_h[ij.x] * S->eps_h[ij.y]);
            p[k] = make_float4((float)sij, (float)(4.0 * eij * S->scale14),
                               (float)(COULOMB_F * S->q_h[ij.x] * S->q_h[ij.y] * S->scale14), 0.f);
        }
        e = hipMemcpyAsync((void *)T.p_p, p.data(), sizeof(float4) * T.n14, hipMemcpyHostToDevice, S->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    return e;
}

// ------------------------------------------------------------------ launches
// forces of replicas [r_off, r_off + nrep) at their current positions.  Stepping calls
// (force_build = 0) rely on k_integrate to clear the energies and maintain the list guard;
// force-only calls (force_build = 1) rebuild the lists and clear the energies here.
static gpr_status launch_forces(gpr_system *S, int r_off, int nrep, long long s, int energy, int apply_b, int force_build,
                                bool timed = false)
{
    const int BTB = 256, BTN = 1024;
    if (force_build) s = S->s - 1;             // a forced build counts as built in the previous step
    if (energy && force_build) {
        HIPCHK(S, hipMemsetAsync(S->d.E + r_off, 0, sizeof(long long) * nrep, S->stream));
    }
    dim3 gb((S->n + BTB - 1) / BTB, nrep);
    hipLaunchKernelGGL(k_bonded, gb, dim3(BTB), 3 * BTB * sizeof(long long), S->stream, S->d_dev, s, r_off, energy);
    LAUNCHCHK(S);
    dim3 gn((S->n * P + BTN - 1) / BTN, nrep);
    if (timed) HIPCHK(S, prof_begin(S));
    hipLaunchKernelGGL(k_nonbonded, gn, dim3(BTN), S->lds_nb, S->stream, S->d_dev, s, r_off, energy, apply_b, force_build);
    LAUNCHCHK(S);
    if (timed) HIPCHK(S, prof_end(S));
    return GPR_OK;
}

// advances replicas [0, nrep) by nsteps from local step counter t0; sample: accumulate the
// observables of workers every t_gr; state_end: state ids at the end
// Workgroups of the persistent kernel that the device holds at once for (bt, lds): the
// occupancy query, kept per system for the last launch shape asked for.
static gpr_status persist_capacity(gpr_system *S, int bt, size_t lds, int &cap)
{
    if (S->cap_bt != bt || S->cap_lds != lds) {
        int dev = 0, cus = 0, per_cu = 0;
        HIPCHK(S, hipGetDevice(&dev));
        HIPCHK(S, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        HIPCHK(S, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_persist, bt, lds));
        S->cap_bt = bt;
        S->cap_lds = lds;
        S->cap_blocks = per_cu * cus;
    }
    cap = S->cap_blocks;
    return GPR_OK;
}

// Workgroup sets of one system in a persistent launch.  With G > 1 workgroups per replica the
// groups of a replica wait for each other, so they must be resident together: the replicas are
// shared by at most capacity / G sets (cap_blocks < 0: the whole device), so that the grid is
// no larger than what the device holds at once, and every workgroup gets a CU as soon as the
// device is free of other work.  (A launch cannot start its workgroups while other kernels
// hold the CUs they need only until those kernels end; should a group still wait longer than
// the barrier's bounded spin, the call reports GPR_EDEVICE, never hangs.)  No cooperative
// launch: it adds tens of microseconds to each launch and is refused while another process
// holds the device's cooperative resources.
static gpr_status persist_item(gpr_system *S, int nrep, int bt, size_t lds, int cap_blocks, PersistItem &it,
                               int &nblocks)
{
    const int G = S->groups;
    it = PersistItem{};
    it.dev = S->d_dev;
    it.sp = S->split;
    it.nrep = nrep;
    it.boff = 0;
    if (G == 1 && cap_blocks < 0) {
        it.nsets = nrep;
        it.xcd = 0;
        nblocks = nrep;
        return GPR_OK;
    }
    if (cap_blocks < 0) {
        const gpr_status rc = persist_capacity(S, bt, lds, cap_blocks);
        if (rc) return rc;
    }
    int nsets = std::min(nrep, cap_blocks / G);
    if (nsets < 1) return fail(S, GPR_EINVAL, "a replica's workgroups do not fit on the device at once");
    it.xcd = 0;
    if (G > 1 && nsets >= 8) {
        nsets -= nsets % 8;
        it.xcd = 1;
    }
    it.nsets = nsets;
    nblocks = nsets * G;
    return GPR_OK;
}

// The layout of a persistent launch checked on the host before it runs, with the device's own
// placement function: items cover the grid in order without overlap, every workgroup is group
// g < G of a set < nsets, every (set, g) occurs once, the groups' atom ranges are ordered,
// within the system and no longer than the LDS arrays (lmax), and the block size is whole waves.
static gpr_status check_layout(gpr_system *S, const PersistBatch &pb, int nblocks, int bt, bool single)
{
    if (pb.nitems < 1 || pb.nitems > MAX_BATCH || bt < 64 || bt > 1024 || bt % 64) return fail(S, GPR_EDEVICE, "bad persistent launch shape");
    int next = 0;
    for (int k = 0; k < pb.nitems; ++k) {
        const PersistItem &it = pb.it[k];
        const Split &sp = it.sp;
        if (it.boff != next || it.nsets < 1 || it.nrep < 1 || sp.G < 1 || sp.G > 8 || !it.dev)
            return fail(S, GPR_EDEVICE, "persistent launch layout: item placement");
        if (!single && k > 0 && pb.it[k - 1].boff >= it.boff) return fail(S, GPR_EDEVICE, "persistent launch layout: item order");
        const int n = sp.bnd[sp.G];
        if (sp.bnd[0] != 0) return fail(S, GPR_EDEVICE, "persistent launch layout: atom ranges");
        for (int g = 0; g < sp.G; ++g)
            if (sp.bnd[g] > sp.bnd[g + 1] || sp.bnd[g + 1] > n || sp.bnd[g + 1] - sp.bnd[g] > sp.lmax)
                return fail(S, GPR_EDEVICE, "persistent launch layout: atom ranges");
        std::vector<unsigned char> seen((size_t)it.nsets * sp.G, 0);
        for (int local = 0; local < it.nsets * sp.G; ++local) {
            int set = -1, g = -1;
            if (!persist_place(it, local, set, g) || set < 0 || set >= it.nsets || g < 0 || g >= sp.G ||
                seen[(size_t)set * sp.G + g]++)
                return fail(S, GPR_EDEVICE, "persistent launch layout: workgroup placement");
        }
        next = it.boff + it.nsets * sp.G;
    }
    if (next != nblocks) return fail(S, GPR_EDEVICE, "persistent launch layout: grid size");
    return GPR_OK;
}

// One item whose sets each take one replica (roff + set) runs k_persist; anything else
// (several systems, or sets that take replicas in turn) runs k_persist_batch.
static gpr_status launch_persist(gpr_system *S, PersistBatch &pb, int nblocks, int bt, size_t lds,
                                 hipStream_t stream, bool one_round = false)
{
    const bool single = pb.nitems == 1 && (one_round || pb.it[0].nsets >= pb.it[0].nrep);
    {
        const gpr_status rc = check_layout(S, pb, nblocks, bt, single);
        if (rc) return rc;
    }
    const void *fn = single ? (const void *)k_persist : (const void *)k_persist_batch;
    void *args_single[] = {(void *)&pb.it[0]};
    void *args_batch[] = {(void *)&pb};
    void **args = single ? args_single : args_batch;
    HIPCHK(S, hipLaunchKernel(fn, dim3(nblocks), dim3(bt), args, lds, stream));
    return GPR_OK;
}

// Step k of a captured cycle on the device clock (code DCLK_*): the kernels read the cycle's
// first step and local step from the device, so every replay continues where the last one
// stopped.  The observables of the workers: with phase >= 0 (the local step at the cycle's
// start, mod t_GR) at the steps that sample; with phase < 0 a launch every step that returns
// unless the step samples.
static gpr_status launch_step_dc(gpr_system *S, int nrep, int code, int phase, int k, hipStream_t st)
{
    const int BTI = 256, BTB = 256, BTN = 1024;
    hipLaunchKernelGGL(k_integrate, dim3((S->n + BTI - 1) / BTI, nrep), dim3(BTI), 0, st, S->d_dev, (long long)k, 0, code);
    LAUNCHCHK(S);
    hipLaunchKernelGGL(k_bonded, dim3((S->n + BTB - 1) / BTB, nrep), dim3(BTB), 3 * BTB * sizeof(long long), st, S->d_dev,
                       (long long)k, 0, code);
    LAUNCHCHK(S);
    hipLaunchKernelGGL(k_nonbonded, dim3((S->n * P + BTN - 1) / BTN, nrep), dim3(BTN), S->lds_nb, st, S->d_dev,
                       (long long)k, 0, code, 1, 0);
    LAUNCHCHK(S);
    if (code == DCLK_SAMPLE && nrep > 1) {
        if (phase < 0) {
            hipLaunchKernelGGL(k_obs, dim3(nrep - 1), dim3(256), S->lds_stage, st, S->d_dev, 1, 3, nullptr, k);
            LAUNCHCHK(S);
        } else if ((phase + k + 1) % S->t_gr == 0) {
            hipLaunchKernelGGL(k_obs, dim3(nrep - 1), dim3(256), S->lds_stage, st, S->d_dev, 1, 0, nullptr, 0);
            LAUNCHCHK(S);
        }
    }
    return GPR_OK;
}

// The executable graph of graph_cycle device-clocked steps and the clock advance for
// (nrep, code, phase), captured on a stream of its own the first time it is needed.
static gpr_status plain_graph(gpr_system *S, int nrep, int code, int phase, hipGraphExec_t *out)
{
    for (auto &g : S->graphs)
        if (g.nrep == nrep && g.code == code && g.phase == phase) { *out = g.exec; return GPR_OK; }
    hipStream_t cs = nullptr;
    HIPCHK(S, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    gpr_status rc = GPR_OK;
    for (int k = 0; k < S->graph_cycle && e == hipSuccess && rc == GPR_OK; ++k)
        rc = launch_step_dc(S, nrep, code, phase, k, cs);
    if (e == hipSuccess && rc == GPR_OK) {
        hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, cs, S->d_dev, (long long)S->graph_cycle);
        e = hipGetLastError();
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipSuccess;
    if (e == hipSuccess && e2 == hipSuccess && rc == GPR_OK) e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (rc) return rc;
    if (e != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return fail(S, GPR_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2 != hipSuccess ? e2 : e3));
    S->graphs.push_back({nrep, code, phase, ex});
    *out = ex;
    return GPR_OK;
}

// nsteps plain steps launched from the host, local steps counted from t0
static gpr_status plain_steps(gpr_system *S, int nrep, long long nsteps, long long t0, bool sample)
{
    const int BTI = 256;
    dim3 gi((S->n + BTI - 1) / BTI, nrep);
    for (long long k = 0; k < nsteps; ++k) {
        const long long tl = t0 + k + 1;
        const bool samp = sample && nrep > 1 && (tl % S->t_gr == 0);
        const int energy = (samp && S->d.need_energy) ? 1 : 0;
        hipLaunchKernelGGL(k_integrate, gi, dim3(BTI), 0, S->stream, S->d_dev, S->s, 0, energy);
        LAUNCHCHK(S);
        gpr_status rc = launch_forces(S, 0, nrep, S->s, energy, 1, 0, true);
        if (rc) return rc;
        S->s += 1;
        if (samp) {
            hipLaunchKernelGGL(k_obs, dim3(nrep - 1), dim3(256), S->lds_stage, S->stream, S->d_dev, 1, 0, nullptr, 0);
            LAUNCHCHK(S);
        }
    }
    return GPR_OK;
}

static gpr_status run_steps(gpr_system *S, int nrep, long long nsteps, long long t0, bool sample, bool state_end)
{
    if (nsteps <= 0) {
        if (state_end) {
            hipLaunchKernelGGL(k_state, dim3(nrep), dim3(256), S->lds_stage, S->stream, S->d_dev, 0);
            LAUNCHCHK(S);
        }
        return GPR_OK;
    }
    if (S->path == GPR_PATH_PERSISTENT) {
        PersistBatch pb{};
        pb.nitems = 1;
        int nblocks = 0;
        const size_t lds = persist_lds(S->n, S->np, S->split);
        gpr_status rc = persist_item(S, nrep, S->bt_persist, lds, -1, pb.it[0], nblocks);
        if (rc) return rc;
        // more replicas than sets that fit at once: rounds of launches, each set taking one
        // replica per launch (replicas are independent between checks)
        const int rounds = (nrep + pb.it[0].nsets - 1) / pb.it[0].nsets;
        long long done = 0;
        while (done < nsteps) {
            const int chunk = (int)std::min<long long>(nsteps - done, 1 << 20);
            const bool last = done + chunk == nsteps;
            PersistItem &it = pb.it[0];
            it.s0 = S->s + done;
            it.nsteps = chunk;
            it.t0 = (int)((t0 + done) % S->t_gr);        // the device uses it modulo t_GR only
            it.sample = sample ? 1 : 0;
            it.state_end = (state_end && last) ? 1 : 0;
            for (int k = 0; k < rounds; ++k) {
                it.roff = k * it.nsets;
                HIPCHK(S, prof_begin(S));
                rc = launch_persist(S, pb, nblocks, S->bt_persist, lds, S->stream, true);
                if (rc) return rc;
                HIPCHK(S, prof_end(S));
            }
            done += chunk;
        }
        S->s += nsteps;
        return GPR_OK;
    }
    // whole cycles replayed from a captured graph, the steps left over launched from the host
    long long left = nsteps, tcur = t0;
    if (S->graph_cycle > 0 && left >= S->graph_cycle) {
        const int code = (sample && nrep > 1) ? DCLK_SAMPLE : DCLK_NOSAMPLE;
        const int phase = (code == DCLK_SAMPLE && S->graph_cycle % S->t_gr == 0) ? (int)(t0 % S->t_gr) : -1;
        hipGraphExec_t ex = nullptr;
        gpr_status rc = plain_graph(S, nrep, code, phase, &ex);
        if (rc) return rc;
        hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(1), 0, S->stream, S->d_dev, S->s, t0);
        LAUNCHCHK(S);
        for (; left >= S->graph_cycle; left -= S->graph_cycle) {
            HIPCHK(S, hipGraphLaunch(ex, S->stream));
            S->s += S->graph_cycle;
            tcur += S->graph_cycle;
        }
    }
    gpr_status rc = plain_steps(S, nrep, left, tcur, sample);
    if (rc) return rc;
    if (state_end) {
        hipLaunchKernelGGL(k_state, dim3(nrep), dim3(256), S->lds_stage, S->stream, S->d_dev, 0);
        LAUNCHCHK(S);
    }
    return GPR_OK;
}

// the error flags a check copied into its status
static gpr_status status_errors(gpr_system *S, const Status &st)
{
    if (st.err[ERR_UNSTABLE]) return fail(S, GPR_EUNSTABLE, "non-finite or overflowing state");
    if (st.err[ERR_LIST]) return fail(S, GPR_EDEVICE, "pair-list capacity exceeded");
    if (st.err[ERR_BARRIER]) return fail(S, GPR_EDEVICE, "persistent-kernel barrier timed out");
    return GPR_OK;
}

// one launch: bookkeeping by block (0, 0), and with CHK_DEPHASE the clone-on-kill copies by
// the blocks of each killed worker's row
static gpr_status check(gpr_system *S, int mode, int nrep, long long check_index)
{
    const dim3 grid = mode == CHK_DEPHASE ? dim3((3 * S->np + 255) / 256, nrep) : dim3(1, 1);
    hipLaunchKernelGGL(k_check, grid, dim3(256), sizeof(int) * nrep, S->stream, S->d_dev, mode, S->s, S->omega, nrep,
                       S->nsamp, check_index, (long long)S->tcp, S->st_dev, S->donor, S->surv, S->fec,
                       (CycRec *)nullptr, 0);
    LAUNCHCHK(S);
    HIPCHK(S, hipMemcpyAsync(S->st_host, S->st_dev, sizeof(Status), hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
    HIPCHK(S, prof_collect(S));
    return status_errors(S, *S->st_host);
}

static gpr_status copy_replica(gpr_system *S, int dst, int src)
{
    std::vector<int> dn(S->R, -1);
    dn[dst] = src;
    HIPCHK(S, hipMemcpyAsync(S->donor, dn.data(), sizeof(int) * S->R, hipMemcpyHostToDevice, S->stream));
    hipLaunchKernelGGL(k_clone, dim3((3 * S->np + 255) / 256, S->R), dim3(256), 0, S->stream, S->d_dev, S->donor, 0);
    LAUNCHCHK(S);
    return GPR_OK;
}

static gpr_status broadcast_reference(gpr_system *S)
{
    std::vector<int> dn(S->R, 0);
    dn[0] = -1;
    HIPCHK(S, hipMemcpyAsync(S->donor, dn.data(), sizeof(int) * S->R, hipMemcpyHostToDevice, S->stream));
    hipLaunchKernelGGL(k_clone, dim3((3 * S->np + 255) / 256, S->R), dim3(256), 0, S->stream, S->d_dev, S->donor, 1);
    LAUNCHCHK(S);
    return GPR_OK;
}

static gpr_status state_of_ref(gpr_system *S, int *out)
{
    gpr_status rc = run_steps(S, 1, 0, 0, false, true);
    if (rc) return rc;
    rc = check(S, CHK_STATE, 1, 0);
    if (rc) return rc;
    *out = S->st_host->to_state;
    return GPR_OK;
}

// ------------------------------------------------------------------ create / destroy
extern "C" void gpr_system_destroy(gpr_system *S)
{
    if (!S) return;
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    for (auto &g : S->graphs) (void)hipGraphExecDestroy(g.exec);
    for (auto &g : S->cgraphs) (void)hipGraphExecDestroy(g.exec);
    if (S->cyc_dev) (void)hipFree(S->cyc_dev);
    if (S->stc_dev) (void)hipFree(S->stc_dev);
    if (S->cyc_host) (void)hipHostFree(S->cyc_host);
    if (S->stc_host) (void)hipHostFree(S->stc_host);
    for (void *p : S->bufs) (void)hipFree(p);
    for (hipEvent_t e : S->ev_a) (void)hipEventDestroy(e);
    for (hipEvent_t e : S->ev_b) (void)hipEventDestroy(e);
    if (S->st_host) (void)hipHostFree(S->st_host);
    if (S->adv_fec) (void)hipHostFree(S->adv_fec);
    if (S->adv_err) (void)hipHostFree(S->adv_err);
    delete S;
}

extern "C" const char *gpr_last_error(const gpr_system *S)
{
    return S ? S->err.c_str() : g_thread_err.c_str();
}


static gpr_status create_impl(const gpr_system_desc *D, gpr_system *S)
{
    const int n = D->n_atoms, R = D->n_replicas;
    S->n = n; S->R = R; S->kind = D->kind;
    S->np = (n + 1 + 63) / 64 * 64;   // room for the dummy atom n
    const int np = S->np;
    S->t_gr = D->t_gr; S->tcd = D->t_check_dephase; S->tcp = D->t_check_parallel;
    S->tol = D->tol; S->dt = D->dt; S->t_min = D->t_min; S->kT = D->kT;
    S->nobs = D->n_obs;
    Dev &d = S->d;
    d.kind = D->kind; d.n = n; d.np = np; d.R = R;

    // per-atom parameters
    const double c1 = std::exp(-D->gamma * D->dt);
    const double c2 = std::sqrt(std::max(0.0, 1.0 - c1 * c1));
    std::vector<float4> prm(np, make_float4(0, 0, 0, 0));
    std::vector<float> sd(np, 0.f), mass(np, 0.f);
    for (int i = 0; i < n; ++i) {
        const double sig = D->kind == GPR_KIND_MOLECULAR ? D->sigma[i] : 0.0;
        const double eps = D->kind == GPR_KIND_MOLECULAR ? D->epsilon[i] : 0.0;
        const double q = D->kind == GPR_KIND_MOLECULAR ? D->charge[i] : 0.0;
        prm[i] = make_float4((float)(0.5 * sig), (float)(2.0 * std::sqrt(eps)), (float)(q * std::sqrt(COULOMB_F)),
                             (float)(1.0 / D->mass[i]));
        sd[i] = (float)(c2 * std::sqrt(D->kT / D->mass[i]));
        mass[i] = (float)D->mass[i];
    }
    HIPCHK(S, upload(S, (float4 **)&d.prm, prm));
    HIPCHK(S, upload(S, (float **)&d.sd, sd));
    HIPCHK(S, upload(S, (float **)&d.mass, mass));

    // exclusions (and 1-4 pairs) as bit masks over index offsets -32..31, and those farther
    // apart as an ascending partner list per atom
    std::vector<unsigned long long> excl(np, 0ull);
    std::vector<std::vector<int>> far(n);
    auto mark = [&](int i, int j) {
        const int off = j - i;
        if (off == 0) return;
        if (off > -32 && off < 32) {
            excl[i] |= 1ull << (off + 32);
            excl[j] |= 1ull << (-off + 32);
        } else {
            far[i].push_back(j);
            far[j].push_back(i);
        }
    };
    if (D->kind == GPR_KIND_MOLECULAR) {
        for (int e = 0; e < D->n_exclusions; ++e) mark(D->exclusion_atoms[2 * e], D->exclusion_atoms[2 * e + 1]);
        for (int p = 0; p < D->n_pairs14; ++p) mark(D->pair14_atoms[2 * p], D->pair14_atoms[2 * p + 1]);
    }
    std::vector<int> far_start(n + 1, 0), far_j;
    for (int i = 0; i < n; ++i) {
        std::sort(far[i].begin(), far[i].end());
        far[i].erase(std::unique(far[i].begin(), far[i].end()), far[i].end());
        far_start[i + 1] = far_start[i] + (int)far[i].size();
        far_j.insert(far_j.end(), far[i].begin(), far[i].end());
    }
    d.has_far = far_j.empty() ? 0 : 1;
    HIPCHK(S, upload(S, (unsigned long long **)&d.excl, excl));
    HIPCHK(S, upload(S, (int **)&d.far_start, far_start));
    HIPCHK(S, upload(S, (int **)&d.far_j, far_j));

    // replica state: every replica starts from (pos, vel)
    const size_t rs = (size_t)R * 3 * np;
    std::vector<float> x0(3 * np, 0.f), v0(3 * np, 0.f);
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < n; ++i) {
            x0[c * np + i] = (float)D->pos[c * n + i];
            if (D->vel) v0[c * np + i] = (float)D->vel[c * n + i];
        }
    if (D->kind == GPR_KIND_TOY2D) { x0[2 * np] = 0.f; v0[2 * np] = 0.f; }
    HIPCHK(S, dalloc(S, &d.x, rs));
    HIPCHK(S, dalloc(S, &d.v, rs));
    HIPCHK(S, dalloc(S, &d.xb, rs));
    HIPCHK(S, dalloc(S, &d.F, rs));
    HIPCHK(S, dalloc(S, &d.E, R));
    HIPCHK(S, hipMemcpy(d.x, x0.data(), sizeof(float) * 3 * np, hipMemcpyHostToDevice));
    HIPCHK(S, hipMemcpy(d.v, v0.data(), sizeof(float) * 3 * np, hipMemcpyHostToDevice));

    // bonded topology, each type sorted by smallest atom
    Topo &T = d.tp;
    std::vector<int> order, start;
    if (D->kind == GPR_KIND_MOLECULAR) {
        {
            sort_terms(D->bond_atoms, D->n_bonds, 2, n, order, start, T.b_span);
            std::vector<int2> ij(D->n_bonds); std::vector<float2> p(D->n_bonds);
            for (int k = 0; k < D->n_bonds; ++k) {
                const int t = order[k];
                ij[k] = make_int2(D->bond_atoms[2 * t], D->bond_atoms[2 * t + 1]);
                p[k] = make_float2((float)D->bond_r0[t], (float)D->bond_k[t]);
            }
            T.nb = D->n_bonds;
            HIPCHK(S, upload(S, (int2 **)&T.b_ij, ij)); HIPCHK(S, upload(S, (float2 **)&T.b_p, p));
            HIPCHK(S, upload(S, (int **)&T.b_start, start));
        }
        {
            sort_terms(D->angle_atoms, D->n_angles, 3, n, order, start, T.a_span);
            std::vector<int4> ijk(D->n_angles); std::vector<float2> p(D->n_angles);
            for (int k = 0; k < D->n_angles; ++k) {
                const int t = order[k];
                ijk[k] = make_int4(D->angle_atoms[3 * t], D->angle_atoms[3 * t + 1], D->angle_atoms[3 * t + 2], 0);
                p[k] = make_float2((float)D->angle_theta0[t], (float)D->angle_k[t]);
            }
            T.na = D->n_angles;
            HIPCHK(S, upload(S, (int4 **)&T.a_ijk, ijk)); HIPCHK(S, upload(S, (float2 **)&T.a_p, p));
            HIPCHK(S, upload(S, (int **)&T.a_start, start));
        }
        {
            sort_terms(D->torsion_atoms, D->n_torsions, 4, n, order, start, T.t_span);
            std::vector<int4> q(D->n_torsions); std::vector<float4> p(D->n_torsions);
            for (int k = 0; k < D->n_torsions; ++k) {
                const int t = order[k];
                q[k] = make_int4(D->torsion_atoms[4 * t], D->torsion_atoms[4 * t + 1], D->torsion_atoms[4 * t + 2],
                                 D->torsion_atoms[4 * t + 3]);
                p[k] = make_float4((float)D->torsion_k[t], (float)std::cos(D->torsion_phi0[t]),
                                   (float)std::sin(D->torsion_phi0[t]), (float)D->torsion_n[t]);
            }
            T.nt = D->n_torsions;
            S->tor_order = order;
            HIPCHK(S, upload(S, (int4 **)&T.t_ijkl, q)); HIPCHK(S, upload(S, (float4 **)&T.t_p, p));
            HIPCHK(S, upload(S, (int **)&T.t_start, start));
        }
        {
            int span0 = 0;
            sort_terms(D->restraint_atom, D->n_restraints, 1, n, order, start, span0);
            std::vector<int> ia(D->n_restraints); std::vector<float4> p(D->n_restraints);
            for (int k = 0; k < D->n_restraints; ++k) {
                const int t = order[k];
                ia[k] = D->restraint_atom[t];
                p[k] = make_float4((float)D->restraint_ref[3 * t], (float)D->restraint_ref[3 * t + 1],
                                   (float)D->restraint_ref[3 * t + 2], (float)D->restraint_k[t]);
            }
            T.nr = D->n_restraints;
            HIPCHK(S, upload(S, (int **)&T.r_i, ia)); HIPCHK(S, upload(S, (float4 **)&T.r_p, p));
            HIPCHK(S, upload(S, (int **)&T.r_start, start));
        }
        {
            sort_terms(D->pair14_atoms, D->n_pairs14, 2, n, order, start, T.p_span);
            std::vector<int2> ij(D->n_pairs14); std::vector<float4> p(D->n_pairs14);
            for (int k = 0; k < D->n_pairs14; ++k) {
                const int t = order[k];
                const int i = D->pair14_atoms[2 * t], j = D->pair14_atoms[2 * t + 1];
                ij[k] = make_int2(i, j);
                const double sij = 0.5 * (D->sigma[i] + D->sigma[j]);
                const double eij = std::sqrt(D->epsilon[i] * D->epsilon[j]);
                p[k] = make_float4((float)sij, (float)(4.0 * eij * D->scale14),
                                   (float)(COULOMB_F * D->charge[i] * D->charge[j] * D->scale14), 0.f);
            }
            T.n14 = D->n_pairs14;
            S->p14_order = order;
            HIPCHK(S, upload(S, (int2 **)&T.p_ij, ij)); HIPCHK(S, upload(S, (float4 **)&T.p_p, p));
            HIPCHK(S, upload(S, (int **)&T.p_start, start));
        }
    }

    // nonbonded constants and pair-list capacity
    d.cutoff_on = (D->kind == GPR_KIND_MOLECULAR && D->cutoff > 0) ? 1 : 0;
    if (d.cutoff_on) {
        const double rc = D->cutoff;
        const double krf = (D->eps_rf - 1.0) / ((2.0 * D->eps_rf + 1.0) * rc * rc * rc);
        d.rc2 = (float)(rc * rc);
        d.krf = (float)krf;
        d.crf = (float)(1.0 / rc + krf * rc * rc);
        d.rl = (float)(rc + D->skin + 1e-4);
        d.rl2 = d.rl * d.rl;
        d.half_skin2 = (float)(0.25 * D->skin * D->skin);
        d.period = std::max(1, D->nlist_period);
    } else {
        d.rc2 = INFINITY; d.krf = 0.f; d.crf = 0.f; d.rl = INFINITY; d.rl2 = INFINITY;
        d.half_skin2 = INFINITY; d.period = 1 << 30;
    }
    // capacity from the initial structure: the largest sub-list within r_list, doubled
    // per-atom work estimate for the persistent split: partners within r_list plus a constant
    // for the bonded terms, the integrator and the list build (about 72 pair evaluations' worth
    // per atom, fitted to measured per-group phase times)
    int maxsub = 0;
    S->work.assign(n, 1.0);
    if (D->kind == GPR_KIND_MOLECULAR) {
        const double rl2 = d.cutoff_on ? (double)d.rl * d.rl * 1.21 : INFINITY;
        const double rl2w = d.cutoff_on ? (double)d.rl * d.rl : INFINITY;
        std::vector<int> cnt(P);
        for (int i = 0; i < n; ++i) {
            std::fill(cnt.begin(), cnt.end(), 0);
            int nw = 0;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                const double dx = D->pos[i] - D->pos[j], dy = D->pos[n + i] - D->pos[n + j], dz = D->pos[2 * n + i] - D->pos[2 * n + j];
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rl2) cnt[j % P]++;
                if (r2 < rl2w) nw++;
            }
            for (int q = 0; q < P; ++q) maxsub = std::max(maxsub, cnt[q]);
            S->work[i] = nw + 72.0;
        }
    }
    const int kmax = std::max(8, d.cutoff_on ? 2 * maxsub + 8 : maxsub + 1);
    d.Kg = std::min(16383, (kmax + 3) / 4);
    HIPCHK(S, dalloc(S, &d.nbl, (size_t)R * d.Kg * np * P));
    HIPCHK(S, dalloc(S, &d.nbc, (size_t)R * np * P));
    HIPCHK(S, dalloc(S, &d.guard, 2 * R));
    HIPCHK(S, dalloc(S, &d.need_build, R));
    HIPCHK(S, dalloc(S, &d.list_pad, R));
    HIPCHK(S, dalloc(S, &d.last_build, 2 * R));
    HIPCHK(S, dalloc(S, &d.clock, 2));
    HIPCHK(S, dalloc(S, &d.err, 4));
    HIPCHK(S, dalloc(S, &d.sync, (size_t)R * 64));
    HIPCHK(S, dalloc(S, &d.xchg, (size_t)R * 6 * np));
    HIPCHK(S, dalloc(S, &d.esum, R));
    HIPCHK(S, dalloc(S, &d.acc, (size_t)R * MAX_OBS * 2));
    HIPCHK(S, dalloc(S, &d.shift, MAX_OBS));
    HIPCHK(S, dalloc(S, &d.state, R));

    // states and observables with their atom groups
    std::vector<int> groups;
    auto add_group = [&](const int32_t *g, int cnt, int &off, double &mtot) {
        off = (int)groups.size();
        mtot = 0;
        for (int k = 0; k < cnt; ++k) { groups.push_back(g[k]); mtot += D->mass[g[k]]; }
    };
    StateDesc st{};
    std::vector<ObsDesc> obs(MAX_OBS);
    st.kind = D->state.kind;
    for (int k = 0; k < 8; ++k) st.atoms[k] = D->state.atoms[k];
    st.nbox = D->state.n_boxes;
    for (int b = 0; b < GPR_MAX_BOXES; ++b)
        for (int c = 0; c < 4; ++c) st.box[b][c] = D->state.box[b][c];
    for (int c = 0; c < 3; ++c) st.center[c] = D->state.center[c];
    st.radius = D->state.radius;
    st.g_n = D->state.kind == GPR_STATE_COM_SPHERE ? D->state.n_group : 0;
    add_group(D->state.group, st.g_n, st.g_off, st.gm);
    d.nobs = D->n_obs;
    d.need_energy = 0;
    for (int j = 0; j < D->n_obs; ++j) {
        const gpr_obs_desc &o = D->obs[j];
        ObsDesc &od = obs[j];
        od.kind = o.kind;
        for (int k = 0; k < 4; ++k) od.atoms[k] = o.atoms[k];
        od.ga_n = (o.kind == GPR_OBS_COM_DISTANCE || o.kind == GPR_OBS_RMS_VELOCITY) ? o.n_a : 0;
        od.gb_n = o.kind == GPR_OBS_COM_DISTANCE ? o.n_b : 0;
        add_group(o.group_a, od.ga_n, od.ga_off, od.ma);
        add_group(o.group_b, od.gb_n, od.gb_off, od.mb);
        if (o.kind == GPR_OBS_POTENTIAL) d.need_energy = 1;
    }
    HIPCHK(S, upload(S, (int **)&d.groups, groups));
    HIPCHK(S, upload(S, (ObsDesc **)&d.obs, obs));
    HIPCHK(S, upload(S, (StateDesc **)&d.st, std::vector<StateDesc>(1, st)));

    d.h = (float)(0.5 * D->dt);
    d.c1 = (float)c1;
    d.key0 = (uint32_t)D->seed;
    d.key1 = (uint32_t)(D->seed >> 32);
    d.t_gr = D->t_gr;
    d.tol = D->tol;
    d.t_min = D->t_min;
    // force-field parameters kept on the host, device buffers of the parameter gradient
    S->mass_h.assign(D->mass, D->mass + n);
    if (D->kind == GPR_KIND_MOLECULAR) {
        S->eps_h.assign(D->epsilon, D->epsilon + n);
        S->sig_h.assign(D->sigma, D->sigma + n);
        S->q_h.assign(D->charge, D->charge + n);
        S->tor_k_h.assign(D->torsion_k, D->torsion_k + D->n_torsions);
        S->tor_phi0_h.assign(D->torsion_phi0, D->torsion_phi0 + D->n_torsions);
        S->tor_n_h.assign(D->torsion_n, D->torsion_n + D->n_torsions);
        for (int t = 0; t < D->n_pairs14; ++t)
            S->p14_h.push_back(make_int2(D->pair14_atoms[2 * t], D->pair14_atoms[2 * t + 1]));
        S->scale14 = D->scale14;
    }
    d.scale14 = (float)D->scale14;
    d.sqrt_f = std::sqrt(COULOMB_F);
    HIPCHK(S, dalloc(S, &d.gacc, (size_t)3 * np + std::max(1, d.tp.nt)));
    {
        std::vector<double> inv2eps(n, 0.0);
        HIPCHK(S, upload(S, (double **)&d.inv2eps, inv2eps));
        std::vector<int> orig(S->tor_order);
        if (orig.empty()) orig.push_back(0);
        HIPCHK(S, upload(S, (int **)&d.tor_orig, orig));
    }
    HIPCHK(S, write_params(S));
    HIPCHK(S, upload(S, &S->d_dev, std::vector<Dev>(1, d)));

    // scratch for the per-check bookkeeping
    HIPCHK(S, dalloc(S, &S->st_dev, 1));
    HIPCHK(S, hipHostMalloc((void **)&S->st_host, sizeof(Status), hipHostMallocDefault));
    HIPCHK(S, hipHostMalloc((void **)&S->adv_fec, sizeof(long long) * R, hipHostMallocDefault));
    HIPCHK(S, hipHostMalloc((void **)&S->adv_err, sizeof(int) * 4, hipHostMallocDefault));
    HIPCHK(S, dalloc(S, &S->donor, R));
    HIPCHK(S, dalloc(S, &S->surv, R));
    HIPCHK(S, dalloc(S, &S->fec, R));
    HIPCHK(S, dalloc(S, &S->obs_out, (size_t)R * MAX_OBS));

    // LDS budgets
    const int nblk = (n + BLK - 1) / BLK;
    S->lds_nb = (size_t)np * 24 + (size_t)nblk * 16 + (size_t)16 * WBLK * 4;
    S->lds_stage = (size_t)np * 16;
    int dev = 0, maxlds = 0;
    HIPCHK(S, hipGetDevice(&dev));
    HIPCHK(S, hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    S->maxlds = maxlds;
    if ((int)S->lds_nb > maxlds || (int)S->lds_stage > maxlds)
        return fail(S, GPR_EINVAL, "system too large for the LDS-staged pair kernel");
    HIPCHK(S, hipFuncSetAttribute((const void *)k_nonbonded, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S->lds_nb));
    HIPCHK(S, hipFuncSetAttribute((const void *)k_grad_nb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S->lds_nb));
    HIPCHK(S, hipFuncSetAttribute((const void *)k_obs, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S->lds_stage));
    HIPCHK(S, hipFuncSetAttribute((const void *)k_state, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S->lds_stage));
    {
        // dynamic LDS available to k_persist next to its static LDS
        hipFuncAttributes fa{};
        HIPCHK(S, hipFuncGetAttributes(&fa, (const void *)k_persist));
        S->maxlds_persist = maxlds - (int)fa.sharedSizeBytes;
        HIPCHK(S, hipFuncSetAttribute((const void *)k_persist, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      S->maxlds_persist));
        hipFuncAttributes fb{};
        HIPCHK(S, hipFuncGetAttributes(&fb, (const void *)k_persist_batch));
        if ((int)fb.sharedSizeBytes != (int)fa.sharedSizeBytes) return fail(S, GPR_EDEVICE, "persistent kernels differ in static LDS");
        HIPCHK(S, hipFuncSetAttribute((const void *)k_persist_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      S->maxlds_persist));
    }
    S->bt_persist = std::min(1024, std::max(64, (n * P + 63) / 64 * 64));
    {
        // persistent split: the fewest workgroups per replica (1, 2, 4 or 8) whose LDS fits, then
        // more while each keeps >= 256 atoms; with more than one, every workgroup of the grid
        // must be resident at once (the grid is sized to what the device holds)
        int cus = 0;
        HIPCHK(S, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        S->max_coresident = cus;
        // usable: the LDS fits and a workgroup can run; all_at_once: every replica's workgroups are
        // resident together (with fewer, sets of workgroups take the replicas in turn)
        auto usable = [&](int G, bool &ok, bool &all_at_once) -> hipError_t {
            const size_t lds = persist_lds(n, np, make_split(S->work, n, np, G));
            ok = all_at_once = false;
            if ((int)lds > S->maxlds_persist) return hipSuccess;
            int per_cu = 0;
            const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_persist,
                                                                              S->bt_persist, lds);
            ok = e == hipSuccess && per_cu >= 1;
            all_at_once = ok && (G == 1 || (long)R * G <= (long)per_cu * cus);
            return e;
        };
        int G = 1;
        bool ok = false, all = false;
        for (; G <= 8; G *= 2) {
            HIPCHK(S, usable(G, ok, all));
            if (ok) break;
        }
        S->persist_ok = ok ? 1 : 0;
        if (ok) {
            while (G < 8 && (n + 2 * G - 1) / (2 * G) >= 256) {
                bool ok2 = false, all2 = false;
                HIPCHK(S, usable(2 * G, ok2, all2));
                if (!ok2 || !all2) break;
                G *= 2;
            }
        } else {
            G = 1;
        }
        S->groups = G;
        S->split = make_split(S->work, n, np, G);
        S->lds_persist = persist_lds(n, np, S->split);
    }

    // initial velocities, copies into every replica, forces, Omega and the observable shift
    if (!D->vel) {
        hipLaunchKernelGGL(k_init_vel, dim3((n + 255) / 256), dim3(256), 0, S->stream, S->d_dev, (float)D->kT);
        LAUNCHCHK(S);
    }
    gpr_status rc = launch_forces(S, 0, 1, -1, 1, 0, 1);
    if (rc) return rc;
    rc = broadcast_reference(S);
    if (rc) return rc;
    HIPCHK(S, hipMemsetAsync(d.need_build, 0, sizeof(int) * R, S->stream));
    rc = launch_forces(S, 0, R, -1, 1, 0, 1);
    if (rc) return rc;
    hipLaunchKernelGGL(k_obs, dim3(1), dim3(256), S->lds_stage, S->stream, S->d_dev, 0, 1, nullptr, 0);
    LAUNCHCHK(S);
    rc = state_of_ref(S, &S->omega);
    if (rc) return rc;
    S->phase = PH_IDLE;
    return GPR_OK;
}

extern "C" gpr_status gpr_system_create(const gpr_system_desc *D, gpr_system **out)
{
    if (!out) return fail(nullptr, GPR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!D) return fail(nullptr, GPR_EINVAL, "descriptor is NULL");
    if (D->kind != GPR_KIND_TOY2D && D->kind != GPR_KIND_MOLECULAR) return fail(nullptr, GPR_EINVAL, "bad kind");
    if (D->n_atoms < 1 || D->n_atoms > 65535 || D->n_replicas < 2 || D->n_replicas > 4096 || !D->mass || !D->pos)
        return fail(nullptr, GPR_EINVAL, "bad sizes or missing arrays");
    if (D->kind == GPR_KIND_TOY2D && D->n_atoms != 1) return fail(nullptr, GPR_EINVAL, "the toy system has one particle");
    if (!(D->dt > 0) || !(D->kT > 0) || !(D->gamma >= 0)) return fail(nullptr, GPR_EINVAL, "bad dynamics parameters");
    if (D->t_gr < 1 || D->t_check_dephase < 1 || D->t_check_parallel < 1) return fail(nullptr, GPR_EINVAL, "bad periods");
    if (D->n_obs < 0 || D->n_obs > GPR_MAX_OBS || (D->n_obs > 0 && !D->obs)) return fail(nullptr, GPR_EINVAL, "bad observables");
    const int n = D->n_atoms;
    for (int i = 0; i < n; ++i) if (!(D->mass[i] > 0)) return fail(nullptr, GPR_EINVAL, "mass <= 0");
    if (D->kind == GPR_KIND_MOLECULAR) {
        if (!D->sigma || !D->epsilon || !D->charge) return fail(nullptr, GPR_EINVAL, "missing nonbonded parameters");
        if (!idx_ok(D->bond_atoms, 2L * D->n_bonds, n) || !idx_ok(D->angle_atoms, 3L * D->n_angles, n) ||
            !idx_ok(D->torsion_atoms, 4L * D->n_torsions, n) || !idx_ok(D->restraint_atom, D->n_restraints, n) ||
            !idx_ok(D->pair14_atoms, 2L * D->n_pairs14, n) || !idx_ok(D->exclusion_atoms, 2L * D->n_exclusions, n))
            return fail(nullptr, GPR_EINVAL, "term atom index out of range");
        if ((D->n_bonds && (!D->bond_r0 || !D->bond_k)) || (D->n_angles && (!D->angle_theta0 || !D->angle_k)) ||
            (D->n_torsions && (!D->torsion_n || !D->torsion_k || !D->torsion_phi0)) ||
            (D->n_restraints && (!D->restraint_ref || !D->restraint_k)))
            return fail(nullptr, GPR_EINVAL, "missing term parameters");
        for (int t = 0; t < D->n_torsions; ++t)
            if (D->torsion_n[t] < 0 || D->torsion_n[t] > 12) return fail(nullptr, GPR_EINVAL, "torsion multiplicity outside [0, 12]");
        if (D->cutoff > 0 && (!(D->skin > 0) || !(D->eps_rf >= 1))) return fail(nullptr, GPR_EINVAL, "bad cutoff parameters");
    }
    const gpr_state_desc &st = D->state;
    if (st.kind == GPR_STATE_SIGN_X) {
        if (!idx_ok(st.atoms, 1, n)) return fail(nullptr, GPR_EINVAL, "bad state atom");
    } else if (st.kind == GPR_STATE_DIHEDRAL_BOXES) {
        if (!idx_ok(st.atoms, 8, n) || st.n_boxes < 1 || st.n_boxes > GPR_MAX_BOXES) return fail(nullptr, GPR_EINVAL, "bad state boxes");
    } else if (st.kind == GPR_STATE_COM_SPHERE) {
        if (st.n_group < 1 || !idx_ok(st.group, st.n_group, n)) return fail(nullptr, GPR_EINVAL, "bad state group");
    } else {
        return fail(nullptr, GPR_EINVAL, "bad state kind");
    }
    for (int j = 0; j < D->n_obs; ++j) {
        const gpr_obs_desc &o = D->obs[j];
        bool ok = true;
        switch (o.kind) {
        case GPR_OBS_COORD: ok = idx_ok(o.atoms, 1, n) && o.atoms[1] >= 0 && o.atoms[1] <= 2; break;
        case GPR_OBS_POTENTIAL: case GPR_OBS_KINETIC: break;
        case GPR_OBS_DIHEDRAL: ok = idx_ok(o.atoms, 4, n); break;
        case GPR_OBS_COM_DISTANCE: ok = o.n_a >= 1 && o.n_b >= 1 && idx_ok(o.group_a, o.n_a, n) && idx_ok(o.group_b, o.n_b, n); break;
        case GPR_OBS_RMS_VELOCITY: ok = o.n_a >= 1 && idx_ok(o.group_a, o.n_a, n); break;
        default: ok = false;
        }
        if (!ok) return fail(nullptr, GPR_EINVAL, "bad observable");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, GPR_EDEVICE, "no HIP device");
    gpr_system *S = new (std::nothrow) gpr_system();
    if (!S) return fail(nullptr, GPR_ENOMEM, "host allocation failed");
    gpr_status rc = create_impl(D, S);
    if (rc != GPR_OK) {
        g_thread_err = S->err;
        gpr_system_destroy(S);
        return rc;
    }
    *out = S;
    return GPR_OK;
}

extern "C" gpr_status gpr_set_stream(gpr_system *S, void *stream)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    HIPCHK(S, hipStreamSynchronize(S->stream));
    S->stream = (hipStream_t)stream;
    return GPR_OK;
}

extern "C" gpr_status gpr_set_path(gpr_system *S, int32_t path)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (path != GPR_PATH_PLAIN && path != GPR_PATH_PERSISTENT) return fail(S, GPR_EINVAL, "bad path");
    if (path == GPR_PATH_PERSISTENT && !S->persist_ok) return fail(S, GPR_EINVAL, "system too large for the persistent path");
    S->path = path;
    return GPR_OK;
}

extern "C" gpr_status gpr_set_launch(gpr_system *S, int32_t block_threads, int32_t groups_per_replica)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (groups_per_replica != 0 && groups_per_replica != 1 && groups_per_replica != 2 && groups_per_replica != 4 &&
        groups_per_replica != 8)
        return fail(S, GPR_EINVAL, "groups_per_replica must be 1, 2, 4 or 8");
    if (block_threads != 0 && (block_threads < 64 || block_threads > 1024 || block_threads % 64))
        return fail(S, GPR_EINVAL, "block_threads must be a multiple of 64 in [64, 1024]");
    const int bt = block_threads != 0 ? block_threads : S->bt_persist;
    {
        const int G = groups_per_replica != 0 ? groups_per_replica : S->groups;
        const size_t lds = persist_lds(S->n, S->np, make_split(S->work, S->n, S->np, G));
        if ((int)lds > S->maxlds_persist)
            return fail(S, GPR_EINVAL, "the per-workgroup LDS of this split exceeds the device limit");
        int per_cu = 0;
        HIPCHK(S, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_persist, bt, lds));
        if (per_cu < 1) return fail(S, GPR_EINVAL, "a workgroup of this shape does not fit on a compute unit");
    }
    drop_cycle_graphs(S);                                   // captured with the old shape
    S->bt_persist = bt;
    if (groups_per_replica != 0) {
        S->groups = groups_per_replica;
        S->split = make_split(S->work, S->n, S->np, groups_per_replica);
    }
    return GPR_OK;
}

// Launch-shape autotuner of the persistent path: every (threads per workgroup, workgroups per
// replica) shape that fits is timed over nsteps steps (after a short warm-up), starting each
// time from the same saved state; the fastest is kept.  The saved state (positions,
// velocities, forces, list-reference positions and ages, step counter) is put back at the end
// with every pair list marked for a rebuild, so the run continues exactly as without the call
// (results do not depend on the shape or on when lists are rebuilt).
extern "C" gpr_status gpr_autotune(gpr_system *S, int32_t nsteps, int32_t *block_threads, int32_t *groups)
{
    if (S) drop_cycle_graphs(S);                            // captured with the old shape
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (nsteps < 1) return fail(S, GPR_EINVAL, "nsteps < 1");
    if (!S->persist_ok) return fail(S, GPR_EINVAL, "system too large for the persistent path");
    const int R = S->R;
    const size_t m = (size_t)R * 3 * S->np;
    Dev &d = S->d;
    // saved state, in scratch freed when the call returns
    struct Scratch {
        std::vector<void *> p;
        ~Scratch() { for (void *q : p) (void)hipFree(q); }
        hipError_t get(void **out, size_t bytes)
        {
            const hipError_t e = hipMalloc(out, bytes);
            if (e == hipSuccess) p.push_back(*out);
            return e;
        }
    } scratch;
    float *sx = nullptr, *sv = nullptr, *sxb = nullptr;
    long long *sF = nullptr, *slb = nullptr;
    HIPCHK(S, scratch.get((void **)&sx, sizeof(float) * m));
    HIPCHK(S, scratch.get((void **)&sv, sizeof(float) * m));
    HIPCHK(S, scratch.get((void **)&sxb, sizeof(float) * m));
    HIPCHK(S, scratch.get((void **)&sF, sizeof(long long) * m));
    HIPCHK(S, scratch.get((void **)&slb, sizeof(long long) * 2 * R));
    auto copy_all = [&](bool save) -> hipError_t {
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        hipError_t e = hipMemcpyAsync(save ? sx : d.x, save ? d.x : sx, sizeof(float) * m, k, S->stream);
        if (!e) e = hipMemcpyAsync(save ? sv : d.v, save ? d.v : sv, sizeof(float) * m, k, S->stream);
        if (!e) e = hipMemcpyAsync(save ? sxb : d.xb, save ? d.xb : sxb, sizeof(float) * m, k, S->stream);
        if (!e) e = hipMemcpyAsync(save ? sF : d.F, save ? d.F : sF, sizeof(long long) * m, k, S->stream);
        if (!e) e = hipMemcpyAsync(save ? slb : d.last_build, save ? d.last_build : slb, sizeof(long long) * 2 * R, k, S->stream);
        if (!e && !save) {
            std::vector<int> ones(R, 1);
            e = hipMemcpyAsync(d.need_build, ones.data(), sizeof(int) * R, hipMemcpyHostToDevice, S->stream);
            if (!e) e = hipStreamSynchronize(S->stream);
        }
        return e;
    };
    HIPCHK(S, copy_all(true));
    const long long s_saved = S->s;
    const int path_saved = S->path, bt_saved = S->bt_persist, g_saved = S->groups;
    const Split sp_saved = S->split;
    int dev = 0, cus = 0;
    HIPCHK(S, hipGetDevice(&dev));
    HIPCHK(S, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipEvent_t e0, e1;
    HIPCHK(S, hipEventCreate(&e0));
    HIPCHK(S, hipEventCreate(&e1));
    float best = -1.f;
    int best_bt = bt_saved, best_g = g_saved;
    gpr_status rc = GPR_OK;
    S->path = GPR_PATH_PERSISTENT;
    for (int G = 1; G <= 8 && rc == GPR_OK; G *= 2) {
        const Split sp = make_split(S->work, S->n, S->np, G);
        const size_t lds = persist_lds(S->n, S->np, sp);
        if ((int)lds > S->maxlds_persist) continue;
        for (int bt = 256; bt <= 1024 && rc == GPR_OK; bt += 256) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_persist, bt, lds) != hipSuccess ||
                per_cu < 1 || (G > 1 && per_cu * cus < G))
                continue;
            S->bt_persist = bt; S->groups = G; S->split = sp;
            hipError_t he = copy_all(false);
            if (he) { rc = fail(S, GPR_EDEVICE, std::string("autotune restore: ") + hipGetErrorString(he)); break; }
            S->s = s_saved;
            rc = run_steps(S, R, std::min(20, nsteps), 0, false, false);
            if (rc) break;
            HIPCHK(S, hipEventRecord(e0, S->stream));
            rc = run_steps(S, R, nsteps, 0, false, false);
            if (rc) break;
            HIPCHK(S, hipEventRecord(e1, S->stream));
            HIPCHK(S, hipEventSynchronize(e1));
            int err[4];
            HIPCHK(S, hipMemcpy(err, d.err, sizeof err, hipMemcpyDeviceToHost));
            if (err[ERR_UNSTABLE] || err[ERR_BARRIER] || err[ERR_LIST]) { rc = fail(S, GPR_EDEVICE, "autotune run failed"); break; }
            float ms = 0.f;
            HIPCHK(S, hipEventElapsedTime(&ms, e0, e1));
            if (best < 0.f || ms < best) { best = ms; best_bt = bt; best_g = G; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // back to the saved state with the chosen shape
    S->path = path_saved;
    S->s = s_saved;
    HIPCHK(S, copy_all(false));
    if (rc) {
        S->bt_persist = bt_saved; S->groups = g_saved; S->split = sp_saved;
        return rc;
    }
    S->bt_persist = best_bt;
    S->groups = best_g;
    S->split = make_split(S->work, S->n, S->np, best_g);
    if (block_threads) *block_threads = best_bt;
    if (groups) *groups = best_g;
    return GPR_OK;
}

extern "C" gpr_status gpr_set_cycles(gpr_system *S, int32_t cycles)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (cycles < 0 || cycles > 4096) return fail(S, GPR_EINVAL, "cycles must be in [0, 4096]");
    if (cycles > 0 && !S->persist_ok) return fail(S, GPR_EINVAL, "system too large for the persistent path");
    if (cycles == S->cycles) return GPR_OK;
    drop_cycle_graphs(S);
    if (S->stc_dev) { (void)hipFree(S->stc_dev); S->stc_dev = nullptr; }
    if (S->stc_host) { (void)hipHostFree(S->stc_host); S->stc_host = nullptr; }
    S->cycles = 0;
    if (cycles == 0) return GPR_OK;
    if (!S->cyc_dev) HIPCHK(S, hipMalloc((void **)&S->cyc_dev, sizeof(CycRec)));
    if (!S->cyc_host) HIPCHK(S, hipHostMalloc((void **)&S->cyc_host, sizeof(CycRec), hipHostMallocDefault));
    HIPCHK(S, hipMalloc((void **)&S->stc_dev, sizeof(Status) * cycles));
    HIPCHK(S, hipHostMalloc((void **)&S->stc_host, sizeof(Status) * cycles, hipHostMallocDefault));
    S->cycles = cycles;
    return GPR_OK;
}

extern "C" gpr_status gpr_set_graph(gpr_system *S, int32_t cycle_steps)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (cycle_steps < 0 || cycle_steps > 10000) return fail(S, GPR_EINVAL, "cycle_steps must be in [0, 10000]");
    if (cycle_steps != S->graph_cycle) {
        HIPCHK(S, hipStreamSynchronize(S->stream));
        for (auto &g : S->graphs) (void)hipGraphExecDestroy(g.exec);
        S->graphs.clear();
        S->graph_cycle = cycle_steps;
    }
    return GPR_OK;
}

extern "C" gpr_status gpr_profile(gpr_system *S, int32_t enable)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    HIPCHK(S, hipStreamSynchronize(S->stream));
    HIPCHK(S, prof_collect(S));
    S->prof = enable != 0;
    S->prof_ms = 0.0;
    S->prof_n = 0;
    while (S->prof && S->ev_a.size() < 8) HIPCHK(S, prof_add_pair(S));
    return GPR_OK;
}

extern "C" gpr_status gpr_profile_read(gpr_system *S, double *ms, int64_t *launches)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    HIPCHK(S, hipStreamSynchronize(S->stream));
    HIPCHK(S, prof_collect(S));
    if (ms) *ms = S->prof_ms;
    if (launches) *launches = S->prof_n;
    return GPR_OK;
}

extern "C" gpr_status gpr_phase_read(gpr_system *S, double *out)
{
    if (!S || !out) return fail(S, GPR_EINVAL, "NULL argument");
    HIPCHK(S, hipStreamSynchronize(S->stream));
    std::vector<unsigned long long> acc((size_t)S->R * PHASE_MAX_G * NPHASE);
    const hipError_t e = phase_take(acc.data(), S->R, S->stream);
    if (e == hipErrorNotSupported) return fail(S, GPR_EINVAL, "library built without the phase timers");
    HIPCHK(S, e);
    int dev = 0, khz = 0;
    HIPCHK(S, hipGetDevice(&dev));
    HIPCHK(S, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return fail(S, GPR_EDEVICE, "no wall-clock rate");
    const double us_per_tick = 1000.0 / (double)khz;
    unsigned long long t0 = ~0ull;                        // the earliest start of the last launches
    for (size_t k = PH_START; k < acc.size(); k += NPHASE)
        if (acc[k]) t0 = std::min(t0, acc[k]);
    for (size_t k = 0; k < acc.size(); ++k) {
        const size_t slot = k % NPHASE;
        if (slot < PH_NSTEP) out[k] = (double)acc[k] * us_per_tick;
        else if (slot < PH_START) out[k] = (double)acc[k];
        else out[k] = acc[k] ? (double)(acc[k] - t0) * us_per_tick : 0.0;
    }
    return GPR_OK;
}

// ------------------------------------------------------------------ queries
extern "C" double gpr_simulated_time(const gpr_system *S) { return S ? (double)S->tsim * S->dt : NAN; }
extern "C" int64_t gpr_simulated_steps(const gpr_system *S) { return S ? S->tsim : -1; }
extern "C" int64_t gpr_global_step(const gpr_system *S) { return S ? S->s : -1; }
extern "C" int32_t gpr_current_state(const gpr_system *S) { return S ? S->omega : INT32_MIN; }
extern "C" int64_t gpr_advance_steps(const gpr_system *S) { return S ? S->adv_t : -1; }

extern "C" gpr_status gpr_energy_forces(gpr_system *S, int32_t r0, int32_t nr, double *energy, double *forces)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (r0 < 0 || nr < 0 || r0 + nr > S->R) return fail(S, GPR_EINVAL, "replica range");
    if (nr == 0) return GPR_OK;
    gpr_status rc = launch_forces(S, r0, nr, -1, 1, 0, 1);
    if (rc) return rc;
    std::vector<long long> F((size_t)nr * 3 * S->np), E(nr);
    HIPCHK(S, hipMemcpyAsync(F.data(), S->d.F + (size_t)r0 * 3 * S->np, F.size() * 8, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipMemcpyAsync(E.data(), S->d.E + r0, E.size() * 8, hipMemcpyDeviceToHost, S->stream));
    int err[4];
    HIPCHK(S, hipMemcpyAsync(err, S->d.err, sizeof err, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
    if (err[ERR_LIST]) return fail(S, GPR_EDEVICE, "pair-list capacity exceeded");
    for (int k = 0; k < nr; ++k) {
        if (energy) energy[k] = (double)E[k] * FIX_INV;
        if (forces)
            for (int c = 0; c < 3; ++c)
                for (int i = 0; i < S->n; ++i)
                    forces[((size_t)k * 3 + c) * S->n + i] = (double)F[((size_t)k * 3 + c) * S->np + i] * FIX_INV;
    }
    return GPR_OK;
}

extern "C" gpr_status gpr_set_params(gpr_system *S, const double *epsilon, const double *sigma, const double *charge,
                                     const double *torsion_k)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (S->kind != GPR_KIND_MOLECULAR) return fail(S, GPR_EINVAL, "force-field parameters need a molecular system");
    const int n = S->n, nt = (int)S->tor_k_h.size();
    for (int i = 0; i < n; ++i) {
        if (epsilon && !(epsilon[i] >= 0 && std::isfinite(epsilon[i]))) return fail(S, GPR_EINVAL, "epsilon < 0 or not finite");
        if (sigma && !(sigma[i] >= 0 && std::isfinite(sigma[i]))) return fail(S, GPR_EINVAL, "sigma < 0 or not finite");
        if (charge && !std::isfinite(charge[i])) return fail(S, GPR_EINVAL, "charge not finite");
    }
    for (int t = 0; t < nt; ++t)
        if (torsion_k && !std::isfinite(torsion_k[t])) return fail(S, GPR_EINVAL, "torsion k not finite");
    if (epsilon) S->eps_h.assign(epsilon, epsilon + n);
    if (sigma) S->sig_h.assign(sigma, sigma + n);
    if (charge) S->q_h.assign(charge, charge + n);
    if (torsion_k) S->tor_k_h.assign(torsion_k, torsion_k + nt);
    HIPCHK(S, write_params(S));
    // the forces the integrator carries must belong to the new parameters
    gpr_status rc = launch_forces(S, 0, S->R, -1, 1, 0, 1);
    if (rc) return rc;
    HIPCHK(S, hipStreamSynchronize(S->stream));
    return GPR_OK;
}

extern "C" gpr_status gpr_energy_forces_dev(gpr_system *S, const float *x_dev, double *energy_dev, float *forces_dev)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (!x_dev) return fail(S, GPR_EINVAL, "NULL positions");
    const int n = S->n, np = S->np, R = S->R;
    HIPCHK(S, hipMemcpy2DAsync(S->d.x, sizeof(float) * np, x_dev, sizeof(float) * n, sizeof(float) * n, (size_t)3 * R,
                               hipMemcpyDeviceToDevice, S->stream));
    gpr_status rc = launch_forces(S, 0, R, -1, 1, 0, 1);
    if (rc) return rc;
    hipLaunchKernelGGL(k_unfix_out, dim3((n + 255) / 256, R), dim3(256), 0, S->stream, S->d_dev, energy_dev, forces_dev);
    LAUNCHCHK(S);
    int err[4];
    HIPCHK(S, hipMemcpyAsync(err, S->d.err, sizeof err, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
    if (err[ERR_LIST]) return fail(S, GPR_EDEVICE, "pair-list capacity exceeded");
    return GPR_OK;
}

extern "C" gpr_status gpr_energy_backward_dev(gpr_system *S, const double *w_dev, float *d_x, double *d_eps,
                                              double *d_sigma, double *d_charge, double *d_torsion_k)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (!w_dev) return fail(S, GPR_EINVAL, "NULL weights");
    const bool params = d_eps || d_sigma || d_charge || d_torsion_k;
    if (params && S->kind != GPR_KIND_MOLECULAR) return fail(S, GPR_EINVAL, "force-field parameters need a molecular system");
    if (d_eps)
        for (double e : S->eps_h)
            if (!(e > 0)) return fail(S, GPR_EINVAL, "the epsilon gradient needs every epsilon > 0");
    const int n = S->n, np = S->np, R = S->R, nt = S->d.tp.nt, n14 = S->d.tp.n14;
    if (d_x) {
        hipLaunchKernelGGL(k_weighted_dx, dim3((n + 255) / 256, R), dim3(256), 0, S->stream, S->d_dev, w_dev, d_x);
        LAUNCHCHK(S);
    }
    if (params) {
        HIPCHK(S, hipMemsetAsync(S->d.gacc, 0, sizeof(long long) * ((size_t)3 * np + std::max(1, nt)), S->stream));
        hipLaunchKernelGGL(k_grad_nb, dim3((n * P + 1023) / 1024, R), dim3(1024), S->lds_nb, S->stream, S->d_dev, w_dev);
        LAUNCHCHK(S);
        const int nterm = std::max(nt, n14);
        if (nterm > 0) {
            hipLaunchKernelGGL(k_grad_terms, dim3((nterm + 255) / 256, R), dim3(256), 0, S->stream, S->d_dev, w_dev);
            LAUNCHCHK(S);
        }
        hipLaunchKernelGGL(k_grad_finish, dim3((std::max(n, nt) + 255) / 256), dim3(256), 0, S->stream, S->d_dev, d_eps,
                           d_sigma, d_charge, d_torsion_k);
        LAUNCHCHK(S);
    }
    HIPCHK(S, hipStreamSynchronize(S->stream));
    return GPR_OK;
}

extern "C" gpr_status gpr_get_state(const gpr_system *Sc, int32_t r, double *q, double *v)
{
    gpr_system *S = const_cast<gpr_system *>(Sc);
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (r < 0 || r >= S->R) return fail(S, GPR_EINVAL, "replica index");
    std::vector<float> x(3 * S->np), vv(3 * S->np);
    HIPCHK(S, hipMemcpyAsync(x.data(), S->d.x + (size_t)r * 3 * S->np, x.size() * 4, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipMemcpyAsync(vv.data(), S->d.v + (size_t)r * 3 * S->np, vv.size() * 4, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < S->n; ++i) {
            if (q) q[c * S->n + i] = x[c * S->np + i];
            if (v) v[c * S->n + i] = vv[c * S->np + i];
        }
    return GPR_OK;
}

extern "C" gpr_status gpr_set_state(gpr_system *S, int32_t r, const double *q, const double *v)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (r < 0 || r >= S->R || !q) return fail(S, GPR_EINVAL, "replica index or NULL positions");
    std::vector<float> x(3 * S->np, 0.f), vv(3 * S->np, 0.f);
    if (!v) {
        HIPCHK(S, hipMemcpyAsync(vv.data(), S->d.v + (size_t)r * 3 * S->np, vv.size() * 4, hipMemcpyDeviceToHost, S->stream));
        HIPCHK(S, hipStreamSynchronize(S->stream));
    }
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < S->n; ++i) {
            x[c * S->np + i] = (float)q[c * S->n + i];
            if (v) vv[c * S->np + i] = (float)v[c * S->n + i];
        }
    if (S->kind == GPR_KIND_TOY2D) { x[2 * S->np] = 0.f; vv[2 * S->np] = 0.f; }
    HIPCHK(S, hipMemcpyAsync(S->d.x + (size_t)r * 3 * S->np, x.data(), x.size() * 4, hipMemcpyHostToDevice, S->stream));
    HIPCHK(S, hipMemcpyAsync(S->d.v + (size_t)r * 3 * S->np, vv.data(), vv.size() * 4, hipMemcpyHostToDevice, S->stream));
    gpr_status rc = launch_forces(S, r, 1, -1, 1, 0, 1);
    if (rc) return rc;
    HIPCHK(S, hipStreamSynchronize(S->stream));
    S->phase = PH_IDLE;
    return GPR_OK;
}

extern "C" gpr_status gpr_get_accumulators(const gpr_system *Sc, int64_t *n, double *S1, double *S2, double *shift)
{
    gpr_system *S = const_cast<gpr_system *>(Sc);
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    std::vector<double> acc((size_t)S->R * MAX_OBS * 2), sh(MAX_OBS);
    HIPCHK(S, hipMemcpyAsync(acc.data(), S->d.acc, acc.size() * 8, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipMemcpyAsync(sh.data(), S->d.shift, sh.size() * 8, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
    if (n) *n = S->nsamp;
    for (int r = 0; r < S->R; ++r)
        for (int j = 0; j < S->nobs; ++j) {
            if (S1) S1[r * S->nobs + j] = acc[((size_t)r * MAX_OBS + j) * 2];
            if (S2) S2[r * S->nobs + j] = acc[((size_t)r * MAX_OBS + j) * 2 + 1];
        }
    if (shift) for (int j = 0; j < S->nobs; ++j) shift[j] = sh[j];
    return GPR_OK;
}

extern "C" gpr_status gpr_observe(gpr_system *S, double *obs, int32_t *state)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (S->d.need_energy) {
        gpr_status rc = launch_forces(S, 0, S->R, -1, 1, 0, 1);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_obs, dim3(S->R), dim3(256), S->lds_stage, S->stream, S->d_dev, 0, 2, S->obs_out, 0);
    LAUNCHCHK(S);
    hipLaunchKernelGGL(k_state, dim3(S->R), dim3(256), S->lds_stage, S->stream, S->d_dev, 0);
    LAUNCHCHK(S);
    std::vector<double> h((size_t)S->R * MAX_OBS);
    std::vector<int> st(S->R);
    HIPCHK(S, hipMemcpyAsync(h.data(), S->obs_out, h.size() * 8, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipMemcpyAsync(st.data(), S->d.state, st.size() * 4, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
    for (int r = 0; r < S->R; ++r) {
        if (obs) for (int j = 0; j < S->nobs; ++j) obs[r * S->nobs + j] = h[(size_t)r * MAX_OBS + j];
        if (state) state[r] = st[r];
    }
    return GPR_OK;
}

// ------------------------------------------------------------------ Gen.ParRep steps
// Each call (transient propagation, convergence step, parallel step; Fig. 1) is a loop of
// chunks of steps, each ending at or before the call's next exit check, followed by that
// check.  PhaseRun holds one call in progress, so that the single-system calls and
// gpr_batch_run (several systems whose chunks share persistent launches) run one logic.
namespace {
struct PhaseRun {
    int op = 0;                          // GPR_OP_*
    long long t_corr = 0, budget = 0;    // budget: steps (transient, convergence) or checks (parallel)
    long long taken = 0;                 // steps (or checks) taken in this call
    bool done = false;
    gpr_status rc = GPR_OK;              // when done: GPR_OK (result written) or GPR_BUDGET
    gpr_event ev{};
    gpr_dephase_out dout{};
    gpr_exit_out pout{};
};
struct Chunk {
    int nrep;                            // replicas stepped
    long long k, t0;                     // steps; local step count at the start (sampling phase)
    bool sample, at_check;               // workers' observables every t_GR; the chunk ends at a check
};
} // namespace

static gpr_status phase_begin(gpr_system *S, PhaseRun &p)
{
    gpr_status rc;
    if (p.op == GPR_OP_DECORRELATE) {
        if (S->phase != PH_DECORR) {
            int st0 = -1;
            rc = state_of_ref(S, &st0);
            if (rc) return rc;
            S->phase = PH_DECORR;
            S->dc_omega = st0;
            S->dc_from = st0;
            S->dc_resid = 0;
            S->dc_steps = 0;
        }
    } else if (p.op == GPR_OP_DEPHASE) {
        if (S->phase != PH_DEPHASE) {
            if (S->omega == -1) return fail(S, GPR_EPHASE, "reference walker is in no state");
            rc = broadcast_reference(S);
            if (rc) return rc;
            HIPCHK(S, hipMemsetAsync(S->d.acc, 0, sizeof(double) * S->R * MAX_OBS * 2, S->stream));
            if (S->d.need_energy) {
                rc = launch_forces(S, 0, 1, -1, 1, 0, 1);
                if (rc) return rc;
            }
            hipLaunchKernelGGL(k_obs, dim3(1), dim3(256), S->lds_stage, S->stream, S->d_dev, 0, 1, nullptr, 0);
            LAUNCHCHK(S);
            S->nsamp = 0;
            S->dp_t = 0;
            S->n_branch = 0;
            S->phase = PH_DEPHASE;
        }
    } else if (p.op == GPR_OP_PARALLEL_STEP) {
        if (S->phase == PH_CONVERGED) { S->phase = PH_PARALLEL; S->par_M = 0; S->par_t = 0; }
        else if (S->phase != PH_PARALLEL) return fail(S, GPR_EPHASE, "parallel step needs a converged dephasing");
    } else {
        return fail(S, GPR_EINVAL, "unknown Gen.ParRep step");
    }
    return GPR_OK;
}

// decisions taken before any further step: residence reached, or the budget spent
static void phase_ready(gpr_system *S, PhaseRun &p)
{
    if (p.done) return;
    if (p.op == GPR_OP_DECORRELATE && S->dc_omega != -1 && S->dc_resid >= p.t_corr) {
        S->omega = S->dc_omega;
        S->phase = PH_IDLE;
        p.ev.kind = GPR_EV_RESIDENT; p.ev.from_state = S->dc_from; p.ev.to_state = S->dc_omega; p.ev.pad = 0;
        p.ev.resident_steps = S->dc_resid; p.ev.steps_taken = S->dc_steps;
        p.done = true; p.rc = GPR_OK;
        return;
    }
    if (p.taken >= p.budget) { p.done = true; p.rc = GPR_BUDGET; }
}

// the next chunk, at most kmax steps
static Chunk phase_chunk(const gpr_system *S, const PhaseRun &p, long long kmax)
{
    Chunk c{};
    if (p.op == GPR_OP_DECORRELATE) {
        const long long pos = S->dc_steps % S->tcd;
        c.nrep = 1; c.k = S->tcd - pos; c.t0 = 0; c.sample = false;
        c.k = std::min(c.k, kmax);
        c.at_check = pos + c.k == S->tcd;
    } else if (p.op == GPR_OP_DEPHASE) {
        const long long pos = S->dp_t % S->tcd;
        c.nrep = S->R; c.t0 = S->dp_t; c.sample = true;
        c.k = std::min(std::min<long long>(S->tcd - pos, p.budget - p.taken), kmax);
        c.at_check = pos + c.k == S->tcd;
    } else {
        c.nrep = S->R; c.t0 = 0; c.sample = false;
        c.k = std::min<long long>(S->tcp - S->par_t, kmax);
        c.at_check = S->par_t + c.k == S->tcp;
    }
    return c;
}

// bookkeeping after a chunk of c.k steps (the steps themselves already taken), then, when
// the chunk ends at a check, the decision the check's status leads to: the status comes from
// running the check (st == nullptr) or from a replay of captured check cycles
static gpr_status phase_advance(gpr_system *S, PhaseRun &p, const Chunk &c, const Status *stc = nullptr)
{
    gpr_status rc;
    if (p.op == GPR_OP_DECORRELATE) {
        S->tsim += c.k;
        p.taken += c.k;
        S->dc_steps += c.k;
        if (!c.at_check) return GPR_OK;
        rc = check(S, CHK_STATE, 1, 0);
        if (rc) return rc;
        const int st = S->st_host->to_state;
        if (st == S->dc_omega) {
            S->dc_resid += S->tcd;
        } else if (S->dc_omega == -1) {
            S->dc_omega = st;              // entered a state: the reaching time ends here
            S->dc_resid = 0;
        } else {
            p.ev.kind = GPR_EV_EXITED; p.ev.from_state = S->dc_omega; p.ev.to_state = st; p.ev.pad = 0;
            p.ev.resident_steps = S->dc_resid + S->tcd; p.ev.steps_taken = S->dc_steps;
            S->omega = st;
            S->phase = PH_IDLE;
            p.done = true; p.rc = GPR_OK;
        }
        return GPR_OK;
    }
    if (p.op == GPR_OP_DEPHASE) {
        S->nsamp += count_samples(S->dp_t, S->dp_t + c.k, S->t_gr);
        S->dp_t += c.k;
        p.taken += c.k;
        if (!c.at_check) return GPR_OK;
        if (!stc) {
            rc = check(S, CHK_DEPHASE, S->R, 0);
            if (rc) return rc;
        }
        const Status &st = stc ? *stc : *S->st_host;
        gpr_dephase_out &o = p.dout;
        if (st.ref_exited) {
            S->tsim += S->dp_t;
            o.outcome = GPR_DEPHASE_REF_EXITED; o.to_state = st.to_state; o.t_steps = S->dp_t;
            o.n_branch = S->n_branch; o.n_samples = S->nsamp;
            for (int j = 0; j < GPR_MAX_OBS; ++j) o.rhat[j] = j < S->nobs ? st.rhat[j] : 0.0;
            S->omega = st.to_state;
            S->phase = PH_IDLE;
            p.done = true; p.rc = GPR_OK;
            return GPR_OK;
        }
        if (st.n_surv == 0 && S->R > 1) {
            S->n_branch += S->R - 1;
            S->nsamp = 0;
        } else {
            S->n_branch += st.n_exited;
        }
        bool conv = S->dp_t >= S->t_min && S->nsamp >= 2;
        for (int j = 0; j < S->nobs && conv; ++j) conv = st.rhat[j] < 1.0 + S->tol;
        if (conv) {
            S->tsim += S->dp_t;
            o.outcome = GPR_DEPHASE_CONVERGED; o.to_state = S->omega; o.t_steps = S->dp_t;
            o.n_branch = S->n_branch; o.n_samples = S->nsamp;
            for (int j = 0; j < GPR_MAX_OBS; ++j) o.rhat[j] = j < S->nobs ? st.rhat[j] : 0.0;
            S->phase = PH_CONVERGED;
            p.done = true; p.rc = GPR_OK;
        }
        return GPR_OK;
    }
    // parallel step
    S->par_t += c.k;
    if (!c.at_check) return GPR_OK;
    S->par_t = 0;
    S->par_M += 1;
    p.taken += 1;
    if (!stc) {
        rc = check(S, CHK_PARALLEL, S->R, S->par_M);
        if (rc) return rc;
    }
    const Status &st = stc ? *stc : *S->st_host;
    const int k = st.k;
    if (k == 0) return GPR_OK;
    // M, k and tau of Eq. 5, voted on the device
    const long long tau = st.tau;
    S->tsim += tau;
    if (k != 1) {
        rc = copy_replica(S, 0, k - 1);
        if (rc) return rc;
    }
    gpr_exit_out &o = p.pout;
    o.M = st.M; o.k = k; o.to_state = st.to_state; o.tau_steps = tau; o.tau = (double)tau * S->dt;
    S->omega = st.to_state;
    S->phase = PH_IDLE;
    HIPCHK(S, hipStreamSynchronize(S->stream));
    p.done = true; p.rc = GPR_OK;
    return GPR_OK;
}

static gpr_status run_cycles(gpr_system *S, PhaseRun &p, bool &ran);

static gpr_status run_phase(gpr_system *S, PhaseRun &p)
{
    gpr_status rc = phase_begin(S, p);
    if (rc) return rc;
    for (;;) {
        phase_ready(S, p);
        if (p.done) return p.rc;
        bool ran = false;
        rc = run_cycles(S, p, ran);
        if (rc) return rc;
        if (ran) continue;
        const Chunk c = phase_chunk(S, p, 1LL << 62);
        rc = run_steps(S, c.nrep, c.k, c.t0, c.sample, c.at_check);
        if (rc) return rc;
        rc = phase_advance(S, p, c);
        if (rc) return rc;
        if (p.done) return p.rc;
    }
}

static void drop_cycle_graphs(gpr_system *S)
{
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    for (auto &g : S->cgraphs) (void)hipGraphExecDestroy(g.exec);
    S->cgraphs.clear();
}

// The captured run of S->cycles check cycles of the convergence step (op GPR_OP_DEPHASE) or
// the parallel step on the persistent path, captured on a stream of its own the first time
// it is needed.  Per cycle: the replicas' barrier counters cleared by a kernel, the persistent
// launch(es) of one check period with the state test at the end, then the check with its
// clone-on-kill copies.  Steps, check indices and Omega come from the cycle record, which the
// host writes before each replay.
static gpr_status cycle_graph(gpr_system *S, int op, hipGraphExec_t *out)
{
    for (auto &g : S->cgraphs)
        if (g.op == op) { *out = g.exec; return GPR_OK; }
    const int nrep = S->R;
    const bool dep = op == GPR_OP_DEPHASE;
    const int nsteps = dep ? S->tcd : S->tcp;
    PersistBatch pb{};
    pb.nitems = 1;
    int nblocks = 0;
    const size_t lds = persist_lds(S->n, S->np, S->split);
    gpr_status rc = persist_item(S, nrep, S->bt_persist, lds, -1, pb.it[0], nblocks);
    if (rc) return rc;
    const int rounds = (nrep + pb.it[0].nsets - 1) / pb.it[0].nsets;
    rc = check_layout(S, pb, nblocks, S->bt_persist, true);
    if (rc) return rc;
    const dim3 cgrid = dep ? dim3((3 * S->np + 255) / 256, nrep) : dim3(1, 1);
    hipStream_t cs = nullptr;
    HIPCHK(S, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (int j = 0; j < S->cycles && e == hipSuccess; ++j) {
        PersistItem it = pb.it[0];
        it.s0 = 0; it.t0 = 0; it.nsteps = nsteps; it.sample = dep ? 1 : 0; it.state_end = 1;
        it.cyc = S->cyc_dev;
        it.cycle = j;
        for (int k = 0; k < rounds && e == hipSuccess; ++k) {
            it.roff = k * it.nsets;
            void *args[] = {(void *)&it};
            e = hipLaunchKernel((const void *)k_persist, dim3(nblocks), dim3(S->bt_persist), args, lds, cs);
        }
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_check, cgrid, dim3(256), sizeof(int) * nrep, cs, S->d_dev, dep ? CHK_DEPHASE : CHK_PARALLEL,
                           0LL, 0, nrep, 0LL, 0LL, (long long)S->tcp, S->stc_dev, S->donor, S->surv, S->fec, S->cyc_dev, j);
        e = hipGetLastError();
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipSuccess;
    if (e == hipSuccess && e2 == hipSuccess) e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return fail(S, GPR_EDEVICE, std::string("check-cycle capture: ") +
                                        hipGetErrorString(e != hipSuccess ? e : e2 != hipSuccess ? e2 : e3));
    S->cgraphs.push_back({op, ex});
    *out = ex;
    return GPR_OK;
}

// S->cycles check cycles replayed from the captured graph, when the call stands at a check
// boundary with room in its budget for all of them; then the host takes, cycle by cycle, the
// decision each status leads to, exactly as after a check it runs itself, and verifies that
// the call ends at the cycle the device stopped at.
static gpr_status run_cycles(gpr_system *S, PhaseRun &p, bool &ran)
{
    ran = false;
    const int C = S->cycles;
    if (C <= 0 || S->path != GPR_PATH_PERSISTENT || (p.op != GPR_OP_DEPHASE && p.op != GPR_OP_PARALLEL_STEP))
        return GPR_OK;
    const bool dep = p.op == GPR_OP_DEPHASE;
    const long long per = dep ? S->tcd : S->tcp;
    if (dep ? (S->dp_t % S->tcd != 0 || p.budget - p.taken < C * per) : (S->par_t != 0 || p.budget - p.taken < C))
        return GPR_OK;
    hipGraphExec_t ex = nullptr;
    gpr_status rc = cycle_graph(S, p.op, &ex);
    if (rc) return rc;
    CycRec &h = *S->cyc_host;
    h.s_start = S->s; h.t_start = dep ? S->dp_t : 0; h.M_start = S->par_M; h.nsamp = S->nsamp;
    h.nsteps = (int)per; h.halt_cycle = NO_HALT; h.omega = S->omega; h.pad = 0;
    HIPCHK(S, hipMemcpyAsync(S->cyc_dev, S->cyc_host, sizeof(CycRec), hipMemcpyHostToDevice, S->stream));
    HIPCHK(S, hipGraphLaunch(ex, S->stream));
    HIPCHK(S, hipMemcpyAsync(S->stc_host, S->stc_dev, sizeof(Status) * C, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipMemcpyAsync(S->cyc_host, S->cyc_dev, sizeof(CycRec), hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
    ran = true;
    const int halt = S->cyc_host->halt_cycle;
    const int ncyc = halt == NO_HALT ? C : halt + 1;
    for (int j = 0; j < ncyc; ++j) {
        const Status &st = S->stc_host[j];
        rc = status_errors(S, st);
        if (rc) return rc;
        Chunk c{};
        c.nrep = S->R; c.k = per; c.t0 = dep ? S->dp_t : 0; c.sample = dep; c.at_check = true;
        S->s += per;
        rc = phase_advance(S, p, c, &st);
        if (rc) return rc;
        if (p.done != (j == halt)) return fail(S, GPR_EDEVICE, "check cycles: device and host disagree on the end of the call");
        if (p.done) break;
    }
    return GPR_OK;
}

extern "C" gpr_status gpr_decorrelate(gpr_system *S, int64_t t_corr, int64_t max_steps, gpr_event *ev)
{
    if (!S || !ev) return fail(S, GPR_EINVAL, "NULL argument");
    PhaseRun p;
    p.op = GPR_OP_DECORRELATE; p.t_corr = t_corr; p.budget = max_steps;
    const gpr_status rc = run_phase(S, p);
    if (rc == GPR_OK) *ev = p.ev;
    return rc;
}

extern "C" gpr_status gpr_dephase(gpr_system *S, int64_t max_steps, gpr_dephase_out *o)
{
    if (!S || !o) return fail(S, GPR_EINVAL, "NULL argument");
    PhaseRun p;
    p.op = GPR_OP_DEPHASE; p.budget = max_steps;
    const gpr_status rc = run_phase(S, p);
    if (rc == GPR_OK) *o = p.dout;
    return rc;
}

// copies the (x, v, F) of one replica between the system and a replica-sized buffer set
static gpr_status move_replica(gpr_system *S, float *dx, float *dv, long long *dF, const float *sx, const float *sv,
                               const long long *sF)
{
    const size_t m = (size_t)3 * S->np;
    HIPCHK(S, hipMemcpyAsync(dx, sx, sizeof(float) * m, hipMemcpyDeviceToDevice, S->stream));
    HIPCHK(S, hipMemcpyAsync(dv, sv, sizeof(float) * m, hipMemcpyDeviceToDevice, S->stream));
    HIPCHK(S, hipMemcpyAsync(dF, sF, sizeof(long long) * m, hipMemcpyDeviceToDevice, S->stream));
    return GPR_OK;
}

extern "C" gpr_status gpr_dephase_fixed(gpr_system *S, int64_t t_phase, int64_t max_steps, gpr_dephase_out *o)
{
    if (!S || !o) return fail(S, GPR_EINVAL, "NULL argument");
    const int R = S->R;
    const size_t m = (size_t)3 * S->np;
    Dev &d = S->d;
    gpr_status rc;
    if (S->phase != PH_DEPHASE_FIXED) {
        if (S->omega == -1) return fail(S, GPR_EPHASE, "reference walker is in no state");
        if (t_phase < 0) return fail(S, GPR_EINVAL, "t_phase < 0");
        if (!S->snap_x) {
            HIPCHK(S, dalloc(S, &S->snap_x, m)); HIPCHK(S, dalloc(S, &S->snap_v, m)); HIPCHK(S, dalloc(S, &S->snap_F, m));
            HIPCHK(S, dalloc(S, &S->samp_x, m * R)); HIPCHK(S, dalloc(S, &S->samp_v, m * R));
            HIPCHK(S, dalloc(S, &S->samp_F, m * R));
        }
        rc = move_replica(S, S->snap_x, S->snap_v, S->snap_F, d.x, d.v, d.F);
        if (rc) return rc;
        rc = broadcast_reference(S);
        if (rc) return rc;
        S->resid.assign(R, 0);
        S->done.assign(R, 0);
        S->dp_t = 0;
        S->n_branch = 0;
        S->phase = PH_DEPHASE_FIXED;
    }
    const int one = 1;
    std::vector<int> st(R);
    long long taken = 0;
    while (taken < max_steps) {
        const long long k = std::min<long long>(S->tcd - S->dp_t % S->tcd, max_steps - taken);
        const bool at_check = (S->dp_t + k) % S->tcd == 0;
        rc = run_steps(S, R, k, S->dp_t, false, at_check);
        if (rc) return rc;
        S->dp_t += k;
        taken += k;
        if (!at_check) break;
        HIPCHK(S, hipMemcpyAsync(st.data(), d.state, sizeof(int) * R, hipMemcpyDeviceToHost, S->stream));
        int err[4];
        HIPCHK(S, hipMemcpyAsync(err, d.err, sizeof err, hipMemcpyDeviceToHost, S->stream));
        HIPCHK(S, hipStreamSynchronize(S->stream));
        if (err[ERR_UNSTABLE]) return fail(S, GPR_EUNSTABLE, "non-finite or overflowing state");
        if (err[ERR_BARRIER]) return fail(S, GPR_EDEVICE, "persistent kernel barrier timed out");
        if (err[ERR_LIST]) return fail(S, GPR_EDEVICE, "pair-list capacity exceeded");
        bool all = true;
        for (int r = 0; r < R; ++r) {
            if (S->done[r]) continue;
            const size_t b = (size_t)r * m;
            if (st[r] != S->omega) {
                rc = move_replica(S, d.x + b, d.v + b, d.F + b, S->snap_x, S->snap_v, S->snap_F);
                if (rc) return rc;
                HIPCHK(S, hipMemcpyAsync(d.need_build + r, &one, sizeof(int), hipMemcpyHostToDevice, S->stream));
                S->resid[r] = 0;
                S->n_branch += 1;
                all = false;
            } else if ((S->resid[r] += S->tcd) >= t_phase) {
                rc = move_replica(S, S->samp_x + b, S->samp_v + b, S->samp_F + b, d.x + b, d.v + b, d.F + b);
                if (rc) return rc;
                S->done[r] = 1;
            } else {
                all = false;
            }
        }
        if (all) {
            for (int r = 0; r < R; ++r) {
                const size_t b = (size_t)r * m;
                rc = move_replica(S, d.x + b, d.v + b, d.F + b, S->samp_x + b, S->samp_v + b, S->samp_F + b);
                if (rc) return rc;
            }
            std::vector<int> ones(R, 1);
            HIPCHK(S, hipMemcpyAsync(d.need_build, ones.data(), sizeof(int) * R, hipMemcpyHostToDevice, S->stream));
            HIPCHK(S, hipStreamSynchronize(S->stream));
            o->outcome = GPR_DEPHASE_CONVERGED; o->to_state = S->omega; o->t_steps = S->dp_t;
            o->n_branch = S->n_branch; o->n_samples = 0;
            for (int j = 0; j < GPR_MAX_OBS; ++j) o->rhat[j] = 0.0;
            S->phase = PH_CONVERGED;
            return GPR_OK;
        }
        HIPCHK(S, hipStreamSynchronize(S->stream));
    }
    return GPR_BUDGET;
}

extern "C" gpr_status gpr_parallel_step(gpr_system *S, int64_t max_checks, gpr_exit_out *o)
{
    if (!S || !o) return fail(S, GPR_EINVAL, "NULL argument");
    PhaseRun p;
    p.op = GPR_OP_PARALLEL_STEP; p.budget = max_checks;
    const gpr_status rc = run_phase(S, p);
    if (rc == GPR_OK) *o = p.pout;
    return rc;
}

extern "C" gpr_status gpr_advance(gpr_system *S, int64_t nsteps, int64_t *first_exit_check)
{
    if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
    if (nsteps < 0) return fail(S, GPR_EINVAL, "nsteps < 0");
    // first exit checks are recorded (and read back) only for a caller that asks for them
    if (first_exit_check) HIPCHK(S, hipMemsetAsync(S->fec, 0, sizeof(long long) * S->R, S->stream));
    // the sampling (every t_GR) and check (every t_check_dephase) schedule runs on the steps
    // counted over all calls, so that short calls sample and check as one long call would
    long long t = S->adv_t;
    const long long end = S->adv_t + nsteps;
    while (t < end) {
        const long long k = std::min<long long>(S->tcd - t % S->tcd, end - t);
        const bool at_check = (t + k) % S->tcd == 0;
        gpr_status rc = run_steps(S, S->R, k, t, true, at_check);
        if (rc) return rc;
        S->nsamp += count_samples(t, t + k, S->t_gr);
        t += k;
        S->adv_t = t;
        if (at_check) {
            rc = check(S, CHK_ADVANCE, S->R, t / S->tcd);
            if (rc) return rc;
        }
    }
    // error flags (and first exit checks) through page-locked memory, one wait
    if (first_exit_check)
        HIPCHK(S, hipMemcpyAsync(S->adv_fec, S->fec, sizeof(long long) * S->R, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipMemcpyAsync(S->adv_err, S->d.err, sizeof(int) * 4, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
    HIPCHK(S, prof_collect(S));
    const int *err = S->adv_err;
    if (err[ERR_UNSTABLE]) return fail(S, GPR_EUNSTABLE, "non-finite or overflowing state");
    if (err[ERR_LIST]) return fail(S, GPR_EDEVICE, "pair-list capacity exceeded");
    if (err[ERR_BARRIER]) return fail(S, GPR_EDEVICE, "persistent-kernel barrier timed out");
    if (first_exit_check) for (int r = 0; r < S->R; ++r) first_exit_check[r] = S->adv_fec[r];
    return GPR_OK;
}

// ------------------------------------------------------------------ several systems in one launch
// validation shared by the batch calls
static gpr_status batch_check(gpr_system *const *systems, int32_t nsys)
{
    if (!systems || nsys < 1 || nsys > MAX_BATCH) return fail(nullptr, GPR_EINVAL, "1 to 8 systems");
    for (int k = 0; k < nsys; ++k) {
        gpr_system *S = systems[k];
        if (!S) return fail(nullptr, GPR_EINVAL, "NULL system");
        for (int j = 0; j < k; ++j)
            if (systems[j] == S) return fail(S, GPR_EINVAL, "a system appears twice");
        if (!S->persist_ok) return fail(S, GPR_EINVAL, "system too large for the persistent path");
        if (S->stream != systems[0]->stream) return fail(S, GPR_EINVAL, "all systems must use one stream");
    }
    return GPR_OK;
}

// block size and LDS of a shared launch (the largest of the systems') and the workgroups the
// device holds at once with them; w[k]: work estimate of one step of all of system k's replicas
struct BatchShape {
    int bt = 64;
    size_t lds = 0;
    int capacity = 0;
    std::vector<double> w;
};

static gpr_status batch_shape(gpr_system *const *systems, int32_t nsys, BatchShape &sh)
{
    sh.w.assign(nsys, 0.0);
    for (int k = 0; k < nsys; ++k) {
        gpr_system *S = systems[k];
        sh.bt = std::max(sh.bt, S->bt_persist);
        sh.lds = std::max(sh.lds, persist_lds(S->n, S->np, S->split));
        double per = 0.0;
        for (double x : S->work) per += x;
        sh.w[k] = per;
    }
    int dev = 0, cus = 0, per_cu = 0;
    HIPCHK(systems[0], hipGetDevice(&dev));
    HIPCHK(systems[0], hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(systems[0], hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_persist_batch, sh.bt, sh.lds));
    sh.capacity = per_cu * cus;
    return GPR_OK;
}

// Items of a shared launch for the systems with nrep[k] > 0 replicas stepped: sets per system
// one each to begin with; then, one set at a time, more for the system whose replicas would
// take longest, estimated as (replicas per set) x (time of one replica-step on one workgroup)
// / G, that time modelled as 5 us of fixed latency plus 2.8e-4 us per unit of the per-atom
// work estimate (both from measured step times).  slot[k]: the item of system k (-1: none).
static gpr_status batch_layout(gpr_system *const *systems, int32_t nsys, const std::vector<int> &nrep,
                               const BatchShape &sh, PersistBatch &pb, std::vector<int> &slot, int &nblocks)
{
    gpr_system *S0 = systems[0];
    std::vector<int> sets(nsys, 0);
    int used = 0;
    for (int k = 0; k < nsys; ++k)
        if (nrep[k] > 0) { sets[k] = 1; used += systems[k]->groups; }
    if (used > sh.capacity) return fail(S0, GPR_EINVAL, "the systems' workgroups do not fit on the device at once");
    auto est = [&](int k, int ns) {
        const double t1 = 5.0 + 2.8e-4 * sh.w[k];
        return (double)((nrep[k] + ns - 1) / ns) * t1 / systems[k]->groups;
    };
    for (;;) {
        int pick = -1;
        for (int k = 0; k < nsys; ++k) {
            if (nrep[k] <= 0 || sets[k] >= nrep[k] || used + systems[k]->groups > sh.capacity) continue;
            if (pick < 0 || est(k, sets[k]) > est(pick, sets[pick])) pick = k;
        }
        if (pick < 0) break;
        sets[pick] += 1;
        used += systems[pick]->groups;
    }
    std::vector<PersistItem> items(nsys);
    std::vector<int> nb(nsys, 0);
    for (int k = 0; k < nsys; ++k) {
        if (nrep[k] <= 0) continue;
        gpr_status rc = persist_item(systems[k], nrep[k], sh.bt, sh.lds, sets[k] * systems[k]->groups, items[k], nb[k]);
        if (rc) return rc;
    }
    slot.assign(nsys, -1);
    pb = PersistBatch{};
    int boff = 0, j = 0;
    for (int pass = 1; pass >= 0; --pass)
        for (int k = 0; k < nsys; ++k) {
            if (nrep[k] <= 0 || items[k].xcd != pass) continue;
            items[k].boff = boff;
            boff += nb[k];
            slot[k] = j;
            pb.it[j++] = items[k];
        }
    pb.nitems = j;
    if (boff > sh.capacity) return fail(S0, GPR_EINVAL, "the systems' workgroups do not fit on the device at once");
    nblocks = boff;
    return GPR_OK;
}

// gpr_advance of every system, with the persistent steps of all systems in shared launches:
// each launch runs up to the next exit check of any of them, then the systems at a check run
// it.  Workgroups are shared out so as to even out the systems' estimated times per step.
extern "C" gpr_status gpr_batch_advance(gpr_system *const *systems, int32_t nsys, int64_t nsteps,
                                        int64_t *const *first_exit_check)
{
    gpr_status rc = batch_check(systems, nsys);
    if (rc) return rc;
    if (nsteps < 0) return fail(systems[0], GPR_EINVAL, "nsteps < 0");
    gpr_system *S0 = systems[0];
    hipStream_t stream = S0->stream;
    BatchShape sh;
    rc = batch_shape(systems, nsys, sh);
    if (rc) return rc;
    std::vector<int> nrep(nsys), slot;
    for (int k = 0; k < nsys; ++k) nrep[k] = systems[k]->R;
    PersistBatch pb{};
    int nblocks = 0;
    rc = batch_layout(systems, nsys, nrep, sh, pb, slot, nblocks);
    if (rc) return rc;
    std::vector<long long> t(nsys, 0);
    for (int k = 0; k < nsys; ++k) t[k] = systems[k]->adv_t;
    for (int k = 0; k < nsys; ++k)
        HIPCHK(systems[k], hipMemsetAsync(systems[k]->fec, 0, sizeof(long long) * systems[k]->R, stream));
    long long done = 0;
    while (done < nsteps) {
        long long kstep = nsteps - done;
        for (int k = 0; k < nsys; ++k) kstep = std::min<long long>(kstep, systems[k]->tcd - t[k] % systems[k]->tcd);
        kstep = std::min<long long>(kstep, 1 << 20);
        for (int k = 0; k < nsys; ++k) {
            gpr_system *S = systems[k];
            PersistItem &it = pb.it[slot[k]];
            it.s0 = S->s;
            it.nsteps = (int)kstep;
            it.t0 = (int)(t[k] % S->t_gr);
            it.sample = 1;
            it.state_end = (t[k] + kstep) % S->tcd == 0 ? 1 : 0;
        }
        rc = launch_persist(S0, pb, nblocks, sh.bt, sh.lds, stream);
        if (rc) return rc;
        for (int k = 0; k < nsys; ++k) {
            gpr_system *S = systems[k];
            S->s += kstep;
            S->nsamp += count_samples(t[k], t[k] + kstep, S->t_gr);
            t[k] += kstep;
            S->adv_t = t[k];
            if (t[k] % S->tcd == 0) {
                rc = check(S, CHK_ADVANCE, S->R, t[k] / S->tcd);
                if (rc) return rc;
            }
        }
        done += kstep;
    }
    for (int k = 0; k < nsys; ++k) {
        gpr_system *S = systems[k];
        std::vector<long long> f(S->R);
        HIPCHK(S, hipMemcpyAsync(f.data(), S->fec, sizeof(long long) * S->R, hipMemcpyDeviceToHost, stream));
        int err[4];
        HIPCHK(S, hipMemcpyAsync(err, S->d.err, sizeof err, hipMemcpyDeviceToHost, stream));
        HIPCHK(S, hipStreamSynchronize(stream));
        if (err[ERR_UNSTABLE]) return fail(S, GPR_EUNSTABLE, "non-finite or overflowing state");
        if (err[ERR_LIST]) return fail(S, GPR_EDEVICE, "pair-list capacity exceeded");
        if (err[ERR_BARRIER]) return fail(S, GPR_EDEVICE, "persistent-kernel barrier timed out");
        if (first_exit_check && first_exit_check[k])
            for (int r = 0; r < S->R; ++r) first_exit_check[k][r] = f[r];
    }
    return GPR_OK;
}

// The Gen.ParRep calls of several systems (Fig. 1 steps), their chunks of steps in shared
// launches: each launch takes every running system up to the nearest exit check among them.
extern "C" gpr_status gpr_batch_run(gpr_system *const *systems, int32_t nsys, gpr_batch_op *ops)
{
    gpr_status rc = batch_check(systems, nsys);
    if (rc) return rc;
    if (!ops) return fail(systems[0], GPR_EINVAL, "NULL ops");
    gpr_system *S0 = systems[0];
    hipStream_t stream = S0->stream;
    BatchShape sh;
    rc = batch_shape(systems, nsys, sh);
    if (rc) return rc;
    std::vector<PhaseRun> p(nsys);
    for (int k = 0; k < nsys; ++k) {
        p[k].op = ops[k].op;
        p[k].t_corr = ops[k].t_corr;
        p[k].budget = ops[k].max_steps;
        ops[k].status = GPR_BUDGET;
    }
    auto finish = [&](int k) {
        ops[k].status = p[k].rc;
        if (p[k].rc == GPR_OK) {
            if (p[k].op == GPR_OP_DECORRELATE) ops[k].event = p[k].ev;
            else if (p[k].op == GPR_OP_DEPHASE) ops[k].dephase = p[k].dout;
            else ops[k].exit = p[k].pout;
        }
    };
    for (int k = 0; k < nsys; ++k) {
        rc = phase_begin(systems[k], p[k]);
        if (rc) { ops[k].status = rc; return rc; }
    }
    std::vector<int> nrep(nsys), slot, last_nrep;
    std::vector<Chunk> c(nsys);
    PersistBatch pb{};
    int nblocks = 0;
    for (;;) {
        long long kstep = 1LL << 20;
        int active = 0;
        for (int k = 0; k < nsys; ++k) {
            phase_ready(systems[k], p[k]);
            nrep[k] = 0;
            if (p[k].done) continue;
            c[k] = phase_chunk(systems[k], p[k], 1LL << 62);
            kstep = std::min(kstep, c[k].k);
            nrep[k] = c[k].nrep;
            ++active;
        }
        if (active == 0) break;
        if (nrep != last_nrep) {                          // the running systems or their replica counts changed
            rc = batch_layout(systems, nsys, nrep, sh, pb, slot, nblocks);
            if (rc) return rc;
            last_nrep = nrep;
        }
        for (int k = 0; k < nsys; ++k) {
            if (nrep[k] == 0) continue;
            gpr_system *S = systems[k];
            c[k] = phase_chunk(S, p[k], kstep);
            PersistItem &it = pb.it[slot[k]];
            it.s0 = S->s;
            it.nsteps = (int)kstep;
            it.t0 = (int)(c[k].t0 % S->t_gr);
            it.sample = c[k].sample ? 1 : 0;
            it.state_end = c[k].at_check ? 1 : 0;
        }
        rc = launch_persist(S0, pb, nblocks, sh.bt, sh.lds, stream);
        if (rc) return rc;
        for (int k = 0; k < nsys; ++k) {
            if (nrep[k] == 0) continue;
            systems[k]->s += kstep;
            rc = phase_advance(systems[k], p[k], c[k]);
            if (rc) { ops[k].status = rc; return rc; }
        }
    }
    for (int k = 0; k < nsys; ++k) finish(k);
    return GPR_OK;
}

// ------------------------------------------------------------------ building blocks
template <class T>
static hipError_t tmp_alloc(std::vector<void *> &v, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) { v.push_back(q); *p = (T *)q; }
    return e;
}

struct TmpBufs {
    std::vector<void *> v;
    ~TmpBufs() { for (void *p : v) (void)hipFree(p); }
};

#define TMPCHK(call)                                                                                \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail(nullptr, GPR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" gpr_status gpr_philox_noise(uint64_t seed, int32_t replica, int64_t step, int32_t stream, int32_t n_atoms,
                                       uint32_t *out_words, float *out_gauss)
{
    if (n_atoms < 0 || stream < 0 || stream > 255) return fail(nullptr, GPR_EINVAL, "bad arguments");
    if (n_atoms == 0) return GPR_OK;
    TmpBufs t;
    uint32_t *w = nullptr;
    float *g = nullptr;
    TMPCHK(tmp_alloc(t.v, &w, 4 * (size_t)n_atoms));
    TMPCHK(tmp_alloc(t.v, &g, 3 * (size_t)n_atoms));
    hipLaunchKernelGGL(k_noise_test, dim3((n_atoms + 255) / 256), dim3(256), 0, 0, (uint32_t)seed,
                       (uint32_t)(seed >> 32), replica, (long long)step, stream, n_atoms, w, g);
    TMPCHK(hipGetLastError());
    if (out_words) TMPCHK(hipMemcpy(out_words, w, 16 * (size_t)n_atoms, hipMemcpyDeviceToHost));
    if (out_gauss) TMPCHK(hipMemcpy(out_gauss, g, 12 * (size_t)n_atoms, hipMemcpyDeviceToHost));
    TMPCHK(hipDeviceSynchronize());
    return GPR_OK;
}

extern "C" gpr_status gpr_fv_plan(uint64_t seed, int64_t step, int32_t R, const uint8_t *exited, int32_t *donor)
{
    if (R < 1 || !exited || !donor) return fail(nullptr, GPR_EINVAL, "bad arguments");
    TmpBufs t;
    uint8_t *ex = nullptr;
    int *dn = nullptr, *sv = nullptr;
    TMPCHK(tmp_alloc(t.v, &ex, R));
    TMPCHK(tmp_alloc(t.v, &dn, R));
    TMPCHK(tmp_alloc(t.v, &sv, R));
    TMPCHK(hipMemcpy(ex, exited, R, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_fvplan_test, dim3(1), dim3(256), 0, 0, (uint32_t)seed, (uint32_t)(seed >> 32), (long long)step, R, ex, dn, sv);
    TMPCHK(hipGetLastError());
    TMPCHK(hipMemcpy(donor, dn, sizeof(int) * R, hipMemcpyDeviceToHost));
    return GPR_OK;
}

// ------------------------------------------------------------------ branching plan without allocation
// Device array that gpr_fv_plan_noalloc stages through, for up to GPR_NOALLOC_MAX_R replicas:
// donors (int) at byte 0, the survivor list (int) at 4 * max, the exited flags at 8 * max.
// Every device the library runs on holds its own copy until the process ends.  In host code
// its name is not a device address: the address is taken per device with
// hipGetSymbolAddress and only that address is used.
constexpr size_t NOALLOC_BYTES = (size_t)9 * GPR_NOALLOC_MAX_R;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[NOALLOC_MAX_DEV] = {};

// the device address of `scratch` on the current device, taken on the first call there
hipError_t scratch_of_current_device(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
} // namespace

extern "C" gpr_status gpr_fv_plan_noalloc(uint64_t seed, int64_t step, int32_t R, const uint8_t *exited, int32_t *donor)
{
    if (R < 1 || !exited || !donor) return fail(nullptr, GPR_EINVAL, "bad arguments");
    if (R > GPR_NOALLOC_MAX_R)
        return fail(nullptr, GPR_EINVAL, "R exceeds GPR_NOALLOC_MAX_R (" + std::to_string(GPR_NOALLOC_MAX_R) + ")");
    unsigned char *base = nullptr;
    TMPCHK(scratch_of_current_device(&base));
    int *dn = (int *)base;
    int *sv = (int *)(base + (size_t)4 * GPR_NOALLOC_MAX_R);
    uint8_t *ex = base + (size_t)8 * GPR_NOALLOC_MAX_R;
    // every word the kernel reads is written first (flags copied in, survivors and donors
    // written before they are read), so nothing needs clearing between calls
    TMPCHK(hipMemcpy(ex, exited, R, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_fvplan_test, dim3(1), dim3(256), 0, 0, (uint32_t)seed, (uint32_t)(seed >> 32), (long long)step, R, ex, dn, sv);
    TMPCHK(hipGetLastError());
    TMPCHK(hipMemcpy(donor, dn, sizeof(int) * R, hipMemcpyDeviceToHost));
    return GPR_OK;
}

extern "C" gpr_status gpr_rhat(int32_t nw, int32_t n_obs, int64_t n, const double *S1, const double *S2, double *rhat)
{
    if (nw < 1 || n_obs < 0 || n_obs > 64 || n < 1 || (n_obs && (!S1 || !S2 || !rhat)))
        return fail(nullptr, GPR_EINVAL, "bad arguments");
    if (n_obs == 0) return GPR_OK;
    TmpBufs t;
    double *a = nullptr, *b = nullptr, *o = nullptr;
    const size_t cnt = (size_t)nw * n_obs;
    TMPCHK(tmp_alloc(t.v, &a, cnt));
    TMPCHK(tmp_alloc(t.v, &b, cnt));
    TMPCHK(tmp_alloc(t.v, &o, n_obs));
    TMPCHK(hipMemcpy(a, S1, cnt * 8, hipMemcpyHostToDevice));
    TMPCHK(hipMemcpy(b, S2, cnt * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_rhat_test, dim3(n_obs), dim3(64), 0, 0, nw, n_obs, (long long)n, a, b, o);
    TMPCHK(hipGetLastError());
    TMPCHK(hipMemcpy(rhat, o, 8 * (size_t)n_obs, hipMemcpyDeviceToHost));
    return GPR_OK;
}

extern "C" gpr_status gpr_exit_vote(int32_t R, const int64_t *fec, int64_t t_check, int64_t *M, int32_t *k, int64_t *tau)
{
    if (R < 1 || !fec || !M || !k || !tau) return fail(nullptr, GPR_EINVAL, "bad arguments");
    TmpBufs t;
    long long *f = nullptr, *o = nullptr;
    TMPCHK(tmp_alloc(t.v, &f, R));
    TMPCHK(tmp_alloc(t.v, &o, 3));
    TMPCHK(hipMemcpy(f, fec, 8 * (size_t)R, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_vote_test, dim3(1), dim3(256), 0, 0, R, f, (long long)t_check, o);
    TMPCHK(hipGetLastError());
    long long h[3];
    TMPCHK(hipMemcpy(h, o, sizeof h, hipMemcpyDeviceToHost));
    if (h[0] == 0) return GPR_BUDGET;
    *M = h[0];
    *k = (int32_t)h[1];
    *tau = h[2];
    return GPR_OK;
}
