"""Throughput of the Gen.ParRep hot path on one MI355X.

Workload: the 2,432-atom receptor-ligand system (2,400-atom restrained receptor chain + a
32-atom ligand in its pocket, 1.0 nm cutoff with reaction field, BAOAB at 1 fs) with 64
replicas.  One step = one BAOAB step of all 64 replicas with everything the dephasing
stage does around it: pair-list maintenance (every 10 steps and on the displacement
guard), bonded and nonbonded forces, observables of the workers every t_GR = 50 steps,
and every t_check = 1000 steps the state test of every replica, the Fleming-Viot
branching plan, the Gelman-Rubin statistics and the exit vote (computed, not acted on, so
that the work per step is fixed).

The samples and checks that fall inside the timed steps are reported ("window"); the schedule
runs on the steps of all calls, so a short timed window may hold none, and the latency of a call
that ends at a check is measured on its own ("check_latency").

The product path (persistent kernel) is timed, then the plain one-launch-per-kernel-per-step
path on the same system and seeds, launched from the host and replayed from a HIP graph.  Prints one JSON line.
`value` comes from the first timed run of --steps steps; both paths are then timed --repeats - 1
more times (each run continuing the trajectory), and the median over all runs is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# published MI355X peaks
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# algorithmic FLOP counts (FMA = 2) per unit of work
FLOP_PAIR = 40          # one in-cutoff nonbonded pair, force only, counted once per unordered pair
FLOP_BOND, FLOP_ANGLE, FLOP_TORSION, FLOP_RESTRAINT, FLOP_PAIR14 = 25, 60, 110, 12, 45
FLOP_ATOM_BAOAB = 20    # kicks, drifts and the Ornstein-Uhlenbeck update of one atom

GRAPH_CYCLE = 50        # steps per captured graph of the plain path (one t_GR period)


def in_cutoff_pairs(spec, q):
    """Number of nonbonded pairs (not excluded, not 1-4) closer than the cutoff."""
    n = spec["n_atoms"]
    rc2 = spec["cutoff"] ** 2
    x = q.T
    skip = set()
    for a, b in np.concatenate([spec["exclusions"], spec["pairs14"]]):
        skip.add((min(a, b), max(a, b)))
    total = 0
    for i0 in range(0, n, 256):
        d = x[i0:i0 + 256, None, :] - x[None, :, :]
        r2 = (d * d).sum(-1)
        ii, jj = np.nonzero(r2 < rc2)
        keep = jj > ii + i0
        total += int(keep.sum())
        for i, j in zip(ii[keep] + i0, jj[keep]):
            if j - i <= 3 and (i, j) in skip:
                total -= 1
    return total


def kernel_source_hash():
    import hashlib
    import glob
    h = hashlib.sha256()
    files = glob.glob(os.path.join(ROOT, "paper_1807_02431_amd", "csrc", "*"))
    files.append(os.path.join(ROOT, "paper_1807_02431_amd", "build.py"))   # the compiler flags
    for f in sorted(files):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_figure(fname, key, steps_per_launch):
    """A per-launch figure of the persistent kernel from a committed rocprofv3 summary, or None
    when the kernel sources (or the compiler flags) differ from the ones the counters were
    taken on.  The summary lists the figure for each launch length it measured
    (``<key>_<steps> <value>``); a launch of another length gets the straight line a + b L
    through the two measured lengths nearest to it (a: the work of a launch's start and end,
    b: the work of one step)."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    kv, pts = {}, {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) != 2:
                continue
            kv[parts[0]] = parts[1]
            if parts[0].startswith(key + "_"):
                try:
                    pts[int(parts[0][len(key) + 1:])] = float(parts[1])
                except ValueError:
                    pass
    if kv.get("source_sha256") != kernel_source_hash() or not pts:
        return None
    L = float(steps_per_launch)
    if int(round(L)) in pts:
        return pts[int(round(L))]
    if len(pts) < 2:
        return None
    (l0, v0), (l1, v1) = sorted(sorted(pts.items(), key=lambda kv_: abs(kv_[0] - L))[:2])
    b = (v1 - v0) / (l1 - l0)
    return v0 + b * (L - l0)


def measured_traffic(steps_per_launch):
    """HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, copy-calibrated)."""
    return _profile_figure("k_persist_rl2432x64_hbm_traffic.md", "hbm_bytes_per_launch", steps_per_launch)


def measured_fp32_flop(steps_per_launch):
    """FP32 FLOP executed per launch (rocprofv3 SQ_INSTS_VALU_{ADD,MUL,TRANS,FMA}_F32)."""
    return _profile_figure("k_persist_rl2432x64_valu_counters.md", "fp32_flop_per_launch", steps_per_launch)


def window_counts(t0, t1, t_gr, t_check):
    """Observable samples and exit checks that fall in the steps (t0, t1] of gpr_advance's
    schedule (samples every t_GR, checks every t_check, counted over all calls)."""
    return dict(samples=t1 // t_gr - t0 // t_gr, checks=t1 // t_check - t0 // t_check)


def flops_per_replica_step(spec, pairs):
    return (pairs * FLOP_PAIR + len(spec["bonds"]) * FLOP_BOND + len(spec["angles"]) * FLOP_ANGLE
            + len(spec["torsions"]) * FLOP_TORSION + len(spec["restraints"]) * FLOP_RESTRAINT
            + len(spec["pairs14"]) * FLOP_PAIR14 + spec["n_atoms"] * FLOP_ATOM_BAOAB)


def timed_advance(sysobj, steps):
    """Wall time of gpr_advance over `steps` steps (first exit checks not read back)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysobj.advance(steps, first_exit=False)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(spec, seconds=15.0):
    """The FP64 oracle, single-threaded, on a bounded sample of the same workload: a few
    replicas for as many steps as fit in about ``seconds``."""
    import oracle
    R = 4
    o = oracle.System(dict(spec, n_replicas=R))
    t0 = time.perf_counter()
    o.advance(1)
    one = time.perf_counter() - t0
    steps = max(1, int(seconds / max(one, 1e-6)))
    t0 = time.perf_counter()
    o.advance(steps)
    dt = time.perf_counter() - t0
    return dict(value=R * steps / dt, unit="replica-steps/s", cores=1, kind="oracle",
                sample="%d replicas x %d steps of the 2,432-atom system (FP64, brute-force pairs)" % (R, steps),
                atom_steps_per_s=R * steps * spec["n_atoms"] / dt)


_ORACLE_WORKER = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import gpr_synth as G
import oracle
o = oracle.System(G.config("rl2432", n_replicas=2))
o.advance(1)
start, seconds = float(sys.argv[2]), float(sys.argv[3])
while time.time() < start:
    time.sleep(0.01)
n, t0 = 0, time.perf_counter()
while time.perf_counter() - t0 < seconds:
    o.advance(1)
    n += 1
print(json.dumps({"replica_steps": 2 * n, "seconds": time.perf_counter() - t0}))
"""


def cpu_baseline_all_cores(seconds=10.0, max_workers=16):
    """The same FP64 oracle in one process per host core (at most 16), each stepping two
    replicas of the workload from a common start time for about ``seconds``; the aggregate is
    the replica-steps of all processes over the longest process's stepping time.  Run before
    the process touches the GPU: the workers are started as child processes."""
    import subprocess
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    workers = max(1, min(max_workers, ncpu))
    start = time.time() + 3.0 + 0.05 * workers
    procs = [subprocess.Popen([sys.executable, "-c", _ORACLE_WORKER, ROOT, repr(start), repr(seconds)],
                              stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True)
             for _ in range(workers)]
    res = []
    for p in procs:
        out, _ = p.communicate(timeout=120 + seconds)
        if p.returncode != 0:
            return None
        res.append(json.loads(out.strip().splitlines()[-1]))
    rs = sum(r["replica_steps"] for r in res)
    wall = max(r["seconds"] for r in res)
    return dict(value=rs / wall, unit="replica-steps/s", cores=workers, kind="oracle",
                sample="%d processes x 2 replicas of the 2,432-atom system, %d replica-steps in %.1f s (FP64, "
                       "brute-force pairs)" % (workers, rs, wall))


def differentiation_bench(spec, iters):
    """Forward (energy and forces) + backward (position and force-field parameter gradients) of
    all replicas through the device-pointer entry points, one batch per evaluation."""
    import torch
    import paper_1807_02431_amd as gpr
    R, n = spec["n_replicas"], spec["n_atoms"]
    s = gpr.System(spec, stream=torch.cuda.current_stream())
    s.advance(20)
    x = torch.tensor(np.stack([s.get_state(r)[0] for r in range(R)]), dtype=torch.float32, device="cuda")
    U = torch.empty(R, dtype=torch.float64, device="cuda")
    w = torch.ones(R, dtype=torch.float64, device="cuda")
    dx = torch.empty_like(x)
    ge, gs, gq = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3))
    gk = torch.empty(max(1, s.nt), dtype=torch.float64, device="cuda")

    def once():
        s.energy_forces_dev(x.data_ptr(), U.data_ptr(), 0)
        s.energy_backward_dev(w.data_ptr(), dx.data_ptr(), ge.data_ptr(), gs.data_ptr(), gq.data_ptr(), gk.data_ptr())

    for _ in range(3):
        once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    s.close()
    return dict(batch_evals_per_s=1.0 / dt, replica_evals_per_s=R / dt, ms_per_batch_eval=1e3 * dt,
                iters=iters, note="forward = energies + forces of all replicas (pair lists rebuilt); "
                "backward = dU/dx and dU/d(eps, sigma, q, torsion k) summed over replicas")


def pair_kernel_bench(pl, spec, pairs, launches=100):
    """The plain path's pair-force kernel (k_nonbonded, all replicas in one launch) timed launch
    by launch with HIP events over one-step calls; the median is a step without a pair-list
    rebuild (the lists are rebuilt on one step in ten).  Its algorithmic rate counts each
    in-cutoff unordered pair once at FLOP_PAIR."""
    R = spec["n_replicas"]
    pl.profile(True)
    prev_ms, prev_n = pl.profile_read()
    per = []
    for _ in range(launches):
        pl.advance(1)
        ms, n_ = pl.profile_read()
        if n_ > prev_n:
            per.append((ms - prev_ms) / (n_ - prev_n))
        prev_ms, prev_n = ms, n_
    pl.profile(False)
    # launches in which some replica rebuilds its lists (period or displacement guard) take
    # about twice as long; the median of the faster cluster is the pair loop alone
    cut = 0.5 * (min(per) + max(per))
    fast = [x for x in per if x <= cut]
    med = float(np.median(fast)) * 1e-3
    achieved = pairs * FLOP_PAIR * R / med / 1e12
    return dict(kernel="k_nonbonded", launches=len(per), launches_without_rebuild=len(fast), median_us=med * 1e6,
                median_all_us=1e3 * float(np.median(per)), max_us=1e3 * max(per), min_us=1e3 * min(per),
                achieved_tflops=achieved, frac=achieved / PEAK_FP32_TFLOPS,
                note="plain path, one launch for all 64 replicas; median of the launches without a pair-list "
                     "rebuild (those below the midpoint of the fastest and slowest launch); full per-atom lists: "
                     "each in-cutoff pair is evaluated twice and counted once")


def check_latency_bench(sysobj, t_check, checks=4):
    """Wall time of the one-step call that ends at an exit check (state test, branching plan,
    R-hat, exit vote, status read back) less that of an ordinary one-step call."""
    import torch

    def one():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sysobj.advance(1)
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    at, plain = [], []
    for _ in range(checks):
        left = (-sysobj.advance_steps() - 1) % t_check
        if left:
            sysobj.advance(left)
        at.append(one())
        plain.append(one())
    return dict(us=1e6 * (float(np.median(at)) - float(np.median(plain))),
                call_at_check_us=1e6 * float(np.median(at)), call_without_check_us=1e6 * float(np.median(plain)),
                checks=checks)


def small_configs_bench(seconds=2.0):
    """The toy (8 replicas) and the 22-atom chain (256 replicas) on the persistent path,
    each beside the oracle on one host core for about ``seconds`` of steps."""
    import torch
    import gpr_synth as G
    import oracle
    import paper_1807_02431_amd as gpr
    out = {}
    for name, steps in (("toy", 20000), ("chain22", 5000)):
        spec = G.config(name)
        R = spec["n_replicas"]
        g = gpr.System(spec, path=gpr.PATH_PERSISTENT, stream=torch.cuda.current_stream())
        g.advance(steps // 10)
        t = timed_advance(g, steps)
        g.close()
        o = oracle.System(spec)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < seconds:
            o.advance(10)
            k += 10
        to = time.perf_counter() - t0
        out[name] = dict(n_atoms=spec["n_atoms"], n_replicas=R, steps=steps,
                         replica_steps_per_s=R * steps / t, atom_steps_per_s=R * spec["n_atoms"] * steps / t,
                         t_gr=spec["t_gr"], t_check=spec["t_check_dephase"],
                         cpu_baseline=dict(value=R * k / to, unit="replica-steps/s", cores=1, kind="oracle",
                                           sample="%d replicas x %d steps (FP64)" % (R, k)))
    return out


def _parrep_loop(s, n_exits, t_corr):
    """The loop of Fig. 1 (transient step, convergence step, parallel step) until n_exits exit
    events; returns the number of events."""
    events = 0
    while events < n_exits:
        rc, ev = s.decorrelate(t_corr)
        if ev["kind"] == 1:
            events += 1
            continue
        rc, d = s.dephase()
        if d["outcome"] == 1:
            events += 1
            continue
        s.parallel_step()
        events += 1
    return events


def toy_parrep_bench(n_exits=40):
    """The Gen.ParRep loop on the toy (8 replicas, exit checks every 10 steps) on the persistent
    path with one host round trip per check, and with check cycles replayed from a captured
    graph (64 cycles per replay), beside the oracle: exit events and simulated steps per second
    of wall time."""
    import torch
    import gpr_synth as G
    import oracle
    import paper_1807_02431_amd as gpr
    out = {}
    for label, cycles in (("host_checks", 0), ("graph_cycles_64", 64)):
        s = gpr.System(G.toy2d(seed=17), path=gpr.PATH_PERSISTENT, stream=torch.cuda.current_stream())
        s.set_cycles(cycles)
        _parrep_loop(s, 3, 100)
        torch.cuda.synchronize()
        t0, st0 = time.perf_counter(), s.simulated_steps()
        _parrep_loop(s, n_exits, 100)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[label] = dict(events_per_s=n_exits / dt, simulated_steps_per_s=(s.simulated_steps() - st0) / dt,
                          seconds=dt)
        s.close()
    o = oracle.System(G.toy2d(seed=17))
    _parrep_loop(o, 3, 100)
    t0, st0 = time.perf_counter(), o.simulated_steps()
    _parrep_loop(o, n_exits, 100)
    dt = time.perf_counter() - t0
    out["oracle_one_core"] = dict(events_per_s=n_exits / dt, simulated_steps_per_s=(o.simulated_steps() - st0) / dt,
                                  seconds=dt)
    out["exits"] = n_exits
    return out


def batching_bench(steps):
    """The uneven mix (22 / 300 / 1,200 / 2,432 atoms x 192 replicas) advanced in shared
    persistent launches, against the same systems advanced one after the other."""
    import torch
    import gpr_synth as G
    import paper_1807_02431_amd as gpr
    specs = G.uneven_batch(192)
    stream = torch.cuda.current_stream()
    batch = [gpr.System(s, path=gpr.PATH_PERSISTENT, stream=stream) for s in specs]
    solo = [gpr.System(s, path=gpr.PATH_PERSISTENT, stream=stream) for s in specs]
    gpr.batch_advance(batch, 100)
    for x in solo:
        x.advance(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gpr.batch_advance(batch, steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    for x in solo:
        x.advance(steps)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    for x in batch + solo:
        x.close()
    reps = sum(s["n_replicas"] for s in specs)
    atoms = sum(s["n_replicas"] * s["n_atoms"] for s in specs)
    return dict(systems="22, 300, 1200, 2432 atoms x 192 replicas each", replicas=reps, steps=steps,
                replica_steps_per_s=reps * steps / tb, atom_steps_per_s=atoms * steps / tb,
                separate_replica_steps_per_s=reps * steps / ts, speedup_vs_separate=ts / tb)


def phases_bench(lengths=(1000, 20), launches=(3, 50), warmup=300):
    """Per-phase time of the persistent kernel from the timer build of the library (the same
    sources with per-phase clocks, loaded in place of the product one; results unchanged):
    for each launch length, µs per step in each phase averaged over every (replica, group),
    the launch prologue and epilogue per launch, pair-list rebuilds per step, and the sum of
    the phases of the slowest group against the kernel's own event timing."""
    import gpr_synth as G
    import paper_1807_02431_amd.gpr as gb
    gb.use_probe_library()
    import torch
    spec = G.config("rl2432")
    s = gb.System(spec, path=gb.PATH_PERSISTENT, stream=torch.cuda.current_stream())
    s.advance(warmup, first_exit=False)
    s.phase_read()
    out = {}
    for L, nl in zip(lengths, launches):
        s.profile(True)
        for _ in range(nl):
            s.advance(L, first_exit=False)
        kms, kn = s.profile_read()
        s.profile(False)
        ph = s.phase_read()                                   # [R, 8, 11]
        live = ph[:, :, 7] > 0                                 # (replica, group) slots that ran
        steps = ph[:, :, 7][live].mean()
        kn = max(kn, 1)                                        # kernel launches (a call that
        per = {}                                               # crosses a check boundary takes two)
        for k, name in enumerate(gb.PHASES):
            v = ph[:, :, k][live]
            if name in ("prologue", "epilogue"):
                per[name + "_us_per_launch"] = float(v.mean() / kn)
            else:
                per[name + "_us_per_step"] = float(v.mean() / steps)
        tot = ph[:, :, :7].sum(axis=2)[live]
        # the work a group does between two exchanges (all but the exchange wait), per step:
        # how far the busiest group of a replica is ahead of the replica's mean
        G = int(live[0].sum())
        own = (ph[:, :G, :7].sum(axis=2) - ph[:, :G, 2]) / steps
        per["group_imbalance_us_per_step"] = float((own.max(axis=1) - own.mean(axis=1)).mean())
        # the last launch: how far apart its workgroups started, and when the last one ended
        per["last_launch_start_spread_us"] = float(ph[:, :, 9][live].max())
        per["last_launch_span_us"] = float(ph[:, :, 10][live].max())
        out["calls_of_%d_steps" % L] = dict(
            calls=nl, kernel_launches=kn, steps_per_group=float(steps),
            rebuilds_per_step=float(ph[:, :, 8][live].mean() / steps),
            kernel_us_per_launch=1000.0 * kms / kn,
            phases_sum_us_per_launch_mean=float(tot.mean() / kn),
            phases_sum_us_per_launch_max_group=float(tot.max() / kn), **per)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of --steps steps per path (value: the first; the median is reported too)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven multi-system batching measurement")
    ap.add_argument("--no-small", action="store_true", help="skip the toy and 22-atom chain measurements")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 256 MiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--phases", action="store_true",
                    help="only measure the persistent kernel's phases with the timer build of the library")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the replicas of one system share one device "
              "(sharding replicas over several GPUs is not implemented); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.phases:
        print(json.dumps({"phases": phases_bench(), "workload": "rl2432 x 64, persistent path",
                          "source_sha256": kernel_source_hash()}))
        return

    # the oracle on all host cores first, while this process has not touched the GPU
    cpu_all = None
    if not args.no_cpu and not args.copy_probe:
        print("# oracle on all host cores", file=sys.stderr, flush=True)
        cpu_all = cpu_baseline_all_cores()

    import torch
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 4, "copy_probe_bytes_written": dst.numel() * 4}))
        return
    import gpr_synth as G
    import paper_1807_02431_amd as gpr

    spec = G.config("rl2432")
    R, n = spec["n_replicas"], spec["n_atoms"]
    stream = torch.cuda.current_stream()

    # ------------------------------------------------------------ product path
    print("# persistent path: warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    ps = gpr.System(spec, path=gpr.PATH_PERSISTENT, stream=stream)
    ps.advance(args.warmup)
    ps.profile(True)
    print("# persistent path: timing %d steps" % args.steps, file=sys.stderr, flush=True)
    a0 = ps.advance_steps()
    t_p = timed_advance(ps, args.steps)
    window = window_counts(a0, ps.advance_steps(), spec["t_gr"], spec["t_check_dephase"])
    kms, klaunch = ps.profile_read()
    ps.profile(False)
    reps_p = [t_p] + [timed_advance(ps, args.steps) for _ in range(args.repeats - 1)]
    q_samples = [ps.get_state(r)[0] for r in (0, R // 2, R - 1)]
    pairs = float(np.mean([in_cutoff_pairs(spec, q) for q in q_samples]))
    frs = flops_per_replica_step(spec, pairs)
    print("# persistent path: latency of an exit check", file=sys.stderr, flush=True)
    check_lat = check_latency_bench(ps, spec["t_check_dephase"])

    # ------------------------------------------------------------ plain path
    plain = plain_graph = k1 = None
    if not args.no_plain:
        print("# plain path: warmup %d, timing %d steps" % (args.warmup, args.steps), file=sys.stderr, flush=True)
        pl = gpr.System(spec, path=gpr.PATH_PLAIN, stream=stream)
        pl.advance(args.warmup)
        t_pl = timed_advance(pl, args.steps)
        reps_pl = [t_pl] + [timed_advance(pl, args.steps) for _ in range(args.repeats - 1)]
        pl.profile(True)
        pl.advance(min(args.steps, 1000))
        nb_ms, nb_n = pl.profile_read()
        pl.profile(False)
        plain = dict(replica_steps_per_s=R * args.steps / t_pl, atom_steps_per_s=R * n * args.steps / t_pl,
                     ms_per_step=1e3 * t_pl / args.steps, launches_per_step=3,
                     median_ms_per_step=1e3 * float(np.median(reps_pl)) / args.steps,
                     pair_kernel_us=1e3 * nb_ms / max(nb_n, 1))
        print("# plain path: pair-force kernel launch by launch", file=sys.stderr, flush=True)
        k1 = pair_kernel_bench(pl, spec, pairs)
        pl.close()
        print("# plain path replayed from a HIP graph: warmup %d, timing %d steps" % (args.warmup, args.steps),
              file=sys.stderr, flush=True)
        pg = gpr.System(spec, path=gpr.PATH_PLAIN, stream=stream)
        pg.set_graph(GRAPH_CYCLE)
        pg.advance(args.warmup)
        t_pg = timed_advance(pg, args.steps)
        plain_graph = dict(replica_steps_per_s=R * args.steps / t_pg, ms_per_step=1e3 * t_pg / args.steps,
                           cycle_steps=GRAPH_CYCLE)
        pg.close()

    diff = None
    if not args.no_diff:
        print("# differentiation: forward + backward", file=sys.stderr, flush=True)
        diff = differentiation_bench(spec, 50)

    batching = None
    if not args.no_batch:
        print("# uneven multi-system batching", file=sys.stderr, flush=True)
        batching = batching_bench(1000)

    small = None
    if not args.no_small:
        print("# toy and 22-atom chain", file=sys.stderr, flush=True)
        small = small_configs_bench()
        small["toy_gen_parrep"] = toy_parrep_bench()

    cpu = None if args.no_cpu else cpu_baseline(spec)
    if cpu is not None:
        cpu["all_cores"] = cpu_all

    steps_per_launch = args.steps / max(klaunch, 1)
    avg_launch_s = kms / 1e3 / max(klaunch, 1)
    achieved = frs * R * steps_per_launch / avg_launch_s / 1e12
    value = R * args.steps / t_p
    traffic = measured_traffic(steps_per_launch)
    exec_flop = measured_fp32_flop(steps_per_launch)
    out = {
        "metric": "replica-steps/s & atom-steps/s, 2,432 atoms x 64 replicas, vs plain GPU path",
        "value": value,
        "unit": "replica-steps/s",
        "atom_steps_per_s": value * n,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_p / args.steps,
        "window": dict(window, note="observable samples (every t_GR = 50) and exit checks (every t_check = "
                                    "1,000) of the product schedule inside the timed steps"),
        "check_latency": check_lat,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "speedup_vs_plain": (value / plain["replica_steps_per_s"]) if plain else None,
        "repeats": {"runs": len(reps_p), "ms_per_step": [1e3 * t / args.steps for t in reps_p],
                    "median_ms_per_step": 1e3 * float(np.median(reps_p)) / args.steps,
                    "median_replica_steps_per_s": R * args.steps / float(np.median(reps_p)),
                    "median_speedup_vs_plain": (float(np.median(reps_pl)) / float(np.median(reps_p))) if plain else None},
        "plain_path": plain,
        "plain_path_graph": plain_graph,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "receptor-ligand, 2,432 atoms (2,400 restrained receptor + 32 ligand) x 64 replicas, "
                               "cutoff 1.0 nm reaction field, BAOAB dt 1 fs, t_GR 50, t_check 1000",
                   "n_atoms": n, "n_replicas": R, "path": "persistent"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "hbm_gbs": (traffic / avg_launch_s / 1e9) if traffic else None, "hbm_peak_gbs": PEAK_HBM_GBS,
                     "executed_fp32_tflops": (exec_flop / avg_launch_s / 1e12) if exec_flop else None,
                     "kernel": "k_persist", "avg_launch_us": avg_launch_s * 1e6,
                     "steps_per_launch": steps_per_launch, "flop_per_replica_step": frs,
                     "in_cutoff_pairs_per_replica": pairs},
        "pair_kernel": k1,
        "cpu_baseline": cpu,
        "differentiation": diff,
        "batching": batching,
        "small_configs": small,
    }
    # handles destroyed before the interpreter ends (device buffers, events, pinned memory)
    ps.close()
    import gc
    gc.collect()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
