"""The loop of Fig. 1 (transient step, convergence step, parallel step) on the 22-atom chain
(256 replicas, t_GR = 10, t_check = 250 / 2,500 steps) and on the 2,432-atom receptor-ligand
system (64 replicas, t_GR = 50, t_check = 1,000), with the settings of the workloads: the clock
adds up (Eq. 6 and the rules after Eq. 4), the convergence step ends with every R-hat below
1 + TOL (Eq. 4) after t_FV / t_GR samples, and the persistent path, the plain path and captured
check cycles give bit-identical events and configurations.  (The oracle cannot follow these
runs: at these sizes an FP32 and an FP64 trajectory part ways within a few thousand steps,
and the full-size oracle is some 10^4 times slower; parity with it is checked on short runs
elsewhere.)"""
import sys

import numpy as np
import pytest

import gpr_synth as G

pytestmark = pytest.mark.gpu


def _gpr():
    import paper_1807_02431_amd as gpr
    return gpr


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cycle(s, t_corr, max_checks, dephase_steps=1 << 62):
    """One pass of Fig. 1: the events and the clock after each call (the convergence step
    within a budget of dephase_steps, the parallel step within max_checks checks)."""
    log = []
    for _ in range(50):                                  # transient steps until a state is held
        t0 = s.simulated_steps()
        rc, ev = s.decorrelate(t_corr)
        assert rc == 0
        log.append(("t", ev["kind"], ev["from_state"], ev["to_state"], ev["steps_taken"], s.simulated_steps() - t0))
        assert s.simulated_steps() - t0 == ev["steps_taken"]
        if ev["kind"] == 0:
            break
    else:
        return log
    t1 = s.simulated_steps()
    rc, d = s.dephase(dephase_steps)
    if rc == 1:
        log.append(("f-budget", s.accumulators()[0]))
        return log
    log.append(("f", d["outcome"], d["to_state"], d["t_steps"], d["n_branch"], d["n_samples"],
                tuple(np.asarray(d["rhat"]).view(np.uint64).tolist())))
    assert s.simulated_steps() - t1 == d["t_steps"]
    if d["outcome"] == 1:
        return log
    t2 = s.simulated_steps()
    rc, e = s.parallel_step(max_checks)
    if rc == 0:
        log.append(("p", e["M"], e["k"], e["tau_steps"], e["to_state"]))
        assert s.simulated_steps() - t2 == e["tau_steps"]
    else:
        log.append(("p-budget",))
        assert s.simulated_steps() == t2
    return log


def _check_dephase(log, spec):
    f = [x for x in log if x[0] == "f"]
    if not f or f[0][1] != 0:
        return False
    _, _, _, t_steps, _, n_samples, rhat_bits = f[0]
    rhat = np.asarray(rhat_bits, np.uint64).view(np.float64)
    assert t_steps % spec["t_check_dephase"] == 0
    assert n_samples <= t_steps // spec["t_gr"] and n_samples >= 2
    assert np.all(rhat < 1.0 + spec["tol"]) and np.all(rhat >= 1.0 - 1e-9)
    return True


def _same(a, b, R):
    for r in (0, 1, R // 2, R - 1):
        qa, va = a.get_state(r)
        qb, vb = b.get_state(r)
        assert np.array_equal(qa, qb) and np.array_equal(va, vb), r


def test_chain22_gen_parrep_pass():
    """The 22-atom chain with 256 replicas: one pass of Fig. 1 on the persistent path, on the
    persistent path with 16 captured check cycles per replay, and on the plain path."""
    gpr = _gpr()
    spec = G.config("chain22")
    R = spec["n_replicas"]
    runs = []
    for path, cycles in ((1, 0), (1, 16), (0, 0)):
        s = gpr.System(spec, path=path)
        if cycles:
            s.set_cycles(cycles)
        say("chain22 pass, path", path, "cycles", cycles)
        runs.append((s, _cycle(s, 1000, 4)))
        say(runs[-1][1])
    (a, la), (b, lb), (c, lc) = runs
    assert la == lb == lc
    assert _check_dephase(la, spec)
    assert a.simulated_steps() == b.simulated_steps() == c.simulated_steps()
    _same(a, b, R)
    _same(a, c, R)


def test_rl2432_gen_parrep_pass():
    """The 2,432-atom receptor-ligand system with 64 replicas: two passes of Fig. 1 (from the
    bound state, t_check = 1,000; each convergence step within 20,000 steps) on the persistent
    path, with and without captured check cycles: the same events, R-hat bits, clock and
    configurations; a convergence step that converges does so below 1 + TOL."""
    gpr = _gpr()
    spec = G.config("rl2432")
    R = spec["n_replicas"]
    runs = []
    for cycles in (0, 4):
        s = gpr.System(spec, path=gpr.PATH_PERSISTENT)
        if cycles:
            s.set_cycles(cycles)
        say("rl2432 pass, cycles", cycles)
        assert s.current_state() == 1                    # the ligand starts bound
        log = _cycle(s, 1000, 2, dephase_steps=20000) + _cycle(s, 1000, 2, dephase_steps=20000)
        runs.append((s, log))
        say(log)
    (a, la), (b, lb) = runs
    assert la == lb
    for x in la:
        if x[0] == "f" and x[1] == 0:
            assert _check_dephase([x], spec)
    assert a.simulated_steps() == b.simulated_steps() and a.global_step() == b.global_step()
    _same(a, b, R)
