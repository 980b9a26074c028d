"""The plain path as replays of a captured HIP graph (gpr_set_graph): the kernels take the step
counter and the sampling decision from device memory, so every replay must continue exactly
where the host-launched steps would.  Checked bit for bit against the host-launched plain path
and the persistent path after every call (several replays per call, eager launches between
them, step counts that are not multiples of the cycle), Gen.ParRep loops included."""
import sys

import numpy as np
import pytest

import gpr_synth as G
from helpers import gen_parrep_exits

pytestmark = pytest.mark.gpu


def _gpr():
    import paper_1807_02431_amd as gpr
    return gpr


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same_state(a, b, R):
    for r in range(R):
        qa, va = a.get_state(r)
        qb, vb = b.get_state(r)
        assert np.array_equal(qa, qb) and np.array_equal(va, vb), r


def _same_acc(a, b):
    na, S1a, S2a, sha = a.accumulators()
    nb, S1b, S2b, shb = b.accumulators()
    assert na == nb
    assert np.array_equal(S1a, S1b) and np.array_equal(S2a, S2b) and np.array_equal(sha, shb)


@pytest.mark.parametrize("name,cycle", [("chain22", 7), ("rl300", 16), ("rl2432", 25)])
def test_graph_replays_match_host_launches(name, cycle):
    gpr = _gpr()
    R = 8
    spec = G.config(name, n_replicas=R)
    say("graph", name, "cycle", cycle)
    g = gpr.System(spec, path=gpr.PATH_PLAIN)
    g.set_graph(cycle)
    h = gpr.System(spec, path=gpr.PATH_PLAIN)
    p = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    for n in (cycle - 1, 3 * cycle + 2, 5 * cycle, 1):
        fg, fh, fp = g.advance(n), h.advance(n), p.advance(n)
        assert np.array_equal(fg, fh) and np.array_equal(fg, fp)
        assert g.global_step() == h.global_step() == p.global_step()
        _same_state(g, h, R)
        _same_state(g, p, R)
        _same_acc(g, h)
        _same_acc(g, p)
        E1, F1 = g.energy_forces()
        E2, F2 = h.energy_forces()
        assert np.array_equal(E1, E2) and np.array_equal(F1, F2)


@pytest.mark.parametrize("seed", [3, 8])
def test_graph_gen_parrep_loop_matches(seed):
    """Decorrelation, Fleming-Viot dephasing (sampling every t_GR inside replayed cycles) and
    parallel steps on the toy landscape: the same exit records, clocks and final states with
    and without the graph, and with the graph switched off half way."""
    gpr = _gpr()
    spec = G.toy2d(n_replicas=16, seed=seed)
    say("graph gen parrep, seed", seed)
    a = gpr.System(spec)
    a.set_graph(4)
    b = gpr.System(spec)
    ea = gen_parrep_exits(a, 3, 100)
    eb = gen_parrep_exits(b, 3, 100)
    assert ea == eb
    a.set_graph(0)
    assert gen_parrep_exits(a, 2, 100) == gen_parrep_exits(b, 2, 100)
    assert a.simulated_steps() == b.simulated_steps()
    _same_state(a, b, 16)


def test_set_graph_refuses_bad_cycles():
    gpr = _gpr()
    g = gpr.System(G.config("chain22", n_replicas=2))
    for bad in (-1, 10001):
        with pytest.raises(gpr.GprError) as e:
            g.set_graph(bad)
        assert e.value.code == -1


def _rl300_flipping():
    """The 300-atom receptor-ligand system with its state split at the current value of a
    ligand dihedral, so that exits come within a few checks, and a tolerance that R-hat meets
    at the first check, so that parallel steps follow."""
    import oracle
    rl = G.config("rl300", n_replicas=8, t_check=200, tol=1e9)
    L = rl["n_atoms"] - 32 + 10
    dih = [L, L + 1, L + 2, L + 3]
    o = oracle.System(dict(rl, n_replicas=2, obs=[dict(kind=G.OBS_DIHEDRAL, atoms=dih)]))
    phi0 = o.observables_of(rl["pos"], np.zeros((3, rl["n_atoms"])), 0.0)[0]
    rl["state"] = dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=dih + dih,
                       boxes=[[-4.0, phi0 + 0.05, -4.0, 4.0], [phi0 + 0.05, 4.0, -4.0, 4.0]])
    return rl


@pytest.mark.parametrize("name,groups,cycles", [("toy", 1, 8), ("toy", 1, 1), ("rl300", 2, 4)])
def test_check_cycles_match_host_checks(name, groups, cycles):
    """Convergence and parallel steps as replays of captured check cycles (gpr_set_cycles): the
    loop of Fig. 1 gives the same events, clock, branch and sample counts, R-hat bits and
    configurations as with one host round trip per check; with two workgroups per replica the
    captured persistent launches synchronise the groups of a replica across CUs."""
    gpr = _gpr()
    if name == "toy":
        spec = dict(G.toy2d(n_replicas=64, seed=9), pos=np.array([[-0.2], [0.0], [0.0]]))
        t_corr, n = 100, 6
    else:
        spec = _rl300_flipping()
        t_corr, n = 400, 4
    R = spec["n_replicas"]
    say("check cycles", name, "groups", groups, "cycles", cycles)
    a = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    b = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    if groups > 1:
        a.set_launch(0, groups)
        b.set_launch(0, groups)
    a.set_cycles(cycles)

    def loop(s):
        out = []
        while len(out) < n:
            rc, ev = s.decorrelate(t_corr)
            assert rc == 0
            if ev["kind"] == 1:
                out.append(("t", ev["from_state"], ev["to_state"], ev["steps_taken"]))
                continue
            rc, d = s.dephase()
            assert rc == 0
            out.append(("f", d["outcome"], d["to_state"], d["t_steps"], d["n_branch"], d["n_samples"],
                        tuple(np.asarray(d["rhat"]).view(np.uint64).tolist())))
            if d["outcome"] == 1:
                continue
            rc, e = s.parallel_step()
            assert rc == 0
            out.append(("p", e["M"], e["k"], e["tau_steps"], e["to_state"]))
        return out
    la, lb = loop(a), loop(b)
    say(la)
    assert la == lb
    assert any(x[0] == "p" for x in la)
    assert a.simulated_steps() == b.simulated_steps() and a.global_step() == b.global_step()
    _same_state(a, b, R)
    _same_acc(a, b)
    # budgets that stop inside a replay's span fall back to host checks, and resume
    rc, _ = a.decorrelate(0)
    rc, _ = b.decorrelate(0)
    if a.current_state() != -1:
        ra, da = a.dephase(max_steps=3 * spec["t_check_dephase"] + 1)
        rb, db = b.dephase(max_steps=3 * spec["t_check_dephase"] + 1)
        assert ra == rb and (ra == 1 or da == db)
        _same_state(a, b, R)
