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
