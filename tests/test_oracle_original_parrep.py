"""Pins of the oracle's original ParRep dephasing (Sec. 2.4.3: fixed decorrelation and dephasing
times, the variant that Gen.ParRep generalises): its invariants, its reduction to plain stepping
when no replica leaves the state, and the exit statistics of the whole original ParRep loop
against brute-force direct simulation."""
import numpy as np
import pytest
from scipy import stats

import gpr_synth as G
import oracle
from helpers import direct_exits, original_parrep_exits


def _toy(x0, seed, R=8):
    return G.round_to_f32(dict(G.toy2d(n_replicas=R, seed=seed), pos=np.array([[x0], [0.0], [0.0]])))


@pytest.mark.parametrize("seed", [3, 4, 6])
def test_fixed_dephasing_invariants(seed):
    o = oracle.System(_toy(-0.01, seed))
    with pytest.raises(oracle.OracleError):
        o.parallel_step()
    rc, ev = o.decorrelate(0)
    assert rc == 0 and ev["to_state"] == 0
    t0 = o.simulated_steps()
    rc, d = o.dephase_fixed(40)
    assert rc == 0 and d["outcome"] == 0
    assert o.simulated_steps() == t0                     # dephasing time is not counted
    assert d["t_steps"] % 10 == 0 and d["t_steps"] >= 40
    assert all(o.state_of(o.get_state(r)[0]) == 0 for r in range(8))
    rc, e = o.parallel_step()
    assert rc == 0 and 1 <= e["k"] <= 8


def test_fixed_dephasing_without_exits_is_plain_stepping():
    """From deep in the left well no replica leaves it within 50 steps: no restart, the
    dephasing takes exactly t_phase steps, and every replica holds the state that plain
    stepping of a copy of the reference walker gives (same noise counters)."""
    spec = _toy(-1.0, 5)
    o = oracle.System(spec)
    o.decorrelate(0)
    rc, d = o.dephase_fixed(50)
    assert rc == 0 and d["n_branch"] == 0 and d["t_steps"] == 50
    ref = oracle.System(spec)
    ref.decorrelate(0)
    q0, v0 = ref.get_state(0)
    for r in range(1, 8):
        ref.set_state(r, q0, v0)
    ref.step_replicas(50, 0, 8)
    for r in range(8):
        assert np.array_equal(o.get_state(r)[0], ref.get_state(r)[0])


def test_budget_resumes_where_it_stopped():
    a = oracle.System(_toy(-0.01, 4))
    b = oracle.System(_toy(-0.01, 4))
    for s in (a, b):
        s.decorrelate(0)
    rc, da = a.dephase_fixed(40)
    steps = 0
    while True:
        rc, db = b.dephase_fixed(40, max_steps=7)
        steps += 1
        if rc == 0:
            break
        assert rc == 1
    assert da == db
    assert np.array_equal(a.get_state(3)[0], b.get_state(3)[0])


@pytest.mark.slow
def test_original_parrep_matches_direct_simulation():
    """With decorrelation and dephasing times long compared with the relaxation inside the
    well, the original ParRep exit times follow those of direct simulation (two-sample KS)."""
    n = 500
    d = direct_exits(oracle.System(G.toy2d(seed=111)), n)
    g = original_parrep_exits(oracle.System(G.toy2d(seed=222)), n, t_corr=100, t_phase=100)
    dd = np.array([x[0] for x in d], float)
    gg = np.array([x[0] for x in g], float)
    assert stats.ks_2samp(dd, gg).pvalue > 0.05
    assert "parallel" in {x[3] for x in g}
