"""GPU parity of the original ParRep dephasing (Sec. 2.4.3) through the C ABI: exact agreement
with the oracle where no replica leaves the state, its invariants where replicas restart, and
the exit statistics of the whole original ParRep loop on the GPU against the oracle's direct
simulation."""
import numpy as np
import pytest
from scipy import stats

import gpr_synth as G
import oracle
from helpers import direct_exits, original_parrep_exits

pytestmark = pytest.mark.gpu


def _gpr():
    import paper_1807_02431_amd as gpr
    return gpr


def _toy(x0, seed, R=8):
    return G.round_to_f32(dict(G.toy2d(n_replicas=R, seed=seed), pos=np.array([[x0], [0.0], [0.0]])))


@pytest.mark.parametrize("path", [0, 1])
def test_fixed_dephasing_matches_oracle_without_exits(path):
    gpr = _gpr()
    spec = _toy(-1.0, 5)
    g = gpr.System(spec, path=path)
    o = oracle.System(spec)
    out = []
    for s in (g, o):
        s.decorrelate(0)
        rc, d = s.dephase_fixed(50)
        assert rc == 0
        out.append(d)
    assert out[0] == out[1] and out[0]["n_branch"] == 0
    for r in range(8):
        assert np.abs(g.get_state(r)[0] - o.get_state(r)[0]).max() < 1e-5


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("seed", [3, 4, 6])
def test_fixed_dephasing_invariants_with_restarts(path, seed):
    gpr = _gpr()
    g = gpr.System(_toy(-0.01, seed), path=path)
    rc, ev = g.decorrelate(0)
    assert rc == 0 and ev["to_state"] == 0
    t0 = g.simulated_steps()
    rc, d = g.dephase_fixed(40)
    assert rc == 0 and d["outcome"] == 0
    assert g.simulated_steps() == t0
    assert d["t_steps"] % 10 == 0 and d["t_steps"] >= 40
    assert np.all(g.observe()[1] == 0)
    rc, e = g.parallel_step()
    assert rc == 0 and 1 <= e["k"] <= 8


@pytest.mark.slow
def test_gpu_original_parrep_matches_direct_simulation():
    gpr = _gpr()
    n = 500
    g = original_parrep_exits(gpr.System(G.toy2d(seed=333), path=gpr.PATH_PERSISTENT), n, t_corr=100, t_phase=100)
    d = direct_exits(oracle.System(G.toy2d(seed=111)), n)
    gg = np.array([x[0] for x in g], float)
    dd = np.array([x[0] for x in d], float)
    assert stats.ks_2samp(gg, dd).pvalue > 0.05
