"""Batching forms of the persistent path on the GPU: the launch-shape autotuner leaves the
trajectory untouched (results do not depend on the shape, and the tuning runs are undone)."""
import numpy as np
import pytest

import gpr_synth as G

pytestmark = pytest.mark.gpu


def _gpr():
    import paper_1807_02431_amd as gpr
    return gpr


@pytest.mark.parametrize("name", ["rl300", "rl2432"])
def test_autotune_keeps_the_trajectory(name):
    gpr = _gpr()
    spec = G.config(name, n_replicas=8)
    a = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    b = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    a.advance(30)
    b.advance(30)
    bt, g = a.autotune(40)
    assert bt in (256, 512, 768, 1024) and g in (1, 2, 4, 8)
    assert a.simulated_steps() == b.simulated_steps() and a.global_step() == b.global_step()
    a.advance(120)
    b.advance(120)
    for r in range(8):
        qa, va = a.get_state(r)
        qb, vb = b.get_state(r)
        assert np.array_equal(qa, qb) and np.array_equal(va, vb)
    na, S1a, S2a, _ = a.accumulators()
    nb, S1b, S2b, _ = b.accumulators()
    assert na == nb and np.array_equal(S1a, S1b) and np.array_equal(S2a, S2b)
