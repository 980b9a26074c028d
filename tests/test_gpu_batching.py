"""Batching forms of the persistent path on the GPU: the launch-shape autotuner leaves the
trajectory untouched (results do not depend on the shape, and the tuning runs are undone), and
several systems of uneven size advanced in shared persistent launches end bit-identical to
separate runs."""
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


def _same(a, b, reps):
    for r in reps:
        qa, va = a.get_state(r)
        qb, vb = b.get_state(r)
        assert np.array_equal(qa, qb) and np.array_equal(va, vb), r


def test_batch_advance_matches_separate_systems():
    """Three systems (22, 300 and 2,432 atoms; exit checks every 250, 1,000 and 1,000 steps) in
    shared persistent launches: each ends bit-identical to its own gpr_advance, first exit
    checks and observable accumulators included."""
    gpr = _gpr()
    specs = [G.config("chain22", n_replicas=8), G.config("rl300", n_replicas=8), G.config("rl2432", n_replicas=8)]
    batch = [gpr.System(s, path=gpr.PATH_PERSISTENT) for s in specs]
    solo = [gpr.System(s, path=gpr.PATH_PERSISTENT) for s in specs]
    fb = gpr.batch_advance(batch, 1300)
    for a, b, f in zip(batch, solo, fb):
        assert np.array_equal(f, b.advance(1300))
        _same(a, b, range(8))
        na, S1a, S2a, _ = a.accumulators()
        nb, S1b, S2b, _ = b.accumulators()
        assert na == nb and np.array_equal(S1a, S1b) and np.array_equal(S2a, S2b)
        assert a.global_step() == b.global_step()


def test_uneven_batch_of_768_replicas():
    """The uneven mix, 22 / 300 / 1,200 / 2,432 atoms x 192 replicas each, in shared launches
    in which sets of workgroups take a system's replicas in turn: sampled replicas are
    bit-identical to separate runs of each system."""
    gpr = _gpr()
    specs = G.uneven_batch(192)
    batch = [gpr.System(s, path=gpr.PATH_PERSISTENT) for s in specs]
    fb = gpr.batch_advance(batch, 300)
    for spec, a, f in zip(specs, batch, fb):
        b = gpr.System(spec, path=gpr.PATH_PERSISTENT)
        assert np.array_equal(f, b.advance(300))
        _same(a, b, (0, 95, 191))
        del b


def test_batch_advance_refuses_bad_input():
    """A system twice, more than eight systems, a negative step count: EINVAL, nothing run."""
    gpr = _gpr()
    a = gpr.System(G.config("rl300", n_replicas=4), path=gpr.PATH_PERSISTENT)
    with pytest.raises(gpr.GprError) as e:
        gpr.batch_advance([a, a], 10)
    assert e.value.code == -1
    many = [gpr.System(G.config("chain22", n_replicas=2), path=gpr.PATH_PERSISTENT) for _ in range(9)]
    with pytest.raises(gpr.GprError) as e:
        gpr.batch_advance(many, 10)
    assert e.value.code == -1
    with pytest.raises(gpr.GprError) as e:
        gpr.batch_advance([a], -1)
    assert e.value.code == -1
    assert a.global_step() == 0 and all(x.global_step() == 0 for x in many)
    # eight is the most a shared launch takes
    f = gpr.batch_advance(many[:8], 20)
    assert len(f) == 8 and all(x.global_step() == 20 for x in many[:8])
