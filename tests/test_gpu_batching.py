"""Batching forms of the persistent path on the GPU: the launch-shape autotuner leaves the
trajectory untouched (results do not depend on the shape, and the tuning runs are undone), and
several systems of uneven size advanced in shared persistent launches end bit-identical to
separate runs."""
import numpy as np
import pytest

import gpr_synth as G
import oracle

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


def _batch_gen_parrep(gpr, systems, n_exits, t_corrs):
    """The loop of Fig. 1 on several systems at once through gpr_batch_run: each system's next
    call follows its own previous result, as in helpers.gen_parrep_exits; systems with enough
    events drop out."""
    logs = [[] for _ in systems]
    last = [s.simulated_steps() for s in systems]
    omega = [s.current_state() for s in systems]
    nxt = [gpr.OP_DECORRELATE] * len(systems)
    rounds = 0
    while any(len(l) < n_exits for l in logs):
        rounds += 1
        assert rounds < 500, logs
        print("round", rounds, [len(l) for l in logs], nxt, flush=True)
        idx = [k for k in range(len(systems)) if len(logs[k]) < n_exits]
        ops = [dict(op=nxt[k], t_corr=t_corrs[k]) for k in idx]
        res = gpr.batch_run([systems[k] for k in idx], ops)
        for k, (st, r) in zip(idx, res):
            assert st == 0
            s = systems[k]
            if nxt[k] == gpr.OP_DECORRELATE:
                if r["kind"] == 1:
                    now = s.simulated_steps()
                    logs[k].append((now - last[k], r["from_state"], r["to_state"], "transient", 0))
                    last[k], omega[k] = now, r["to_state"]
                else:
                    nxt[k] = gpr.OP_DEPHASE
            elif nxt[k] == gpr.OP_DEPHASE:
                if r["outcome"] == 1:
                    now = s.simulated_steps()
                    logs[k].append((now - last[k], omega[k], r["to_state"], "dephase", 0))
                    last[k], omega[k] = now, r["to_state"]
                    nxt[k] = gpr.OP_DECORRELATE
                else:
                    nxt[k] = gpr.OP_PARALLEL_STEP
            else:
                now = s.simulated_steps()
                logs[k].append((now - last[k], omega[k], r["to_state"], "parallel", r["tau_steps"]))
                last[k], omega[k] = now, r["to_state"]
                nxt[k] = gpr.OP_DECORRELATE
    return logs


def test_batch_gen_parrep_matches_separate_systems():
    """The Gen.ParRep loop (transient step, convergence step with branching, parallel step) on
    three systems whose steps share persistent launches (the toy with checks every 10 steps, a
    22-atom chain and a 300-atom receptor-ligand system, each with its state split near its
    start so that exits come within a few checks, checked every 250 and 200 steps): every event,
    its time and the clock equal the same loop run on each system alone, and the final
    configurations are bit-identical."""
    from helpers import gen_parrep_exits
    gpr = _gpr()
    toy = dict(G.toy2d(n_replicas=16, seed=7), pos=np.array([[-0.3], [0.0], [0.0]]))
    # convergence at the first check for the chain and the receptor-ligand system (a tolerance
    # their R-hat always meets), so that their loops reach parallel steps within seconds; the
    # toy converges on R-hat below 1.05
    chain = G.chain(seed=3, n_replicas=8, t_check=250, t_check_parallel=250, tol=1e9)
    psi_b = -np.pi / 2 + 0.08
    chain["state"] = dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=chain["state"]["atoms"],
                          boxes=[[-4.0, 4.0, -4.0, psi_b], [-4.0, 4.0, psi_b, 4.0]])
    # the 300-atom system with its state split at the current value of a ligand dihedral, so
    # that the walker leaves and comes back within a few checks
    rl = G.config("rl300", n_replicas=8, t_check=200, tol=1e9)
    L = rl["n_atoms"] - 32 + 10
    dih = [L, L + 1, L + 2, L + 3]
    o = oracle.System(dict(rl, n_replicas=2, obs=[dict(kind=G.OBS_DIHEDRAL, atoms=dih)]))
    phi0 = o.observables_of(rl["pos"], np.zeros((3, rl["n_atoms"])), 0.0)[0]
    cut = phi0 + 0.05
    rl["state"] = dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=dih + dih,
                       boxes=[[-4.0, cut, -4.0, 4.0], [cut, 4.0, -4.0, 4.0]])
    assert abs(phi0) < np.pi - 0.1
    specs, t_corrs, n = [toy, chain, rl], [100, 500, 400], 3
    batch = [gpr.System(s, path=gpr.PATH_PERSISTENT) for s in specs]
    print("batched Gen.ParRep", flush=True)
    logs = _batch_gen_parrep(gpr, batch, n, t_corrs)
    for k, spec in enumerate(specs):
        solo = gpr.System(spec, path=gpr.PATH_PERSISTENT)
        print("solo Gen.ParRep", k, flush=True)
        ref = gen_parrep_exits(solo, n, t_corrs[k])
        assert logs[k] == ref, (k, logs[k], ref)
        assert batch[k].simulated_steps() == solo.simulated_steps()
        assert batch[k].global_step() == solo.global_step()
        _same(batch[k], solo, range(spec["n_replicas"]))
    kinds = {e[3] for l in logs for e in l}
    assert "parallel" in kinds
