"""GPU against the oracle on the Gen.ParRep steps the product runs (Sec. 2.4): the parallel
step's exit vote and clock (Sec. 2.4.2, Eqs. 5-6) from the same converged dephasing, a
convergence step on the 22-atom chain with branching (Sec. 2.4.1), the replicas of one system
inside a shared multi-system launch, and transient propagation through configurations in no
state (Sec. 2.2, Sec. 2.4 transient step).

Bars: integer bookkeeping (M, k, tau, to_state, the clock, the partition of the workers into
clones, sample and branch counts) identical; positions within 1e-5 of the largest coordinate;
R-hat, whose FP64 sums are fed by FP32 observables on the GPU, within 1e-3 relative."""
import math
import sys

import numpy as np
import pytest

import gpr_synth as G
import oracle
from helpers import mini

pytestmark = pytest.mark.gpu


def _gpr():
    import paper_1807_02431_amd as gpr
    return gpr


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pos_err(qg, qo):
    return np.abs(qg - qo).max() / max(np.abs(qo).max(), 1e-30)


def _clone_groups(q):
    groups = {}
    for r in range(1, len(q)):
        groups.setdefault(q[r].tobytes(), []).append(r)
    return sorted(tuple(g) for g in groups.values())


@pytest.mark.parametrize("path", [0, 1])
def test_parallel_step_matches_oracle(path):
    """64 toy walkers released near the barrier top (x = -0.05): a convergence step with a
    tolerance that the first check meets, then the parallel step.  Both sides take the same
    branching, reach the same (M, k, tau_steps, to_state), advance the clock by the same
    t_FV + tau and put the same exit configuration X^k into replica 0."""
    gpr = _gpr()
    cases = 0
    k_gt1 = 0
    for seed in range(40, 60):
        spec = G.round_to_f32(dict(G.toy2d(n_replicas=64, seed=seed, tol=1e9), pos=np.array([[-0.05], [0.0], [0.0]])))
        say("parallel step, seed", seed, "path", path)
        g = gpr.System(spec, path=path)
        o = oracle.System(spec)
        outs = []
        for s in (g, o):
            rc, ev = s.decorrelate(0)
            assert rc == 0 and ev["kind"] == 0 and ev["to_state"] == 0
            rc, d = s.dephase()
            assert rc == 0
            outs.append(d)
        dg, do = outs
        assert (dg["outcome"], dg["to_state"], dg["t_steps"], dg["n_branch"], dg["n_samples"]) == \
               (do["outcome"], do["to_state"], do["t_steps"], do["n_branch"], do["n_samples"])
        if dg["outcome"] != 0:
            continue                                   # the reference walker left first
        assert np.allclose(dg["rhat"], do["rhat"], rtol=1e-3)
        qg = np.stack([g.get_state(r)[0][:, 0] for r in range(64)])
        qo = np.stack([o.get_state(r)[0][:, 0] for r in range(64)])
        assert _clone_groups(qg) == _clone_groups(qo)
        rc, eg = g.parallel_step()
        assert rc == 0
        rc, eo = o.parallel_step()
        assert rc == 0
        for key in ("M", "k", "tau_steps", "to_state"):
            assert eg[key] == eo[key], (seed, key, eg, eo)
        assert eg["tau_steps"] == (64 * (eg["M"] - 1) + eg["k"]) * 10
        assert eg["tau"] == pytest.approx(eg["tau_steps"] * 0.01, rel=1e-15)
        assert g.simulated_steps() == o.simulated_steps() == dg["t_steps"] + eg["tau_steps"]
        assert g.global_step() == o.global_step()
        assert g.current_state() == o.current_state() == eg["to_state"]
        q0g, _ = g.get_state(0)
        q0o, _ = o.get_state(0)
        qkg, _ = g.get_state(eg["k"] - 1)
        assert np.array_equal(q0g, qkg)                # X^k copied into replica 0
        assert _pos_err(q0g, q0o) < 1e-5
        cases += 1
        k_gt1 += eg["k"] > 1
        if cases >= 6 and k_gt1 >= 2:
            break
    assert cases >= 3 and k_gt1 >= 1, (cases, k_gt1)


def _chain_band(seed, R=16, d=0.06):
    """The 22-atom chain with its state split by psi at psi0 + d (phi ignored): workers
    starting at psi0 cross within one 250-step check often, so that a check branches."""
    spec = G.chain(seed=seed, n_replicas=R, tol=1e9)
    psi_b = -math.pi / 2 + d
    spec["state"] = dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=spec["state"]["atoms"],
                         boxes=[[-4.0, 4.0, -4.0, psi_b], [-4.0, 4.0, psi_b, 4.0]])
    return G.round_to_f32(spec)


@pytest.mark.parametrize("path", [0, 1])
def test_chain_dephasing_check_matches_oracle(path):
    """One convergence-step check on the 22-atom chain (t_GR = 10, t_check = 250) with
    exits among the 15 workers: the same outcome, t_FV, branch and sample counts and clone
    partition as the oracle, positions within 1e-5, R-hat within 1e-3 relative."""
    gpr = _gpr()
    compared = 0
    for seed in range(2, 14):
        spec = _chain_band(seed)
        say("chain dephasing, seed", seed, "path", path)
        g = gpr.System(spec, path=path)
        o = oracle.System(spec)
        outs = []
        for s in (g, o):
            rc, ev = s.decorrelate(0)
            assert rc == 0 and ev["kind"] == 0
            rc, d = s.dephase()
            assert rc == 0
            outs.append(d)
        dg, do = outs
        for key in ("outcome", "to_state", "t_steps", "n_branch", "n_samples"):
            assert dg[key] == do[key], (seed, key, dg, do)
        if dg["outcome"] != 0 or dg["n_branch"] == 0:
            continue
        assert np.allclose(dg["rhat"], do["rhat"], rtol=1e-3), (dg["rhat"], do["rhat"])
        qg = np.stack([g.get_state(r)[0] for r in range(16)])
        qo = np.stack([o.get_state(r)[0] for r in range(16)])
        assert _clone_groups(qg) == _clone_groups(qo)
        assert max(_pos_err(qg[r], qo[r]) for r in range(16)) < 1e-5
        ng, S1g, S2g, _ = g.accumulators()
        no, S1o, S2o, _ = o.accumulators()
        assert ng == no
        assert np.allclose(S1g, S1o, rtol=1e-4, atol=1e-4 * np.abs(S1o).max())
        compared += 1
        if compared >= 2:
            break
    assert compared >= 1


def test_batched_system_replicas_match_oracle():
    """Replicas of the 22-atom chain and of a 300-atom receptor-ligand system advanced 100
    steps in shared persistent launches, compared replica by replica with the oracle."""
    gpr = _gpr()
    specs = [G.round_to_f32(G.config("chain22", n_replicas=4)), G.round_to_f32(G.config("rl300", n_replicas=4))]
    batch = [gpr.System(s, path=gpr.PATH_PERSISTENT) for s in specs]
    say("batched vs oracle")
    gpr.batch_advance(batch, 100)
    for spec, g in zip(specs, batch):
        o = oracle.System(spec)
        o.step_replicas(100, 0, 4)
        for r in range(4):
            err = _pos_err(g.get_state(r)[0], o.get_state(r)[0])
            assert err < 1e-5, (spec["n_atoms"], r, err)


# ------------------------------------------------------------------ states with gaps
def _butane(seed, R=2):
    """Four atoms with one torsion (minima at +-60 and 180 degrees), state = a box around
    each gauche minimum; the trans region between them is no state."""
    def four(a):
        return [[0.15, 0, 0], [0, 0, 0], [0, 0, 0.15], [0.15 * math.cos(a), 0.15 * math.sin(a), 0.15]]
    boxes = [[math.radians(-100), math.radians(-20), -4, 4], [math.radians(20), math.radians(100), -4, 4]]
    spec = mini(four(math.pi), mass=[12.0] * 4, epsilon=0.0, R=R, seed=seed, kT=G.KB * 300.0,
                bonds=np.array([[0, 1], [1, 2], [2, 3]], np.int32), bond_r0=np.full(3, 0.15),
                bond_k=np.full(3, 2.0e5), angles=np.array([[0, 1, 2], [1, 2, 3]], np.int32),
                angle_theta0=np.full(2, math.pi / 2), angle_k=np.full(2, 400.0),
                torsions=np.array([[0, 1, 2, 3]], np.int32), torsion_n=np.array([3], np.int32),
                torsion_k=np.array([2.0]), torsion_phi0=np.array([0.0]),
                t_check_dephase=10, t_check_parallel=10,
                state=dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=[0, 1, 2, 3, 0, 1, 2, 3], boxes=boxes))
    spec["vel"] = None
    return G.round_to_f32(spec)


def _replay(gpr, spec, t_corr, path, max_checks=100000):
    """The rules of the transient step applied to the GPU's own trajectory of replica 0,
    stepped one check period at a time by gpr_advance (replica 0's noise depends only on the
    global step, so the trajectory is the one gpr_decorrelate follows)."""
    s = gpr.System(spec, path=path)
    tc = spec["t_check_dephase"]
    cur = int(s.observe()[1][0])
    start, resid = cur, 0
    for m in range(1, max_checks + 1):
        if cur != -1 and resid >= t_corr:
            return dict(kind=0, from_state=start, to_state=cur, resident_steps=resid, steps_taken=(m - 1) * tc)
        s.advance(tc)
        st = int(s.observe()[1][0])
        if st == cur:
            resid += tc
        elif cur == -1:
            cur, resid = st, 0
        else:
            return dict(kind=1, from_state=cur, to_state=st, resident_steps=resid + tc, steps_taken=m * tc)
    raise AssertionError("no event")


@pytest.mark.parametrize("path", [0, 1])
def test_transient_step_through_no_state_gpu(path):
    """The transient step on the GPU leaves the trans region (no state) and reports -1 as the
    starting state and as the state of an exit into the gap, with the reaching time on the
    clock; its events equal the rules applied to its own trajectory; the state ids of the
    configurations it passes through equal the oracle's."""
    gpr = _gpr()
    o = oracle.System(_butane(1))
    seen_from_none = seen_to_none = 0
    for seed in range(11, 19):
        spec = _butane(seed)
        say("transient through no state, seed", seed, "path", path)
        g = gpr.System(spec, path=path)
        assert int(g.observe()[1][0]) == -1
        rc, ev = g.decorrelate(300)
        assert rc == 0 and g.simulated_steps() == ev["steps_taken"]
        ref = _replay(gpr, spec, 300, path)
        assert ev == ref, (seed, ev, ref)
        seen_from_none += ev["kind"] == 0 and ev["from_state"] == -1
        seen_to_none += ev["kind"] == 1 and ev["to_state"] == -1
        q, _ = g.get_state(0)
        assert g.observe()[1][0] == o.state_of(q)
        with pytest.raises(gpr.GprError) if g.current_state() == -1 else _nothing():
            g.dephase(10)
    assert seen_from_none >= 1 and seen_to_none >= 1, (seen_from_none, seen_to_none)


class _nothing:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False
