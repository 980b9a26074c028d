"""GPU edge cases, through the C ABI: the largest systems the LDS-resident kernels take and a
clean refusal beyond them, workgroups that own no atoms, the smallest replica count, launch
shapes the device cannot hold, and the degenerate Fleming-Viot check at which every worker
exits (all are re-copied from the reference walker and the accumulators restart)."""
import sys

import numpy as np
import pytest

import gpr_synth as G
import oracle

pytestmark = pytest.mark.gpu


def _gpr():
    import paper_1807_02431_amd as gpr
    return gpr


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _force_err(Fg, Fo):
    return np.abs(Fg - Fo).max() / np.abs(Fo).max()


def test_largest_persistent_system():
    """4,600 atoms (receptor 4,568 + ligand 32 in a 5 nm sphere), 8 replicas: the persistent path
    splits each replica over 8 workgroups (fewer do not fit in LDS); forces of sampled replicas
    match the oracle, and both stepping paths give identical bits."""
    gpr = _gpr()
    spec = G.round_to_f32(G.receptor_ligand(n_receptor=4568, radius=5.0, n_replicas=8))
    say("largest persistent system, n =", spec["n_atoms"])
    runs = []
    for path in (gpr.PATH_PERSISTENT, gpr.PATH_PLAIN):
        g = gpr.System(spec, path=path)
        g.advance(25)
        runs.append(np.stack([g.get_state(r)[0] for r in range(8)]))
    assert np.array_equal(runs[0], runs[1])
    E, F = g.energy_forces()
    o = oracle.System(dict(spec, n_replicas=2))
    for r in (0, 7):
        Uo, Fo = o.eval(runs[0][r])
        err = _force_err(F[r], Fo)
        say("replica", r, "force rel err", err)
        assert err < 1e-5
        assert abs(E[r] - Uo) <= 1e-5 * abs(Uo)


def test_system_beyond_persistent_limit_runs_plain():
    """5,200 atoms: no split of a replica fits the persistent kernel's LDS, so selecting that
    path is refused with EINVAL and nothing changes; the plain path still matches the oracle."""
    gpr = _gpr()
    spec = G.round_to_f32(G.receptor_ligand(n_receptor=5168, radius=5.2, n_replicas=2))
    say("beyond persistent limit, n =", spec["n_atoms"])
    g = gpr.System(spec)
    with pytest.raises(gpr.GprError) as e:
        g.set_path(gpr.PATH_PERSISTENT)
    assert e.value.code == -1
    g.advance(10)
    E, F = g.energy_forces()
    o = oracle.System(spec)
    q, _ = g.get_state(1)
    Uo, Fo = o.eval(q)
    assert _force_err(F[1], Fo) < 1e-5


def test_system_too_large_is_refused():
    """6,500 atoms exceed the LDS of the plain pair kernel too: creation fails with EINVAL."""
    gpr = _gpr()
    spec = G.receptor_ligand(n_receptor=6468, radius=5.6, n_replicas=2)
    say("too large, n =", spec["n_atoms"])
    with pytest.raises(gpr.GprError) as e:
        gpr.System(spec)
    assert e.value.code == -1


def test_groups_without_atoms_and_two_replicas():
    """The 22-atom chain split over 8 workgroups of 64 threads (six of them own no atom) and with
    2 replicas, the smallest count: positions match the oracle after 100 steps, and the bits
    equal the plain path's after 100 and after 300 steps."""
    gpr = _gpr()
    spec = G.round_to_f32(G.config("chain22", n_replicas=2))
    say("empty groups, chain22 x 2")
    a = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    a.set_launch(64, 8)
    b = gpr.System(spec, path=gpr.PATH_PLAIN)
    o = oracle.System(spec)
    o.step_replicas(100, 0, 2)
    for steps in (100, 200):
        a.advance(steps)
        b.advance(steps)
        for r in range(2):
            qa, va = a.get_state(r)
            qb, vb = b.get_state(r)
            assert np.array_equal(qa, qb) and np.array_equal(va, vb)
            if steps == 100:
                qo, _ = o.get_state(r)
                assert np.abs(qa - qo).max() < 1e-5 * np.abs(qo).max()


def test_impossible_launch_shape_is_refused_and_changes_nothing():
    gpr = _gpr()
    spec = G.config("rl2432")
    g = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    for bt, grp in ((1024, 1), (100, 4), (1024, 3)):
        with pytest.raises(gpr.GprError) as e:
            g.set_launch(bt, grp)
        assert e.value.code == -1
    ref = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    g.advance(20)
    ref.advance(20)
    assert np.array_equal(g.get_state(5)[0], ref.get_state(5)[0])


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("seed", [19, 25])
def test_every_worker_exits_at_a_check(path, seed):
    """Two replicas started at x = -0.05 on the toy: at the first check of the dephasing the one
    worker has crossed to x > 0 while the reference walker has not (seeds chosen with the
    oracle; the crossing margin is > 1e-4).  With no survivor the worker is re-copied from the
    reference walker and the accumulators restart, as the oracle does."""
    gpr = _gpr()
    spec = G.round_to_f32(dict(G.toy2d(n_replicas=2, seed=seed), pos=np.array([[-0.05], [0.0], [0.0]])))
    say("all workers exit, seed", seed, "path", path)
    g = gpr.System(spec, path=path)
    o = oracle.System(spec)
    for s in (g, o):
        rc, ev = s.decorrelate(0)
        assert rc == 0 and ev["to_state"] == 0
        rc, out = s.dephase(10)
        assert rc == 1
    for s in (g, o):
        q0, v0 = s.get_state(0)
        q1, v1 = s.get_state(1)
        assert np.array_equal(q0, q1) and np.array_equal(v0, v1)
        assert s.accumulators()[0] == 0
    assert np.abs(g.get_state(0)[0] - o.get_state(0)[0]).max() < 1e-5
    assert g.simulated_steps() == o.simulated_steps()


@pytest.mark.parametrize("path", [0, 1])
def test_overlapping_atoms_are_reported_unstable(path):
    """Two non-bonded atoms placed 0.001 nm apart (forced from the host with gpr_set_state): the
    Lennard-Jones force, far beyond any stable value, is reported as GPR_EUNSTABLE by the next
    call that steps, on both paths; the other replica stays finite."""
    gpr = _gpr()
    spec = G.config("rl300", n_replicas=2)
    say("overlap, path", path)
    g = gpr.System(spec, path=path)
    q0, _ = g.get_state(0)
    q, v = g.get_state(1)
    q[:, 10] = q[:, 200] + np.array([1e-3, 0.0, 0.0])
    g.set_state(1, q, v)
    with pytest.raises(gpr.GprError) as e:
        g.advance(20)
    assert e.value.code == -5
    assert np.isfinite(g.get_state(0)[0]).all()


def _scrambled_chain(n=64, R=4):
    """A chain of the 22-atom workload's force field, n atoms long, whose atom indices are
    permuted (chain atom k becomes atom 17 k mod n) so that neighbours along the chain sit 17 or
    47 indices apart: its excluded and 1-4 pairs join atoms up to 51 indices apart (beyond the
    per-atom bit mask), as in rings or branched molecules, while the geometry stays that of a
    relaxed chain."""
    spec = G.chain(seed=4, n_atoms=n, n_replicas=R)
    new = (17 * np.arange(n)) % n
    out = dict(spec)
    for key in ("mass", "sigma", "epsilon", "charge"):
        v = np.asarray(spec[key], np.float64)
        w = np.empty_like(v)
        w[new] = v
        out[key] = w
    pos = np.asarray(spec["pos"], np.float64)
    out["pos"] = np.empty_like(pos)
    out["pos"][:, new] = pos
    for key in ("bonds", "angles", "torsions", "pairs14", "exclusions"):
        out[key] = new[np.asarray(spec[key])].astype(np.int32)
    st = dict(spec["state"])
    st["atoms"] = [int(new[a]) for a in st["atoms"]]
    out["state"] = st
    obs = []
    for o in spec["obs"]:
        o = dict(o)
        if "atoms" in o:
            o["atoms"] = [int(new[a]) for a in o["atoms"]]
        obs.append(o)
    out["obs"] = obs
    return G.round_to_f32(out)


@pytest.mark.parametrize("path", [0, 1])
def test_far_exclusions_match_oracle(path):
    """Excluded and 1-4 pairs of a chain whose atom indices are scrambled lie up to 51 indices
    apart (beyond the per-atom bit mask): forces and energies at the start and positions after
    100 steps match the oracle, which excludes them by definition."""
    gpr = _gpr()
    spec = _scrambled_chain()
    span = max(np.abs(np.diff(spec[k], axis=1)).max() for k in ("exclusions", "pairs14"))
    assert span >= 32
    say("scrambled chain, path", path)
    g = gpr.System(spec, path=path)
    o = oracle.System(spec)
    Eg, Fg = g.energy_forces()
    Eo, Fo = o.energy_forces()
    for r in range(spec["n_replicas"]):
        assert np.abs(Fg[r] - Fo[r]).max() < 1e-5 * np.abs(Fo[r]).max()
        assert abs(Eg[r] - Eo[r]) <= 1e-5 * max(1.0, abs(Eo[r]))
    g.advance(100)
    o.step_replicas(100, 0, spec["n_replicas"])
    for r in range(spec["n_replicas"]):
        qg, _ = g.get_state(r)
        qo, _ = o.get_state(r)
        assert np.abs(qg - qo).max() < 1e-5 * np.abs(qo).max()


@pytest.mark.parametrize("path", [0, 1])
def test_advance_without_first_exit_readback(path):
    """gpr_advance with first_exit_check = NULL records and reads back nothing of the checks
    and takes the same steps: after calls without the readback, a call with it reports the
    first exit checks of its own steps only (counted over all calls), as on a handle that read
    them back all along.  The 300-atom system's state is split near its start so that
    replicas leave it within a few checks (t_check = 20)."""
    gpr = _gpr()
    rl = G.config("rl300", n_replicas=8, t_check=20)
    L = rl["n_atoms"] - 32 + 10
    dih = [L, L + 1, L + 2, L + 3]
    o = oracle.System(dict(rl, n_replicas=2, obs=[dict(kind=G.OBS_DIHEDRAL, atoms=dih)]))
    phi0 = o.observables_of(rl["pos"], np.zeros((3, rl["n_atoms"])), 0.0)[0]
    rl["state"] = dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=dih + dih,
                       boxes=[[-4.0, phi0 + 0.02, -4.0, 4.0], [phi0 + 0.02, 4.0, -4.0, 4.0]])
    a = gpr.System(rl, path=path)
    b = gpr.System(rl, path=path)
    say("advance without readback, path", path)
    fa = [a.advance(30) for _ in range(3)]
    for _ in range(3):
        assert b.advance(30, first_exit=False) is None
    assert a.advance_steps() == b.advance_steps() == 90
    for r in range(8):
        assert np.array_equal(a.get_state(r)[0], b.get_state(r)[0])
        assert np.array_equal(a.get_state(r)[1], b.get_state(r)[1])
    ga, gb = a.advance(60), b.advance(60)
    assert np.array_equal(ga, gb)
    # checks at steps 100, 120, 140 of the schedule: indices 5, 6, 7
    assert all(v == 0 or 5 <= v <= 7 for v in gb), gb
    assert any(np.any(f > 0) for f in fa + [ga]), "no replica left the state; the split is too far"
