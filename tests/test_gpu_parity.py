"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bars: bit-exact for integer and index work (Philox words, Fleming-Viot plans, exit votes)
and for the FP64 Gelman-Rubin reduction on identical inputs; forces within 1e-5 of the
largest force component (per replica) at identical positions; positions within 1e-5 of the
largest coordinate after 100 BAOAB steps under identical Philox streams, velocities within
the bar that this implies through the stiffest harmonic term (_vel_bar); the two stepping
paths bit-identical to each other; exit statistics by a two-sample KS test (p > 0.05)."""
import sys

import numpy as np
import pytest
from scipy import stats

import gpr_synth as G
import oracle

pytestmark = pytest.mark.gpu


def _gpr():
    import paper_1807_02431_amd as gpr
    return gpr


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------------ building blocks
def test_philox_words_bit_exact_and_gaussians():
    gpr = _gpr()
    for seed, rep, step, stream, n in ((1, 0, 0, 0, 1000), (0xDEADBEEFCAFE, 37, (3 << 32) + 5, 0, 777),
                                       (7, 255, 123456, 1, 300), (99, 3, 17, 2, 64)):
        wg, gg = gpr.philox_noise(seed, rep, step, stream, n)
        wo, go = oracle.noise(seed, rep, step, stream, n)
        assert np.array_equal(wg, wo)
        assert np.allclose(gg, go, rtol=1e-6, atol=2e-6)


def test_fv_plan_bit_exact():
    gpr = _gpr()
    rng = np.random.default_rng(4)
    for R in (2, 8, 64, 256, 1000):
        for trial in range(20):
            p = rng.choice([0.0, 0.1, 0.5, 0.95, 1.0])
            ex = (rng.random(R) < p).astype(np.uint8)
            step = int(rng.integers(0, 2 ** 40))
            assert np.array_equal(gpr.fv_plan(11, step, ex), oracle.fv_plan(11, step, ex)), (R, trial)


def test_rhat_bit_exact():
    gpr = _gpr()
    rng = np.random.default_rng(5)
    for nw, no in ((1, 1), (7, 3), (63, 6), (255, 8), (1023, 4)):
        n = int(rng.integers(2, 500))
        S1 = rng.normal(size=(nw, no)) * n
        S2 = np.abs(rng.normal(size=(nw, no))) * n * 3 + S1 ** 2 / n
        g = gpr.rhat(n, S1, S2)
        o = oracle.rhat(n, S1, S2)
        assert np.array_equal(g.view(np.uint64), o.view(np.uint64)), (nw, g, o)


def test_exit_vote_bit_exact():
    gpr = _gpr()
    rng = np.random.default_rng(6)
    for R in (1, 4, 64, 300):
        for _ in range(50):
            fec = rng.integers(0, 6, R)
            assert gpr.exit_vote(fec, 1000) == oracle.exit_vote(fec, 1000)


# ------------------------------------------------------------------ forces and energies
def _force_err(Fg, Fo):
    return np.abs(Fg - Fo).max() / np.abs(Fo).max()


@pytest.mark.parametrize("name,kw", [("toy", {}), ("chain22", dict(n_replicas=4)),
                                     ("rl300", dict(n_replicas=4))])
def test_forces_energy_parity_small(name, kw):
    gpr = _gpr()
    spec = G.config(name, **kw)
    if name == "toy":
        spec["pos"] = np.array([[-0.7], [0.3], [0.0]])     # off the minimum: nonzero force
    spec = G.round_to_f32(spec)
    say("forces", name)
    g = gpr.System(spec)
    o = oracle.System(spec)
    Eg, Fg = g.energy_forces()
    Eo, Fo = o.energy_forces()
    for r in range(spec["n_replicas"]):
        assert _force_err(Fg[r], Fo[r]) < 1e-5
        assert abs(Eg[r] - Eo[r]) <= 1e-5 * max(1.0, abs(Eo[r]))


def test_forces_parity_full_size_sampled():
    """2,432 atoms x 64 replicas after 30 steps: each sampled replica's GPU positions are
    handed to the oracle, whose FP64 forces and energy are compared element by element."""
    gpr = _gpr()
    spec = G.round_to_f32(G.config("rl2432"))
    say("forces rl2432")
    g = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    g.advance(30)
    o = oracle.System(dict(spec, n_replicas=2))
    Eg, Fg = g.energy_forces()
    for r in (0, 1, 37, 63):
        q, _ = g.get_state(r)
        Uo, Fo = o.eval(q)
        err = _force_err(Fg[r], Fo)
        say("replica", r, "force rel err", err, "energy", Eg[r], Uo)
        assert err < 1e-5
        assert abs(Eg[r] - Uo) <= 1e-5 * abs(Uo)


# ------------------------------------------------------------------ trajectories
def _pos_err(qg, qo):
    return np.abs(qg - qo).max() / np.abs(qo).max()


def _vel_bar(spec, qo):
    """The velocity bar that the position bar implies.  The fastest motion is the stiffest
    harmonic term (bond: omega = sqrt(k / mu), mu the reduced mass; restraint: sqrt(k / m)),
    and a position error dx on it appears in the velocity as about omega * dx; with dx at the
    position bar, 1e-5 of the largest coordinate: |dv| <= omega_max * 1e-5 * max|x|."""
    m = np.asarray(spec["mass"], np.float64)
    b = np.asarray(spec["bonds"]).reshape(-1, 2)
    om = 0.0
    if len(b):
        mu = m[b[:, 0]] * m[b[:, 1]] / (m[b[:, 0]] + m[b[:, 1]])
        om = np.sqrt(np.asarray(spec["bond_k"], np.float64) / mu).max()
    ri = np.asarray(spec.get("restraints", []), np.int64)
    if len(ri):
        om = max(om, np.sqrt(np.asarray(spec["restraint_k"], np.float64) / m[ri]).max())
    assert om > 0
    return om * 1e-5 * np.abs(qo).max()


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("name", ["chain22", "rl300"])
def test_positions_100_steps_small(name, path):
    gpr = _gpr()
    spec = G.round_to_f32(G.config(name, n_replicas=4))
    say("positions", name, "path", path)
    g = gpr.System(spec, path=path)
    o = oracle.System(spec)
    g.advance(100)
    o.step_replicas(100, 0, 4)
    assert g.global_step() == o.global_step() == 100
    for r in range(4):
        qg, vg = g.get_state(r)
        qo, vo = o.get_state(r)
        err = _pos_err(qg, qo)
        assert err < 1e-5, (r, err)
        assert np.abs(vg - vo).max() < _vel_bar(spec, qo), (r, np.abs(vg - vo).max(), _vel_bar(spec, qo))


@pytest.mark.parametrize("path", [0, 1])
def test_positions_100_steps_full_size_sampled(path):
    gpr = _gpr()
    spec = G.round_to_f32(G.config("rl2432"))
    say("positions rl2432 path", path)
    g = gpr.System(spec, path=path)
    g.advance(100)
    for r in (0, 37, 63):
        o = oracle.System(spec)
        o.step_replicas(100, r, r + 1)
        qg, vg = g.get_state(r)
        qo, vo = o.get_state(r)
        err = _pos_err(qg, qo)
        dv = np.abs(vg - vo).max()
        say("replica", r, "pos rel err", err, "vel err", dv, "bar", _vel_bar(spec, qo))
        assert err < 1e-5
        assert dv < _vel_bar(spec, qo)


def test_plain_and_persistent_paths_bit_identical():
    """Same arithmetic on both paths, fixed-point force accumulation, sub-lists in index
    order: identical bits, across pair-list rebuilds, launch shapes (block size, replica split
    over 1, 2 or 4 workgroups) and repeated runs."""
    gpr = _gpr()
    spec = G.config("rl300", n_replicas=8)
    say("bit identity rl300")
    runs = []
    for path, bt, groups in ((0, 0, 0), (1, 0, 1), (1, 320, 1), (1, 1024, 1), (1, 0, 2), (1, 256, 4), (0, 0, 0)):
        s = gpr.System(spec, path=path)
        if bt or groups:
            s.set_launch(bt, groups)
        s.advance(120)
        q = np.stack([s.get_state(r)[0] for r in range(8)])
        v = np.stack([s.get_state(r)[1] for r in range(8)])
        E, F = s.energy_forces()
        runs.append((q, v, F, E))
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)


def test_observables_and_states_parity():
    gpr = _gpr()
    spec = G.round_to_f32(G.config("rl300", n_replicas=4))
    g = gpr.System(spec)
    g.advance(40)
    o = oracle.System(spec)
    obs, st = g.observe()
    E, _ = g.energy_forces()
    for r in range(4):
        q, v = g.get_state(r)
        Uo, _ = o.eval(q)
        ref = o.observables_of(q, v, Uo)
        assert np.allclose(obs[r], ref, rtol=1e-5, atol=1e-6), (obs[r], ref)
        assert st[r] == o.state_of(q)
    spec2 = G.round_to_f32(G.config("chain22", n_replicas=4))
    g2 = gpr.System(spec2)
    g2.advance(200)
    o2 = oracle.System(spec2)
    obs, st = g2.observe()
    for r in range(4):
        q, v = g2.get_state(r)
        Uo, _ = o2.eval(q)
        assert np.allclose(obs[r], o2.observables_of(q, v, Uo), rtol=1e-5, atol=1e-6)
        assert st[r] == o2.state_of(q)


# ------------------------------------------------------------------ Gen.ParRep on the GPU
def test_forced_reference_exit_and_clock_gpu():
    gpr = _gpr()
    g = gpr.System(G.toy2d(), path=gpr.PATH_PERSISTENT)
    rc, ev = g.decorrelate(0)
    assert rc == 0 and ev["kind"] == 0
    q, v = g.get_state(0)
    q[0, 0] = 1.5
    g.set_state(0, q, v)
    t0 = g.simulated_steps()
    rc, o = g.dephase()
    assert rc == 0 and o["outcome"] == 1 and o["to_state"] == 1 and o["t_steps"] == 10
    assert g.simulated_steps() - t0 == 10
    with pytest.raises(gpr.GprError):
        g.parallel_step()


def _clone_groups(q):
    """Partition of the workers into groups of bit-identical configurations."""
    groups = {}
    for r in range(1, len(q)):
        groups.setdefault(q[r].tobytes(), []).append(r)
    return sorted(tuple(g) for g in groups.values())


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("seed", [5, 11])
def test_dephase_branching_matches_oracle(path, seed):
    """One dephasing check with many exits (all walkers start near the barrier top, x = -0.05):
    the GPU's Fleming-Viot plan and clone copies give the same partition of the workers into
    bit-identical copies as the oracle's, every worker is back in Omega, and the positions
    agree with the oracle's."""
    gpr = _gpr()
    spec = G.round_to_f32(dict(G.toy2d(n_replicas=64, seed=seed), pos=np.array([[-0.05], [0.0], [0.0]])))
    g = gpr.System(spec, path=path)
    o = oracle.System(spec)
    for sys_ in (g, o):
        rc, ev = sys_.decorrelate(0)
        assert rc == 0 and ev["to_state"] == 0
        rc, _ = sys_.dephase(10)
        assert rc == 1                                  # budget: one check done, not converged
    qg = np.stack([g.get_state(r)[0][:, 0] for r in range(64)])
    qo = np.stack([o.get_state(r)[0][:, 0] for r in range(64)])
    assert np.abs(qg - qo).max() < 1e-5
    cg, co = _clone_groups(qg), _clone_groups(qo)
    assert cg == co
    assert any(len(c) > 1 for c in cg)                  # branching happened
    assert np.all(g.observe()[1] == 0)
    ng, S1g, _, _ = g.accumulators()
    no, S1o, _, _ = o.accumulators()
    assert ng == no == 10
    assert np.allclose(S1g, S1o, rtol=1e-5, atol=1e-6)


@pytest.mark.slow
def test_toy_gen_parrep_gpu_matches_direct_simulation():
    from helpers import direct_exits, gen_parrep_exits
    gpr = _gpr()
    n = 500
    say("toy Gen.ParRep on GPU")
    g = gen_parrep_exits(gpr.System(G.toy2d(seed=303), path=gpr.PATH_PERSISTENT), n, t_corr=100)
    d = direct_exits(oracle.System(G.toy2d(seed=101)), n)
    gg = np.array([x[0] for x in g], float)
    dd = np.array([x[0] for x in d], float)
    p = stats.ks_2samp(gg, dd).pvalue
    say("KS p", p, "means", gg.mean(), dd.mean())
    assert p > 0.05
