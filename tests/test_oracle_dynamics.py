"""Pins of the oracle's Langevin integrator (Eq. 1 discretised by BAOAB).

Closed forms of the BAOAB scheme on a harmonic well (Leimkuhler and Matthews, Appl. Math.
Res. Express 2013): the position variance is exactly kT/k at any stable dt and any
friction, and the end-of-step kinetic energy is (3/2) kT (1 - (omega dt)^2 / 4).  With zero
friction the scheme is velocity Verlet: energy is conserved without drift and the
trajectory is reversible under a momentum flip."""
import math

import numpy as np
import pytest

import gpr_synth as G
import oracle
from helpers import mini


def _pooled_moments(sys, j):
    n, S1, S2, c = sys.accumulators()
    S1, S2 = S1[1:, j], S2[1:, j]
    mean = S1.sum() / (n * len(S1))
    m2 = S2.sum() / (n * len(S2))
    return mean + c[j], m2 - mean * mean


def test_baoab_harmonic_variances_large_dt():
    kT, k, m, dt = 2.494, 1000.0, 12.0, 0.1
    omega = math.sqrt(k / m)
    assert omega * dt < 2
    spec = mini([[0.0, 0.0, 0.0]], mass=[m], epsilon=0.0, R=8, kT=kT, gamma=5.0, dt=dt,
                restraints=np.array([0], np.int32), restraint_ref=np.zeros((1, 3)),
                restraint_k=np.array([k]), vel=None,
                obs=[dict(kind=G.OBS_COORD, atoms=[0, 0]), dict(kind=G.OBS_COORD, atoms=[0, 1]),
                     dict(kind=G.OBS_COORD, atoms=[0, 2]), dict(kind=G.OBS_KINETIC)])
    s = oracle.System(spec)
    s.advance(2000)          # equilibrate
    s.dephase(0)             # clears accumulators (dephasing starts; budget 0 steps)
    s.advance(200000)
    for j in range(3):
        mean, var = _pooled_moments(s, j)
        assert abs(mean) < 0.01 * math.sqrt(kT / k) * 10
        assert var == pytest.approx(kT / k, rel=0.02)
    meanK, _ = _pooled_moments(s, 3)
    expect = 1.5 * kT * (1 - (omega * dt) ** 2 / 4)
    assert meanK == pytest.approx(expect, rel=0.02)
    # the splitting is identified: 1.5 kT itself is excluded at this dt
    assert abs(meanK - 1.5 * kT) > 5 * 0.02 * expect


def test_toy_y_variance_is_kT_over_4():
    s = oracle.System(G.toy2d(n_replicas=8, seed=11))
    s.advance(1000)
    s.dephase(0)
    s.advance(200000)
    _, var = _pooled_moments(s, 1)
    assert var == pytest.approx(0.2 / 4.0, rel=0.03)


def _nve_chain():
    spec = G.chain(n_replicas=2, gamma=0.0)
    spec["obs"] = [dict(kind=G.OBS_POTENTIAL), dict(kind=G.OBS_KINETIC)]
    return spec


def test_zero_friction_conserves_energy():
    s = oracle.System(_nve_chain())
    E, K = [], []
    for _ in range(200):
        s.advance(50)
        obs, _ = s.observe()
        E.append(obs[0, 0] + obs[0, 1])
        K.append(obs[0, 1])
    E = np.array(E)
    t = np.arange(len(E))
    slope = np.polyfit(t, E, 1)[0]
    assert E.std() < 0.05 * np.std(K)              # total energy fluctuates far less than K
    assert abs(slope * len(E)) < 3 * E.std() + 1e-6   # no drift beyond the fluctuation


def test_zero_friction_reversible():
    s = oracle.System(_nve_chain())
    q0, v0 = s.get_state(0)
    s.advance(300)
    q1, v1 = s.get_state(0)
    assert np.abs(q1 - q0).max() > 1e-3
    s.set_state(0, q1, -v1)
    s.advance(300)
    q2, v2 = s.get_state(0)
    assert np.abs(q2 - q0).max() < 1e-9
    assert np.abs(v2 + v0).max() < 1e-7


def test_replicas_get_independent_noise_and_identical_start():
    s = oracle.System(G.chain(n_replicas=3))
    q0, _ = s.get_state(0)
    for r in (1, 2):
        assert np.array_equal(s.get_state(r)[0], q0)
    s.advance(20)
    a, b = s.get_state(1)[0], s.get_state(2)[0]
    assert np.abs(a - b).max() > 1e-6
    assert s.global_step() == 20


def test_maxwell_boltzmann_initial_velocities():
    spec = G.receptor_ligand(n_receptor=268, radius=2.2, n_replicas=2)
    s = oracle.System(spec)
    _, v = s.get_state(0)
    m = spec["mass"]
    z = v * np.sqrt(m / spec["kT"])
    assert abs(z.mean()) < 0.1 and z.var() == pytest.approx(1.0, rel=0.1)
