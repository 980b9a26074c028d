"""Pins of the oracle's force-field parameter gradient dU/d(eps_i, sigma_i, q_i, torsion k_t):
closed forms on two- and four-atom systems, and central finite differences of the oracle's own
energy (itself pinned by closed forms) with respect to every sampled parameter, in vacuum with
all pairs and with the reaction-field cutoff."""
import math

import numpy as np
import pytest

import gpr_synth as G
import oracle
from helpers import chain_terms, mini

F_COUL = 138.935458


def test_two_atom_closed_forms():
    si, sj, ei, ej, qi, qj, r = 0.28, 0.33, 0.3, 0.7, 0.4, -0.25, 0.37
    spec = mini([[0, 0, 0], [0, r, 0]], sigma=[si, sj], epsilon=[ei, ej], charge=[qi, qj])
    g = oracle.System(spec).param_grad(spec["pos"])
    sij, eij = 0.5 * (si + sj), math.sqrt(ei * ej)
    s6 = (sij / r) ** 6
    ulj = 4 * eij * (s6 * s6 - s6)
    # eps enters through sqrt(eps_i eps_j): d/d eps_i = U_LJ / (2 eps_i)
    assert g["epsilon"] == pytest.approx([ulj / (2 * ei), ulj / (2 * ej)], rel=1e-12)
    # sigma enters through (sigma_i + sigma_j)/2: the same derivative for both atoms
    dsig = 0.5 * 4 * eij * (12 * s6 * s6 - 6 * s6) / sij
    assert g["sigma"] == pytest.approx([dsig, dsig], rel=1e-12)
    # vacuum Coulomb f q_i q_j / r
    assert g["charge"] == pytest.approx([F_COUL * qj / r, F_COUL * qi / r], rel=1e-12)


def test_lj_minimum_has_zero_sigma_gradient():
    """At r = 2^(1/6) sigma_ij the LJ energy is minimal in r, and U depends on sigma_ij only
    through sigma_ij / r: dU/dsigma_ij = -(r / sigma_ij) dU/dr = 0."""
    si, sj = 0.26, 0.34
    r = 2 ** (1 / 6) * 0.5 * (si + sj)
    spec = mini([[0, 0, 0], [r, 0, 0]], sigma=[si, sj], epsilon=[0.2, 0.8])
    g = oracle.System(spec).param_grad(spec["pos"])
    assert np.abs(g["sigma"]).max() < 1e-9


def test_torsion_constant_gradient_closed_form():
    t = chain_terms(4)
    cis = [[0, 0.1, 0], [0, 0, 0], [0.1, 0, 0], [0.1, 0.1, 0]]        # phi = 0
    trans = [[0, 0.1, 0], [0, 0, 0], [0.1, 0, 0], [0.1, -0.1, 0]]     # phi = pi
    for pos, phi in ((cis, 0.0), (trans, math.pi)):
        for n, p0 in ((3, 0.0), (1, math.pi / 3), (2, 0.5)):
            spec = mini(pos, epsilon=0.0, torsions=t["torsions"], torsion_n=np.array([n], np.int32),
                        torsion_k=np.array([4.0]), torsion_phi0=np.array([p0]))
            g = oracle.System(spec).param_grad(spec["pos"])
            assert g["torsion_k"][0] == pytest.approx(1 + math.cos(n * phi - p0), abs=1e-12)


def _perturbed_energy(spec, q, key, idx, delta):
    s = dict(spec)
    s[key] = np.array(spec[key], np.float64).copy()
    s[key][idx] += delta
    return oracle.System(s).eval(q)[0]


def _fd_check(spec, q, atoms, torsions, rel=1e-6):
    g = oracle.System(spec).param_grad(q)
    for key, name in (("epsilon", "epsilon"), ("sigma", "sigma"), ("charge", "charge")):
        scale = np.abs(g[name]).max()
        for i in atoms:
            h = 1e-6 * max(abs(spec[key][i]), 1e-2)
            fd = (_perturbed_energy(spec, q, key, i, h) - _perturbed_energy(spec, q, key, i, -h)) / (2 * h)
            assert g[name][i] == pytest.approx(fd, abs=rel * scale), (name, i)
    scale = max(np.abs(g["torsion_k"]).max(), 1e-3)
    for t in torsions:
        h = 1e-6 * abs(spec["torsion_k"][t])
        fd = (_perturbed_energy(spec, q, "torsion_k", t, h) -
              _perturbed_energy(spec, q, "torsion_k", t, -h)) / (2 * h)
        assert g["torsion_k"][t] == pytest.approx(fd, abs=rel * scale), ("torsion", t)
    return g


def _moved(spec, steps=200):
    """Positions after some Langevin steps (off the generated geometry: no torsion at pi)."""
    o = oracle.System(dict(spec, n_replicas=2))
    o.step_replicas(steps, 0, 1)
    return o.get_state(0)[0]


def test_gradient_matches_finite_differences_vacuum_chain():
    spec = G.config("chain22", n_replicas=2)
    q = _moved(spec)
    g = _fd_check(spec, q, range(spec["n_atoms"]), range(len(spec["torsion_k"])))
    assert np.abs(g["torsion_k"]).max() > 0.1


def test_gradient_matches_finite_differences_reaction_field():
    spec = G.config("rl300", n_replicas=2)
    q = _moved(spec, steps=50)
    rng = np.random.default_rng(1)
    atoms = sorted(rng.choice(spec["n_atoms"], 10, replace=False)) + [spec["n_atoms"] - 1]
    torsions = sorted(rng.choice(len(spec["torsion_k"]), 6, replace=False))
    _fd_check(spec, q, atoms, torsions)
