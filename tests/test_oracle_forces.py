"""Pins of the oracle's force field (the engine requirement of Sec. 3.2: V(q) and its
gradient).  Closed forms on two- to four-atom inputs fix every energy term, central finite
differences of the oracle's own energy fix every force, and translation invariance fixes
the action-reaction pairing."""
import math

import numpy as np
import pytest

import gpr_synth as G
import oracle
from helpers import chain_terms, mini

F_COUL = 138.935458


def U_of(spec, pos=None):
    s = oracle.System(spec)
    q = spec["pos"] if pos is None else np.asarray(pos, np.float64).T
    return s.eval(q)


def test_lj_minimum_lorentz_berthelot():
    si, sj, ei, ej = 0.26, 0.34, 0.2, 0.8
    sij = 0.5 * (si + sj)
    r = 2 ** (1 / 6) * sij
    spec = mini([[0, 0, 0], [r, 0, 0]], sigma=[si, sj], epsilon=[ei, ej])
    U, F = U_of(spec)
    assert U == pytest.approx(-math.sqrt(ei * ej), rel=1e-12)
    assert np.abs(F).max() < 1e-9
    # at r = sigma_ij the LJ energy is exactly zero
    U0, _ = U_of(spec, [[0, 0, 0], [sij, 0, 0]])
    assert abs(U0) < 1e-12


def test_vacuum_coulomb():
    spec = mini([[0, 0, 0], [0, 0.7, 0]], epsilon=0.0, charge=[0.5, -0.3])
    U, F = U_of(spec)
    assert U == pytest.approx(F_COUL * 0.5 * -0.3 / 0.7, rel=1e-12)
    # attraction: atom 0 pulled toward +y with |F| = f |q q| / r^2
    assert F[1, 0] == pytest.approx(F_COUL * 0.15 / 0.49, rel=1e-12)
    assert F[1, 1] == pytest.approx(-F[1, 0], rel=1e-15)


def test_reaction_field_closed_form_and_cutoff():
    rc, erf = 1.0, 78.5
    krf = (erf - 1) / ((2 * erf + 1) * rc ** 3)
    crf = 1 / rc + krf * rc ** 2
    qi, qj = 0.4, 0.6
    for r in (0.35, 0.8):
        spec = mini([[0, 0, 0], [0, 0, r]], epsilon=0.0, charge=[qi, qj], cutoff=rc, eps_rf=erf)
        U, _ = U_of(spec)
        assert U == pytest.approx(F_COUL * qi * qj * (1 / r + krf * r * r - crf), rel=1e-12)
    # E(r_c) = 0: the energy vanishes continuously at the cutoff, and is zero beyond it
    spec = mini([[0, 0, 0], [0, 0, rc - 1e-7]], epsilon=0.0, charge=[qi, qj], cutoff=rc, eps_rf=erf)
    assert abs(U_of(spec)[0]) < 1e-4
    spec = mini([[0, 0, 0], [0, 0, rc + 1e-9]], epsilon=0.5, charge=[qi, qj], cutoff=rc, eps_rf=erf)
    U, F = U_of(spec)
    assert U == 0.0 and np.all(F == 0.0)


def test_bond_angle_torsion_restraint_closed_forms():
    t = chain_terms(4)
    # right-angle, planar trans chain: bond lengths 0.1, angles pi/2, dihedral pi
    pos = [[0, 0.1, 0], [0, 0, 0], [0.1, 0, 0], [0.1, -0.1, 0]]
    base = dict(epsilon=0.0, charge=0.0)
    s = mini(pos, bonds=t["bonds"][:1], bond_r0=np.array([0.12]), bond_k=np.array([2e5]), **base)
    assert U_of(s)[0] == pytest.approx(0.5 * 2e5 * 0.02 ** 2, rel=1e-12)
    s = mini(pos, angles=t["angles"][:1], angle_theta0=np.array([1.91]), angle_k=np.array([400.0]), **base)
    assert U_of(s)[0] == pytest.approx(0.5 * 400 * (math.pi / 2 - 1.91) ** 2, rel=1e-12)
    for n, k, p0, expect in ((3, 5.0, 0.0, 0.0), (1, 5.0, 0.0, 0.0), (2, 5.0, 0.0, 10.0),
                             (1, 2.0, math.pi / 3, 2.0 * (1 + math.cos(math.pi - math.pi / 3)))):
        s = mini(pos, torsions=t["torsions"], torsion_n=np.array([n], np.int32),
                 torsion_k=np.array([k]), torsion_phi0=np.array([p0]), **base)
        assert U_of(s)[0] == pytest.approx(expect, abs=1e-12)
    # cis: dihedral 0 -> k (1 + cos(0)) = 2k for n = 3
    cis = [[0, 0.1, 0], [0, 0, 0], [0.1, 0, 0], [0.1, 0.1, 0]]
    s = mini(cis, torsions=t["torsions"], torsion_n=np.array([3], np.int32),
             torsion_k=np.array([5.0]), torsion_phi0=np.array([0.0]), **base)
    assert U_of(s)[0] == pytest.approx(10.0, rel=1e-12)
    s = mini(pos, restraints=np.array([2], np.int32), restraint_ref=np.array([[0.1, 0.03, -0.04]]),
             restraint_k=np.array([1000.0]), **base)
    U, F = U_of(s)
    assert U == pytest.approx(0.5 * 1000 * (0.03 ** 2 + 0.04 ** 2), rel=1e-12)
    assert F[:, 2] == pytest.approx([0.0, 30.0, -40.0], rel=1e-12)


def test_dihedral_sign_iupac():
    """IUPAC convention (Rules for the Nomenclature of Organic Chemistry, Section E,
    1974): the torsion angle is positive when, looking from j along j->k, the bond j-i
    must be rotated clockwise by less than 180 degrees to eclipse the bond k-l.  With j at
    the origin, k on +z and i on +x, the viewer looks along +z and sees x->y as a
    clockwise turn, so l = k + (cos a, sin a, 0) has torsion +a."""
    for a in (math.radians(60), math.radians(-100), math.radians(170)):
        pos = [[1, 0, 0], [0, 0, 0], [0, 0, 1], [math.cos(a), math.sin(a), 1]]
        spec = mini(pos, epsilon=0.0, obs=[dict(kind=G.OBS_DIHEDRAL, atoms=[0, 1, 2, 3])])
        s = oracle.System(spec)
        o = s.observables_of(spec["pos"], np.zeros((3, 4)), 0.0)
        assert o[0] == pytest.approx(a, abs=1e-12)


def test_exclusions_and_14_scaling():
    t = chain_terms(4)
    pos = [[0, 0, 0], [0.3, 0, 0], [0.6, 0.1, 0], [0.9, 0.3, 0.2]]
    q = [0.3, -0.2, 0.1, -0.4]
    sig, eps = [0.3, 0.32, 0.28, 0.31], [0.4, 0.5, 0.6, 0.7]
    excl = np.concatenate([t["bonds"], t["angles"][:, [0, 2]]])
    s = mini(pos, sigma=sig, epsilon=eps, charge=q, exclusions=excl,
             pairs14=np.array([[0, 3]], np.int32), scale14=0.5)
    U, _ = U_of(s)
    r = math.dist(pos[0], pos[3])
    sij, eij = 0.5 * (sig[0] + sig[3]), math.sqrt(eps[0] * eps[3])
    lj = 4 * eij * ((sij / r) ** 12 - (sij / r) ** 6)
    assert U == pytest.approx(0.5 * (lj + F_COUL * q[0] * q[3] / r), rel=1e-12)
    # with nothing excluded, six pairs contribute
    s_all = mini(pos, sigma=sig, epsilon=eps, charge=q)
    Ua, _ = U_of(s_all)
    tot = 0.0
    for i in range(4):
        for j in range(i + 1, 4):
            r = math.dist(pos[i], pos[j])
            sij, eij = 0.5 * (sig[i] + sig[j]), math.sqrt(eps[i] * eps[j])
            tot += 4 * eij * ((sij / r) ** 12 - (sij / r) ** 6) + F_COUL * q[i] * q[j] / r
    assert Ua == pytest.approx(tot, rel=1e-12)


def _fd_check(spec, atoms, h=1e-6, rel=2e-6):
    s = oracle.System(spec)
    q0 = np.array(spec["pos"], np.float64)
    U0, F = s.eval(q0)
    scale = np.abs(F).max()
    for i in atoms:
        for d in range(3):
            qp = q0.copy(); qp[d, i] += h
            qm = q0.copy(); qm[d, i] -= h
            g = (s.eval(qp)[0] - s.eval(qm)[0]) / (2 * h)
            assert -g == pytest.approx(F[d, i], abs=rel * scale), (i, d)
    return F


def test_forces_are_minus_gradient_chain22():
    spec = G.chain()
    F = _fd_check(spec, range(spec["n_atoms"]))
    # no restraints: translation invariance gives a zero net force
    assert np.abs(F.sum(1)).max() < 1e-9 * np.abs(F).max()


def test_forces_are_minus_gradient_receptor_ligand():
    spec = G.config("rl300", n_replicas=2)
    rng = np.random.default_rng(0)
    atoms = list(rng.choice(spec["n_atoms"], 12, replace=False)) + [spec["n_atoms"] - 1]
    _fd_check(spec, atoms)


def test_net_force_zero_with_cutoff_no_restraints():
    spec = G.config("rl300", n_replicas=2)
    spec["restraints"] = np.zeros((0,), np.int32)
    spec["restraint_ref"] = np.zeros((0, 3))
    spec["restraint_k"] = np.zeros((0,))
    U, F = U_of(spec)
    assert np.abs(F.sum(1)).max() < 1e-9 * np.abs(F).max()


def test_toy_potential_closed_form():
    s = oracle.System(G.toy2d())
    for x, y in ((-1.0, 0.0), (0.0, 0.0), (0.5, -0.3)):
        U, F = s.eval(np.array([[x], [y], [0.0]]))
        assert U == pytest.approx((x * x - 1) ** 2 + 2 * y * y, abs=1e-15)
        assert F[:, 0] == pytest.approx([-4 * x * (x * x - 1), -4 * y, 0.0], abs=1e-15)
