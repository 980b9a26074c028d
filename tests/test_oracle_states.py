"""Pins of the oracle's state functions and observables (Sec. 2.2 states, Sec. 2.4.1
observables of Eq. 2; the state definitions of the two applications, Sec. 4.1.2 and Sec.
4.2.2) on hand-built geometries whose answers are worked out by hand, so that a plausible
slip (an unweighted centre of mass, <= instead of < at a radius, [lo, hi) instead of
(lo, hi] box edges, a root of a sum instead of a mean) fails one of them; and of transient
propagation through configurations that belong to no state (Sec. 2.2: the states need not
cover the whole space; Sec. 2.4 transient step)."""
import math

import numpy as np
import pytest

import gpr_synth as G
import oracle
from helpers import mini


def _soa(pos):
    return np.asarray(pos, np.float64).T.copy()


# ------------------------------------------------------------------ centre of mass in a sphere
def _com_state(pos, mass, group, center, radius):
    spec = mini(pos, mass=mass, epsilon=0.0,
                state=dict(kind=G.STATE_COM_SPHERE, group=np.asarray(group, np.int32), center=center, radius=radius))
    return oracle.System(spec), spec


def test_com_sphere_state_is_mass_weighted():
    # masses 1 and 3 at x = 0 and x = 4/3: centre of mass at x = 1 (unweighted mean 2/3);
    # atom 2 (mass 16, far away) is not in the group and must not count
    pos = [[0.0, 0.0, 0.0], [4.0 / 3.0, 0.0, 0.0], [9.0, 9.0, 9.0]]
    s, spec = _com_state(pos, [1.0, 3.0, 16.0], [0, 1], [1.0, 0.0, 0.0], 0.05)
    assert s.state_of(spec["pos"]) == 1
    s, spec = _com_state(pos, [1.0, 3.0, 16.0], [0, 1], [2.0 / 3.0, 0.0, 0.0], 0.05)
    assert s.state_of(spec["pos"]) == 0


def test_com_sphere_boundary_is_outside():
    # two atoms of mass 12 at x = 0.25 and 0.75: centre (0.5, 0, 0), exactly representable;
    # sphere of radius 0.5 about the origin: |c - p| = radius is outside (strict <)
    pos = [[0.25, 0.0, 0.0], [0.75, 0.0, 0.0]]
    s, spec = _com_state(pos, [12.0, 12.0], [0, 1], [0.0, 0.0, 0.0], 0.5)
    assert s.state_of(spec["pos"]) == 0
    s, spec = _com_state(pos, [12.0, 12.0], [0, 1], [0.0, 0.0, 0.0], 0.5 + 2.0 ** -40)
    assert s.state_of(spec["pos"]) == 1
    # the distance is Euclidean in three dimensions: centre (0.3, 0.4, 0) is 0.5 from the origin
    pos = [[0.3, 0.4, 0.0], [0.3, 0.4, 0.0]]
    s, spec = _com_state(pos, [12.0, 12.0], [0, 1], [0.0, 0.0, 0.0], 0.5 + 1e-9)
    assert s.state_of(spec["pos"]) == 1
    s, spec = _com_state(pos, [12.0, 12.0], [0, 1], [0.0, 0.0, 0.0], 0.5 - 1e-9)
    assert s.state_of(spec["pos"]) == 0


# ------------------------------------------------------------------ dihedral boxes
def _two_dihedrals(phi, psi):
    """Eight atoms: (0,1,2,3) with torsion phi, (4,5,6,7) with torsion psi, each built as
    j at the origin, k on +z, i on +x and l = k + (cos a, sin a, 0), whose IUPAC torsion is
    +a (the sign convention pinned in the force tests)."""
    def four(a, off):
        o = np.array([off, 0.0, 0.0])
        return [o + [1, 0, 0], o + [0, 0, 0], o + [0, 0, 1], o + [math.cos(a), math.sin(a), 1]]
    return four(phi, 0.0) + four(psi, 10.0)


def _box_system(phi, psi, boxes):
    pos = _two_dihedrals(phi, psi)
    spec = mini(pos, epsilon=0.0,
                state=dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=list(range(8)), boxes=boxes),
                obs=[dict(kind=G.OBS_DIHEDRAL, atoms=[0, 1, 2, 3]), dict(kind=G.OBS_DIHEDRAL, atoms=[4, 5, 6, 7])])
    s = oracle.System(spec)
    vals = s.observables_of(spec["pos"], np.zeros((3, 8)), 0.0)
    return s, spec, vals


def test_dihedral_boxes_use_both_dihedrals_in_order():
    phi, psi = math.radians(-100.0), math.radians(40.0)
    boxes = [[-4, 0, -4, 0], [-4, 0, 0, 4], [0, 4, -4, 0], [0, 4, 0, 4]]
    s, spec, (p, q) = _box_system(phi, psi, boxes)
    assert p == pytest.approx(phi, abs=1e-12) and q == pytest.approx(psi, abs=1e-12)
    assert s.state_of(spec["pos"]) == 1                 # phi < 0, psi > 0
    s, spec, _ = _box_system(psi, phi, boxes)
    assert s.state_of(spec["pos"]) == 2                 # swapped: phi > 0, psi < 0


def test_dihedral_box_edges_are_lower_open_upper_closed():
    s, spec, (p, q) = _box_system(math.radians(75.0), math.radians(-20.0), [[0, 1, 0, 1]])
    # the same configuration against boxes whose edges sit exactly on the computed angles
    def state(boxes):
        t = oracle.System(dict(spec, state=dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=list(range(8)), boxes=boxes)))
        return t.state_of(spec["pos"])
    assert state([[p - 1, p, q - 1, q]]) == 0            # phi = hi and psi = hi: inside
    assert state([[p, p + 1, q - 1, q]]) == -1           # phi = lo: outside
    assert state([[p - 1, p, q, q + 1]]) == -1           # psi = lo: outside
    # the lower box claims the shared edge
    assert state([[p - 1, p, q - 1, q + 1], [p, p + 1, q - 1, q + 1]]) == 0
    assert state([[p, p + 1, q - 1, q + 1], [p - 1, p, q - 1, q + 1]]) == 1


def test_dihedral_boxes_first_match_and_no_state():
    s, spec, (p, q) = _box_system(math.radians(30.0), math.radians(30.0), [[0, 1, 0, 1]])

    def state(boxes):
        t = oracle.System(dict(spec, state=dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=list(range(8)), boxes=boxes)))
        return t.state_of(spec["pos"])
    big, small = [-4, 4, -4, 4], [0, 1, 0, 1]
    assert state([big, small]) == 0 and state([small, big]) == 0      # overlapping: first listed wins
    assert state([[-4, 0, -4, 4], [1, 4, -4, 4], small]) == 2
    assert state([[-4, 0, -4, 4], [1, 4, -4, 4]]) == -1                  # in the gap: no state


# ------------------------------------------------------------------ observables
def test_com_distance_observable_is_mass_weighted():
    # group a = atoms 0, 1 (masses 1, 3 at x = 0, 4): centre (3, 0, 0); group b = atom 2 at
    # (3, 4, 0): distance 4 (an unweighted centre (2, 0, 0) would give sqrt(17))
    pos = [[0.0, 0.0, 0.0], [4.0, 0.0, 0.0], [3.0, 4.0, 0.0], [7.0, 7.0, 7.0]]
    obs = [dict(kind=G.OBS_COM_DISTANCE, group_a=np.array([0, 1], np.int32), group_b=np.array([2], np.int32)),
           dict(kind=G.OBS_COM_DISTANCE, group_a=np.array([2], np.int32), group_b=np.array([0, 1, 3], np.int32))]
    spec = mini(pos, mass=[1.0, 3.0, 5.0, 4.0], epsilon=0.0, obs=obs)
    s = oracle.System(spec)
    o = s.observables_of(spec["pos"], np.zeros((3, 4)), 0.0)
    assert o[0] == pytest.approx(4.0, rel=1e-14)
    # second: centre of {0, 1, 3} = (1*0 + 3*4 + 4*7, 4*7, 4*7) / 8 = (5, 3.5, 3.5)
    assert o[1] == pytest.approx(math.sqrt(2.0 ** 2 + 0.5 ** 2 + 3.5 ** 2), rel=1e-14)


def test_rms_velocity_and_kinetic_energy_observables():
    pos = [[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [2.0, 0.0, 0.0], [3.0, 0.0, 0.0]]
    vel = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 0.0], [1.0, 2.0, 2.0], [5.0, 5.0, 5.0]]).T.copy()
    obs = [dict(kind=G.OBS_RMS_VELOCITY, group_a=np.array([0, 1, 2], np.int32)), dict(kind=G.OBS_KINETIC),
           dict(kind=G.OBS_POTENTIAL), dict(kind=G.OBS_COORD, atoms=[2, 1])]
    spec = mini(pos, mass=[2.0, 7.0, 4.0, 1.0], epsilon=0.0, obs=obs)
    s = oracle.System(spec)
    o = s.observables_of(spec["pos"], vel, -12.5)
    # |v|^2 = 25, 0, 9 over the group of three: root of the mean, not of the sum, and
    # independent of the masses
    assert o[0] == pytest.approx(math.sqrt(34.0 / 3.0), rel=1e-14)
    # K = 1/2 (2*25 + 7*0 + 4*9 + 1*75) over every atom
    assert o[1] == pytest.approx(0.5 * (50.0 + 36.0 + 75.0), rel=1e-14)
    assert o[2] == -12.5
    assert o[3] == 0.0                                   # y of atom 2


# ------------------------------------------------------------------ states that do not cover the space
def _butane(phi0, seed, boxes, R=2, t_check=10):
    """Four atoms of mass 12 with 0.15 nm bonds, right angles and one torsion (n = 3 minima
    at +-60 and 180 degrees, barrier 2k = 4 kJ/mol, about 1.6 kT at 300 K); the state is a
    box in that dihedral, so configurations between the boxes belong to no state."""
    pos = 0.15 * np.asarray(_two_dihedrals(phi0, phi0)[:4])
    s = mini(pos, mass=[12.0, 12.0, 12.0, 12.0], epsilon=0.0, R=R, seed=seed, kT=G.KB * 300.0,
             bonds=np.array([[0, 1], [1, 2], [2, 3]], np.int32), bond_r0=np.full(3, 0.15),
             bond_k=np.full(3, 2.0e5),
             angles=np.array([[0, 1, 2], [1, 2, 3]], np.int32), angle_theta0=np.full(2, math.pi / 2),
             angle_k=np.full(2, 400.0),
             torsions=np.array([[0, 1, 2, 3]], np.int32), torsion_n=np.array([3], np.int32),
             torsion_k=np.array([2.0]), torsion_phi0=np.array([0.0]),
             t_check_dephase=t_check, t_check_parallel=t_check,
             state=dict(kind=G.STATE_DIHEDRAL_BOXES, atoms=[0, 1, 2, 3, 0, 1, 2, 3], boxes=boxes))
    s["vel"] = None
    return s


# two boxes around the gauche minima; the trans region and the eclipsed ones are no state
GAPPED = [[math.radians(-100), math.radians(-20), -4, 4], [math.radians(20), math.radians(100), -4, 4]]


def _replay_transient(spec, t_corr, max_checks=200000):
    """Brute force of the transient step on a fresh copy of the system: step replica 0 one
    check period at a time (the noise of replica 0 depends only on the global step, so the
    trajectory is the one the oracle's transient step follows) and apply the rules of the
    step directly: a state is entered at the first check that finds one; the walker is
    resident once t_corr steps have passed at later checks in that state; leaving it at a
    check (into another state or into none) is an exit."""
    s = oracle.System(spec)
    tc = spec["t_check_dephase"]
    cur = s.state_of(s.get_state(0)[0])
    start = cur
    resid = 0
    for m in range(1, max_checks + 1):
        if cur != -1 and resid >= t_corr:
            return dict(kind=0, from_state=start, to_state=cur, resident_steps=resid, steps_taken=(m - 1) * tc)
        s.step_replicas(tc, 0, 1)
        st = s.state_of(s.get_state(0)[0])
        if st == cur:
            resid += tc
        elif cur == -1:
            cur, resid = st, 0
        else:
            return dict(kind=1, from_state=cur, to_state=st, resident_steps=resid + tc, steps_taken=m * tc)
    raise AssertionError("no event")


def test_transient_step_through_no_state():
    """Starting between the boxes (trans, phi = 180 degrees) the walker spends the time it
    needs to reach a box in no state, and that time is on the clock (the reaching time of the
    transient step); from a box it may leave into no state, which is an exit with to_state
    -1, after which the next transient step starts again in no state.  Every first event
    equals a brute-force replay of the rules, and both kinds of event occur over the seeds."""
    t_corr = 300
    reach, to_none = 0, 0
    for seed in range(11, 19):
        spec = _butane(math.pi, seed, GAPPED)
        s = oracle.System(spec)
        assert s.state_of(spec["pos"]) == -1
        rc, ev = s.decorrelate(t_corr)
        assert rc == 0 and s.simulated_steps() == ev["steps_taken"]
        ref = _replay_transient(spec, t_corr)
        assert ev == ref, (seed, ev, ref)
        if ev["kind"] == 0:
            reach += ev["from_state"] == -1 and ev["to_state"] in (0, 1)
            continue
        # entered a box, then left it before t_corr: into the other box or into no state
        assert ev["from_state"] in (0, 1) and ev["to_state"] != ev["from_state"]
        to_none += ev["to_state"] == -1
        if ev["to_state"] == -1:
            t0 = s.simulated_steps()
            rc, ev2 = s.decorrelate(t_corr)
            assert rc == 0 and s.simulated_steps() - t0 == ev2["steps_taken"]
            assert ev2["kind"] == 1 or ev2["from_state"] == -1
    assert reach >= 1 and to_none >= 1, (reach, to_none)


def test_transient_reaching_time_counts_and_dephasing_refuses_no_state():
    spec = _butane(math.pi, 5, GAPPED)
    s = oracle.System(spec)
    rc, ev = s.decorrelate(10 ** 9, max_steps=10)   # one check, still budgeted
    assert rc == oracle.BUDGET and s.simulated_steps() == 10
    # the reference walker in no state cannot start a convergence step
    t = oracle.System(spec)
    with pytest.raises(oracle.OracleError):
        t.dephase()
