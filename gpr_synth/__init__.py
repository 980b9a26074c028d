"""Seeded synthetic inputs for the Gen.ParRep hot path.

The paper's workloads (alanine dipeptide with CHARMM22, the FKBP-DMSO complex with
ff14SB/GAFF in implicit solvent; arXiv 1807.02431 Sec. 4.1-4.2) need force-field files and
structures that are not available here, so systems of the same scale and character are
generated from a seed:

* ``toy2d``: one particle in the double well U(x, y) = (x^2-1)^2 + 2 y^2 (state = sign x);
* ``chain``: a 22-atom chain the size of alanine dipeptide, vacuum, all pairs, whose two
  central dihedrals (phi, psi) carry extra terms giving four basins; state = (phi, psi)
  quadrant (the role of the C7eq/C7ax Ramachandran states of Sec. 4.1.2);
* ``receptor_ligand``: a restrained receptor chain folded into a sphere with a pocket and
  a free ligand chain in it, reaction-field electrostatics with a cutoff, state = "ligand
  centre of mass within 0.4 nm of the pocket centre" (the role of the bound state of
  Sec. 4.2.2).

Each generator returns a plain dict of numpy arrays and scalars (the system descriptor).
This module builds inputs only: geometry by internal coordinates, random parameters,
topology lists.  It evaluates no energy, force, dynamics, state or statistic.
"""
from __future__ import annotations

import functools
import math

import numpy as np

KB = 0.0083144626  # kJ/mol/K
TOY2D = 1
MOLECULAR = 2
STATE_SIGN_X = 1
STATE_DIHEDRAL_BOXES = 2
STATE_COM_SPHERE = 3
OBS_COORD = 1
OBS_POTENTIAL = 2
OBS_KINETIC = 3
OBS_DIHEDRAL = 4
OBS_COM_DISTANCE = 5
OBS_RMS_VELOCITY = 6

_EMPTY_I = np.zeros((0,), dtype=np.int32)
_EMPTY_D = np.zeros((0,), dtype=np.float64)


def _base(kind, n, R):
    return dict(
        kind=kind, n_atoms=n, n_replicas=R, mass=None, pos=None, vel=None,
        sigma=None, epsilon=None, charge=None,
        cutoff=0.0, eps_rf=1.0, skin=0.0, nlist_period=1,
        bonds=np.zeros((0, 2), np.int32), bond_r0=_EMPTY_D, bond_k=_EMPTY_D,
        angles=np.zeros((0, 3), np.int32), angle_theta0=_EMPTY_D, angle_k=_EMPTY_D,
        torsions=np.zeros((0, 4), np.int32), torsion_n=_EMPTY_I, torsion_k=_EMPTY_D,
        torsion_phi0=_EMPTY_D,
        restraints=_EMPTY_I, restraint_ref=np.zeros((0, 3)), restraint_k=_EMPTY_D,
        pairs14=np.zeros((0, 2), np.int32), scale14=0.5,
        exclusions=np.zeros((0, 2), np.int32),
        kT=1.0, gamma=1.0, dt=0.001, seed=1,
        t_gr=1, t_check_dephase=1, t_check_parallel=1, tol=0.05, t_min=0,
        state=None, obs=[],
    )


def round_to_f32(spec):
    """Copy of ``spec`` whose positions and velocities are exactly representable in
    binary32, so that an FP32 and an FP64 implementation start from the same point."""
    s = dict(spec)
    s["pos"] = np.asarray(spec["pos"], np.float64).astype(np.float32).astype(np.float64)
    if spec.get("vel") is not None:
        s["vel"] = np.asarray(spec["vel"], np.float64).astype(np.float32).astype(np.float64)
    return s


# ---------------------------------------------------------------------------- toy
def toy2d(seed: int = 1, n_replicas: int = 8, beta: float = 5.0, dt: float = 0.01,
          gamma: float = 1.0, t_gr: int = 1, t_check: int = 10, tol: float = 0.05):
    """Config: one unit-mass particle at (-1, 0) in U = (x^2-1)^2 + 2y^2, beta = 5,
    BAOAB dt = 0.01, gamma = 1, state = sign(x), observables (x, y, U).  Initial
    momenta are drawn by the library (Maxwell-Boltzmann, p ~ N(0, 1/beta))."""
    s = _base(TOY2D, 1, n_replicas)
    s.update(mass=np.ones(1), pos=np.array([[-1.0], [0.0], [0.0]]), vel=None,
             kT=1.0 / beta, gamma=gamma, dt=dt, seed=seed, t_gr=t_gr,
             t_check_dephase=t_check, t_check_parallel=t_check, tol=tol,
             state=dict(kind=STATE_SIGN_X, atoms=[0]),
             obs=[dict(kind=OBS_COORD, atoms=[0, 0]), dict(kind=OBS_COORD, atoms=[0, 1]),
                  dict(kind=OBS_POTENTIAL)])
    return s


# ---------------------------------------------------------------------------- geometry
def _place(a, b, c, bond, angle, dihedral):
    """Position of atom d with |cd| = bond, angle(b, c, d) = angle and IUPAC dihedral
    (a, b, c, d) = dihedral (natural extension of reference frame)."""
    bc = c - b
    bc /= np.linalg.norm(bc)
    nrm = np.cross(b - a, bc)
    nrm /= np.linalg.norm(nrm)
    m = np.cross(nrm, bc)
    d2 = np.array([-bond * math.cos(angle),
                   bond * math.sin(angle) * math.cos(dihedral),
                   bond * math.sin(angle) * math.sin(dihedral)])
    return c + d2[0] * bc + d2[1] * m + d2[2] * nrm


def _chain_topology(first: int, count: int, rng, bond_k=2.0e5, angle_k=400.0,
                    theta0=1.91, r0=None):
    """Bonded lists of a linear chain of atoms first..first+count-1."""
    idx = np.arange(first, first + count)
    bonds = np.stack([idx[:-1], idx[1:]], 1)
    angles = np.stack([idx[:-2], idx[1:-1], idx[2:]], 1)
    dihed = np.stack([idx[:-3], idx[1:-2], idx[2:-1], idx[3:]], 1)
    if r0 is None:
        r0 = rng.uniform(0.10, 0.15, len(bonds))
    return dict(bonds=bonds, bond_r0=np.asarray(r0, np.float64), bond_k=np.full(len(bonds), bond_k),
                angles=angles, angle_theta0=np.full(len(angles), theta0),
                angle_k=np.full(len(angles), angle_k), dihedrals=dihed,
                barrier=rng.uniform(4.0, 12.0, len(dihed)))


def _nonbonded_params(rng, count):
    sigma = rng.uniform(0.25, 0.35, count)
    eps = rng.uniform(0.1, 0.9, count)
    q = rng.normal(0.0, 0.3, count)
    q -= q.mean()  # neutral molecule
    return sigma, eps, q


def _merge_topologies(tops):
    out = {}
    for key in ("bonds", "angles", "dihedrals"):
        out[key] = np.concatenate([t[key] for t in tops]).astype(np.int32)
    for key in ("bond_r0", "bond_k", "angle_theta0", "angle_k", "barrier"):
        out[key] = np.concatenate([t[key] for t in tops]).astype(np.float64)
    return out


def _fill_bonded(s, top, extra_torsions=()):
    """Torsions: n = 3 with k = barrier/2 (barrier = 2k for k(1 + cos n phi)) on every
    dihedral; 1-2 and 1-3 pairs excluded; 1-4 pairs scaled by 0.5."""
    dih = top["dihedrals"]
    tors = [dih]
    tn = [np.full(len(dih), 3, np.int32)]
    tk = [top["barrier"] / 2.0]
    tp = [np.zeros(len(dih))]
    for atoms, n, k, p0 in extra_torsions:
        tors.append(np.array([atoms], np.int32))
        tn.append(np.array([n], np.int32))
        tk.append(np.array([k], np.float64))
        tp.append(np.array([p0], np.float64))
    s.update(bonds=top["bonds"], bond_r0=top["bond_r0"], bond_k=top["bond_k"],
             angles=top["angles"], angle_theta0=top["angle_theta0"], angle_k=top["angle_k"],
             torsions=np.concatenate(tors).astype(np.int32), torsion_n=np.concatenate(tn),
             torsion_k=np.concatenate(tk), torsion_phi0=np.concatenate(tp))
    excl = np.concatenate([top["bonds"], top["angles"][:, [0, 2]]]).astype(np.int32)
    s["exclusions"] = excl
    s["pairs14"] = dih[:, [0, 3]].astype(np.int32).copy()
    s["scale14"] = 0.5


# ---------------------------------------------------------------------------- 22-atom chain
def chain(seed: int = 2, n_replicas: int = 256, n_atoms: int = 22, phi0: float = -math.pi / 2,
          psi0: float = -math.pi / 2, k1: float = 1.0, k2: float = 6.0, temperature: float = 300.0,
          gamma: float = 1.0, dt: float = 0.001, t_gr: int = 10, t_check: int = 250,
          t_check_parallel: int = 2500, tol: float = 0.05):
    """Config: the alanine-dipeptide-sized chain.  Masses from {1, 12, 14, 16} amu; bonds
    r0 ~ U(0.10, 0.15) nm, k = 2e5; angles theta0 = 1.91 rad, k = 400; n = 3 torsions with
    barrier ~ U(4, 12) kJ/mol on every dihedral and extra n = 1 (k1) and n = 2 (k2) terms on
    phi = (9,10,11,12) and psi = (10,11,12,13); LJ sigma ~ U(0.25, 0.35), eps ~ U(0.1, 0.9);
    charges ~ N(0, 0.3) neutralised; vacuum, all pairs; T = 300 K, gamma = 1/ps, dt = 1 fs.
    Start: all-trans chain with (phi, psi) = (phi0, psi0).  State = 2 [phi > 0] + [psi > 0].
    Periods follow Sec. 4.1.2 (t_GR = 10 dt, t_check = 250 dt / 2500 dt)."""
    rng = np.random.default_rng(seed)
    n = n_atoms
    top = _chain_topology(0, n, rng)
    phi_a, psi_a = (9, 10, 11, 12), (10, 11, 12, 13)
    if n < 14:
        phi_a, psi_a = (n // 2 - 2, n // 2 - 1, n // 2, n // 2 + 1), (n // 2 - 1, n // 2, n // 2 + 1, n // 2 + 2)
    dih = np.full(n, math.pi)
    dih[phi_a[3]] = phi0
    dih[psi_a[3]] = psi0
    pos = np.zeros((n, 3))
    pos[1] = [top["bond_r0"][0], 0.0, 0.0]
    th = 1.91
    pos[2] = pos[1] + top["bond_r0"][1] * np.array([-math.cos(th), math.sin(th), 0.0])
    for i in range(3, n):
        pos[i] = _place(pos[i - 3], pos[i - 2], pos[i - 1], top["bond_r0"][i - 1], th, dih[i])
    pos -= pos.mean(0)
    s = _base(MOLECULAR, n, n_replicas)
    sigma, eps, q = _nonbonded_params(rng, n)
    mass = rng.choice(np.array([1.0, 12.0, 14.0, 16.0]), n)
    _fill_bonded(s, top, extra_torsions=[(phi_a, 1, k1, 0.0), (phi_a, 2, k2, 0.0),
                                         (psi_a, 1, k1, 0.0), (psi_a, 2, k2, 0.0)])
    lo, mid, hi = -4.0, 0.0, 4.0
    boxes = [[lo, mid, lo, mid], [lo, mid, mid, hi], [mid, hi, lo, mid], [mid, hi, mid, hi]]
    s.update(mass=mass, pos=pos.T.copy(), vel=None, sigma=sigma, epsilon=eps, charge=q,
             cutoff=0.0, kT=KB * temperature, gamma=gamma, dt=dt, seed=seed, t_gr=t_gr,
             t_check_dephase=t_check, t_check_parallel=t_check_parallel, tol=tol,
             state=dict(kind=STATE_DIHEDRAL_BOXES, atoms=list(phi_a) + list(psi_a), boxes=boxes),
             obs=[dict(kind=OBS_POTENTIAL), dict(kind=OBS_KINETIC),
                  dict(kind=OBS_DIHEDRAL, atoms=list(phi_a)), dict(kind=OBS_DIHEDRAL, atoms=list(psi_a))])
    return s


# ---------------------------------------------------------------------------- receptor-ligand
def _grow_chain(rng, count, start, inside, others, min_dist, bond_r0, theta0=1.91, tries=60):
    """Self-avoiding chain growth by internal coordinates: random dihedrals in
    [60, 300] degrees; each new atom must satisfy ``inside`` and keep ``min_dist`` from every
    earlier atom except its three chain predecessors and from every atom in ``others``."""
    pts = np.zeros((count, 3))
    pts[0] = start
    attempt = 0
    i = 1
    while i < count:
        attempt += 1
        if attempt > 200 * count:
            raise RuntimeError("chain growth failed")
        ok = False
        for _ in range(tries):
            if i == 1:
                d = rng.normal(size=3)
                cand = pts[0] + bond_r0[0] * d / np.linalg.norm(d)
            elif i == 2:
                u = pts[1] - pts[0]
                u /= np.linalg.norm(u)
                w = rng.normal(size=3)
                w -= w.dot(u) * u
                w /= np.linalg.norm(w)
                cand = pts[1] + bond_r0[1] * (-math.cos(theta0) * u + math.sin(theta0) * w)
            else:
                phi = math.radians(rng.uniform(60.0, 300.0))
                cand = _place(pts[i - 3], pts[i - 2], pts[i - 1], bond_r0[i - 1], theta0, phi)
            if not inside(cand):
                continue
            if i > 3 and np.min(np.sum((pts[: i - 3] - cand) ** 2, 1)) < min_dist ** 2:
                continue
            if len(others) and np.min(np.sum((others - cand) ** 2, 1)) < min_dist ** 2:
                continue
            ok = True
            break
        if ok:
            pts[i] = cand
            i += 1
        else:
            i = max(1, i - 4)  # back up a few atoms and regrow
    return pts


@functools.lru_cache(maxsize=8)
def _receptor_ligand_cached(seed, n_receptor, n_ligand, radius, pocket_dist, cavity,
                            ligand_radius, min_dist):
    rng = np.random.default_rng(seed)
    p = np.array([pocket_dist, 0.0, 0.0])
    rtop = _chain_topology(0, n_receptor, rng)
    ltop = _chain_topology(n_receptor, n_ligand, rng)

    def in_receptor(x):
        return x.dot(x) < radius ** 2 and np.sum((x - p) ** 2) > cavity ** 2

    start = -p * 0.9
    rec = _grow_chain(rng, n_receptor, start, in_receptor, np.zeros((0, 3)), min_dist, rtop["bond_r0"])

    def in_pocket(x):
        return np.sum((x - p) ** 2) < ligand_radius ** 2

    lig = _grow_chain(rng, n_ligand, p + np.array([-0.2, 0.0, 0.0]), in_pocket, rec, min_dist,
                      ltop["bond_r0"])
    return rng.bit_generator.state, rec, lig, rtop, ltop, p


def receptor_ligand(seed: int = 3, n_replicas: int = 64, n_receptor: int = 2400, n_ligand: int = 32,
                    radius: float = 4.0, pocket_dist: float | None = None, cavity: float = 1.0,
                    ligand_radius: float = 0.7, min_dist: float = 0.3, restraint_k: float = 1000.0,
                    temperature: float = 300.0, gamma: float = 1.0, dt: float = 0.001,
                    cutoff: float = 1.0, eps_rf: float = 78.5, skin: float = 0.1,
                    nlist_period: int = 10, bound_radius: float = 0.4, t_gr: int = 50,
                    t_check: int = 1000, tol: float = 0.05):
    """Config: receptor chain of ``n_receptor`` atoms grown inside a sphere of ``radius`` nm
    around a cavity of radius 1 nm whose centre p lies ``pocket_dist`` nm (default radius/2)
    from the sphere centre, harmonically restrained (k = 1000) to its generated positions;
    a ligand chain of ``n_ligand`` atoms grown within 0.7 nm of p; bonded terms, masses,
    LJ and charge distributions as in the 22-atom chain (each molecule neutralised);
    cutoff 1.0 nm with reaction-field Coulomb (eps_rf = 78.5); pair list every 10 steps
    with a 0.1 nm skin; state = bound (1) while the ligand COM is within 0.4 nm of p;
    observables V, K, d1, d2, receptor-ligand COM distance, ligand RMS velocity; periods
    t_GR = 50 dt and t_check = 1000 dt as in Sec. 4.2.2."""
    if pocket_dist is None:
        pocket_dist = radius / 2.0
    _, rec, lig, rtop, ltop, p = _receptor_ligand_cached(seed, n_receptor, n_ligand, radius,
                                                         pocket_dist, cavity, ligand_radius, min_dist)
    rng = np.random.default_rng(seed + 7919)
    n = n_receptor + n_ligand
    pos = np.concatenate([rec, lig])
    s = _base(MOLECULAR, n, n_replicas)
    top = _merge_topologies([rtop, ltop])
    _fill_bonded(s, top)
    sr, er, qr = _nonbonded_params(rng, n_receptor)
    sl, el, ql = _nonbonded_params(rng, n_ligand)
    mass = rng.choice(np.array([1.0, 12.0, 14.0, 16.0]), n)
    lig_idx = np.arange(n_receptor, n, dtype=np.int32)
    rec_idx = np.arange(0, n_receptor, dtype=np.int32)
    dpock = np.sum((rec - p) ** 2, 1)
    near = np.argsort(dpock)[:6].astype(np.int32)
    s.update(mass=mass, pos=pos.T.copy(), vel=None,
             sigma=np.concatenate([sr, sl]), epsilon=np.concatenate([er, el]),
             charge=np.concatenate([qr, ql]),
             cutoff=cutoff, eps_rf=eps_rf, skin=skin, nlist_period=nlist_period,
             restraints=rec_idx, restraint_ref=rec.copy(), restraint_k=np.full(n_receptor, restraint_k),
             kT=KB * temperature, gamma=gamma, dt=dt, seed=seed, t_gr=t_gr,
             t_check_dephase=t_check, t_check_parallel=t_check, tol=tol,
             state=dict(kind=STATE_COM_SPHERE, group=lig_idx, center=p.tolist(), radius=bound_radius),
             obs=[dict(kind=OBS_POTENTIAL), dict(kind=OBS_KINETIC),
                  dict(kind=OBS_COM_DISTANCE, group_a=lig_idx[:1], group_b=near[:1]),
                  dict(kind=OBS_COM_DISTANCE, group_a=lig_idx[-1:], group_b=near),
                  dict(kind=OBS_COM_DISTANCE, group_a=lig_idx, group_b=rec_idx),
                  dict(kind=OBS_RMS_VELOCITY, group_a=lig_idx)])
    return s


def config(name: str, **kw):
    """The named workloads: 'toy' (2D double well, R = 8), 'chain22' (22 atoms, R = 256),
    'rl2432' (2,400 + 32 atoms, R = 64), 'rl300' (a 268 + 32-atom receptor-ligand system of
    the uneven-batching mix), 'rl1200' (1,168 + 32 atoms, also of that mix)."""
    if name == "toy":
        return toy2d(**kw)
    if name == "chain22":
        return chain(**kw)
    if name == "rl2432":
        return receptor_ligand(**kw)
    if name == "rl300":
        kw.setdefault("n_receptor", 268)
        kw.setdefault("radius", 2.2)
        return receptor_ligand(**kw)
    if name == "rl1200":
        kw.setdefault("n_receptor", 1168)
        kw.setdefault("radius", 3.2)
        return receptor_ligand(**kw)
    raise KeyError(name)


def uneven_batch(n_replicas: int = 192):
    """The uneven-batching mix: systems of 22, 300, 1,200 and 2,432 atoms (the chain and three
    receptor-ligand systems, each with its own state function), n_replicas each."""
    return [config(name, n_replicas=n_replicas) for name in ("chain22", "rl300", "rl1200", "rl2432")]
