"""ctypes wrapper of the FP64 CPU oracle (``gpr_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference implementation of the
Gen.ParRep hot path (arXiv 1807.02431, Sec. 2.1-2.4 and the force field of Sec. 3.2) that
the GPU library is checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU library and
does not import it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpr_oracle.c")
_LIB = os.path.join(_HERE, "libgpr_oracle.so")

OK, BUDGET = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _State(C.Structure):
    _fields_ = [("kind", C.c_int32), ("atoms", C.c_int32 * 8), ("n_boxes", C.c_int32),
                ("box", (C.c_double * 4) * 8), ("n_group", C.c_int32),
                ("group", C.POINTER(C.c_int32)), ("center", C.c_double * 3), ("radius", C.c_double)]


class _Obs(C.Structure):
    _fields_ = [("kind", C.c_int32), ("atoms", C.c_int32 * 4), ("n_a", C.c_int32),
                ("group_a", C.POINTER(C.c_int32)), ("n_b", C.c_int32), ("group_b", C.POINTER(C.c_int32))]


_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)


class _Spec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_atoms", C.c_int32), ("n_replicas", C.c_int32),
                ("mass", _PD), ("pos", _PD), ("vel", _PD),
                ("sigma", _PD), ("epsilon", _PD), ("charge", _PD),
                ("cutoff", C.c_double), ("eps_rf", C.c_double), ("skin", C.c_double),
                ("nlist_period", C.c_int32),
                ("n_bonds", C.c_int32), ("bond_atoms", _PI), ("bond_r0", _PD), ("bond_k", _PD),
                ("n_angles", C.c_int32), ("angle_atoms", _PI), ("angle_theta0", _PD), ("angle_k", _PD),
                ("n_torsions", C.c_int32), ("torsion_atoms", _PI), ("torsion_n", _PI),
                ("torsion_k", _PD), ("torsion_phi0", _PD),
                ("n_restraints", C.c_int32), ("restraint_atom", _PI), ("restraint_ref", _PD),
                ("restraint_k", _PD),
                ("n_pairs14", C.c_int32), ("pair14_atoms", _PI), ("scale14", C.c_double),
                ("n_exclusions", C.c_int32), ("exclusion_atoms", _PI),
                ("kT", C.c_double), ("gamma", C.c_double), ("dt", C.c_double), ("seed", C.c_uint64),
                ("t_gr", C.c_int32), ("t_check_dephase", C.c_int32), ("t_check_parallel", C.c_int32),
                ("tol", C.c_double), ("t_min", C.c_int64),
                ("state", _State), ("n_obs", C.c_int32), ("obs", C.POINTER(_Obs))]


class _Event(C.Structure):
    _fields_ = [("kind", C.c_int32), ("from_state", C.c_int32), ("to_state", C.c_int32),
                ("pad", C.c_int32), ("resident_steps", C.c_int64), ("steps_taken", C.c_int64)]


class _Dephase(C.Structure):
    _fields_ = [("outcome", C.c_int32), ("to_state", C.c_int32), ("t_steps", C.c_int64),
                ("n_branch", C.c_int64), ("n_samples", C.c_int64), ("rhat", C.c_double * 8)]


class _Exit(C.Structure):
    _fields_ = [("M", C.c_int64), ("k", C.c_int32), ("to_state", C.c_int32),
                ("tau_steps", C.c_int64), ("tau", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        vp = C.c_void_p
        L.gro_create.argtypes = [C.POINTER(_Spec), C.POINTER(vp)]
        L.gro_destroy.argtypes = [vp]
        L.gro_destroy.restype = None
        L.gro_error.restype = C.c_char_p
        L.gro_eval.argtypes = [vp, _PD, _PD, _PD]
        L.gro_param_grad.argtypes = [vp, _PD, _PD, _PD, _PD, _PD]
        L.gro_energy_forces.argtypes = [vp, C.c_int32, C.c_int32, _PD, _PD]
        L.gro_decorrelate.argtypes = [vp, C.c_int64, C.c_int64, C.POINTER(_Event)]
        L.gro_dephase.argtypes = [vp, C.c_int64, C.POINTER(_Dephase)]
        L.gro_dephase_fixed.argtypes = [vp, C.c_int64, C.c_int64, C.POINTER(_Dephase)]
        L.gro_parallel_step.argtypes = [vp, C.c_int64, C.POINTER(_Exit)]
        L.gro_advance.argtypes = [vp, C.c_int64, C.POINTER(C.c_int64)]
        L.gro_step_replicas.argtypes = [vp, C.c_int64, C.c_int32, C.c_int32]
        L.gro_simulated_time.argtypes = [vp]
        L.gro_simulated_time.restype = C.c_double
        for f in ("gro_simulated_steps", "gro_global_step"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = C.c_int64
        L.gro_current_state.argtypes = [vp]
        L.gro_current_state.restype = C.c_int32
        L.gro_get_state.argtypes = [vp, C.c_int32, _PD, _PD]
        L.gro_set_state.argtypes = [vp, C.c_int32, _PD, _PD]
        L.gro_get_accumulators.argtypes = [vp, C.POINTER(C.c_int64), _PD, _PD, _PD]
        L.gro_observe.argtypes = [vp, _PD, _PI]
        L.gro_state_of.argtypes = [vp, _PD]
        L.gro_state_of.restype = C.c_int32
        L.gro_observables_of.argtypes = [vp, _PD, _PD, C.c_double, _PD]
        L.gro_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.gro_philox4x32_10.restype = None
        L.gro_noise.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                C.POINTER(C.c_uint32), _PD]
        L.gro_noise.restype = None
        L.gro_fv_plan.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.POINTER(C.c_uint8), _PI]
        L.gro_rhat.argtypes = [C.c_int32, C.c_int32, C.c_int64, _PD, _PD, _PD]
        L.gro_exit_vote.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.c_int64,
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a):
    return a.ctypes.data_as(_PD) if a is not None and a.size else None


def _pi(a):
    return a.ctypes.data_as(_PI) if a is not None and a.size else None


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc < 0:
        raise OracleError("%s failed (%d): %s" % (what, rc, lib().gro_error().decode()))
    return rc


class System:
    """One oracle system built from a descriptor dict (see ``gpr_synth``)."""

    def __init__(self, spec: dict):
        L = lib()
        self._keep = []
        k = self._keep.append
        n = int(spec["n_atoms"])
        self.n = n
        self.R = int(spec["n_replicas"])
        self.nobs = len(spec.get("obs", []))
        self.nt = len(spec.get("torsion_k", []) if spec.get("torsion_k") is not None else [])
        s = _Spec()
        s.kind, s.n_atoms, s.n_replicas = int(spec["kind"]), n, self.R

        def D(key, shape=None):
            v = spec.get(key)
            if v is None:
                return None
            a = _d(v)
            k(a)
            return _pd(a)

        def I(key):
            v = spec.get(key)
            if v is None:
                return None
            a = _i(v)
            k(a)
            return _pi(a)

        s.mass, s.pos, s.vel = D("mass"), D("pos"), D("vel")
        s.sigma, s.epsilon, s.charge = D("sigma"), D("epsilon"), D("charge")
        s.cutoff, s.eps_rf, s.skin = float(spec["cutoff"]), float(spec["eps_rf"]), float(spec["skin"])
        s.nlist_period = int(spec["nlist_period"])
        s.n_bonds = len(spec["bonds"]); s.bond_atoms = I("bonds"); s.bond_r0 = D("bond_r0"); s.bond_k = D("bond_k")
        s.n_angles = len(spec["angles"]); s.angle_atoms = I("angles")
        s.angle_theta0 = D("angle_theta0"); s.angle_k = D("angle_k")
        s.n_torsions = len(spec["torsions"]); s.torsion_atoms = I("torsions"); s.torsion_n = I("torsion_n")
        s.torsion_k = D("torsion_k"); s.torsion_phi0 = D("torsion_phi0")
        s.n_restraints = len(spec["restraints"]); s.restraint_atom = I("restraints")
        s.restraint_ref = D("restraint_ref"); s.restraint_k = D("restraint_k")
        s.n_pairs14 = len(spec["pairs14"]); s.pair14_atoms = I("pairs14"); s.scale14 = float(spec["scale14"])
        s.n_exclusions = len(spec["exclusions"]); s.exclusion_atoms = I("exclusions")
        s.kT, s.gamma, s.dt = float(spec["kT"]), float(spec["gamma"]), float(spec["dt"])
        s.seed = int(spec["seed"]) & 0xFFFFFFFFFFFFFFFF
        s.t_gr, s.t_check_dephase = int(spec["t_gr"]), int(spec["t_check_dephase"])
        s.t_check_parallel = int(spec["t_check_parallel"])
        s.tol, s.t_min = float(spec["tol"]), int(spec.get("t_min", 0))
        st = spec["state"]
        s.state.kind = int(st["kind"])
        for a, v in enumerate(st.get("atoms", [])):
            s.state.atoms[a] = int(v)
        boxes = st.get("boxes", [])
        s.state.n_boxes = len(boxes)
        for b, row in enumerate(boxes):
            for c in range(4):
                s.state.box[b][c] = float(row[c])
        if st.get("group") is not None:
            g = _i(st["group"]); k(g)
            s.state.n_group = len(g); s.state.group = _pi(g)
        for c, v in enumerate(st.get("center", [0, 0, 0])):
            s.state.center[c] = float(v)
        s.state.radius = float(st.get("radius", 0.0))
        obs = (_Obs * max(1, self.nobs))()
        for j, o in enumerate(spec.get("obs", [])):
            obs[j].kind = int(o["kind"])
            for a, v in enumerate(o.get("atoms", [])):
                obs[j].atoms[a] = int(v)
            for nm, cnt in (("group_a", "n_a"), ("group_b", "n_b")):
                if o.get(nm) is not None:
                    g = _i(o[nm]); k(g)
                    setattr(obs[j], nm, _pi(g)); setattr(obs[j], cnt, len(g))
        k(obs)
        s.n_obs = self.nobs
        s.obs = obs
        h = C.c_void_p()
        _check(L.gro_create(C.byref(s), C.byref(h)), "gro_create")
        self._h = h
        self._keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().gro_destroy(h)
            self._h = None

    # -------------------------------------------------------------- queries
    def eval(self, q):
        q = _d(q).reshape(3, self.n)
        F = np.zeros((3, self.n))
        U = C.c_double()
        _check(lib().gro_eval(self._h, _pd(q), _pd(F), C.byref(U)), "gro_eval")
        return U.value, F

    def param_grad(self, q):
        """dU/d(eps, sigma, charge, torsion k) at positions q (Sec. 3.2 force field)."""
        q = _d(q).reshape(3, self.n)
        nt = self.nt
        ge, gs, gq = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        gk = np.zeros(max(1, nt))
        _check(lib().gro_param_grad(self._h, _pd(q), _pd(ge), _pd(gs), _pd(gq), _pd(gk)), "gro_param_grad")
        return dict(epsilon=ge, sigma=gs, charge=gq, torsion_k=gk[:nt])

    def energy_forces(self, r0=0, nr=None):
        nr = self.R - r0 if nr is None else nr
        E = np.zeros(nr)
        F = np.zeros((nr, 3, self.n))
        _check(lib().gro_energy_forces(self._h, r0, nr, _pd(E), _pd(F)), "gro_energy_forces")
        return E, F

    def get_state(self, r):
        q = np.zeros((3, self.n)); v = np.zeros((3, self.n))
        _check(lib().gro_get_state(self._h, r, _pd(q), _pd(v)), "gro_get_state")
        return q, v

    def set_state(self, r, q, v=None):
        q = _d(q).reshape(3, self.n)
        vv = None if v is None else _d(v).reshape(3, self.n)
        _check(lib().gro_set_state(self._h, r, _pd(q), _pd(vv)), "gro_set_state")

    def simulated_time(self):
        return lib().gro_simulated_time(self._h)

    def simulated_steps(self):
        return lib().gro_simulated_steps(self._h)

    def global_step(self):
        return lib().gro_global_step(self._h)

    def current_state(self):
        return lib().gro_current_state(self._h)

    def state_of(self, q):
        return lib().gro_state_of(self._h, _pd(_d(q).reshape(3, self.n)))

    def observables_of(self, q, v, U):
        out = np.zeros(max(1, self.nobs))
        _check(lib().gro_observables_of(self._h, _pd(_d(q)), _pd(_d(v)), float(U), _pd(out)), "observables")
        return out[: self.nobs]

    def observe(self):
        obs = np.zeros((self.R, max(1, self.nobs)))
        st = np.zeros(self.R, np.int32)
        _check(lib().gro_observe(self._h, _pd(obs), _pi(st)), "gro_observe")
        return obs[:, : self.nobs], st

    def accumulators(self):
        n = C.c_int64()
        S1 = np.zeros((self.R, max(1, self.nobs)))
        S2 = np.zeros((self.R, max(1, self.nobs)))
        sh = np.zeros(max(1, self.nobs))
        _check(lib().gro_get_accumulators(self._h, C.byref(n), _pd(S1), _pd(S2), _pd(sh)), "accumulators")
        return n.value, S1[:, : self.nobs], S2[:, : self.nobs], sh[: self.nobs]

    # -------------------------------------------------------------- Gen.ParRep steps
    def decorrelate(self, t_corr, max_steps=1 << 62):
        ev = _Event()
        rc = _check(lib().gro_decorrelate(self._h, int(t_corr), int(max_steps), C.byref(ev)), "decorrelate")
        return rc, dict(kind=ev.kind, from_state=ev.from_state, to_state=ev.to_state,
                        resident_steps=ev.resident_steps, steps_taken=ev.steps_taken)

    def dephase(self, max_steps=1 << 62):
        o = _Dephase()
        rc = _check(lib().gro_dephase(self._h, int(max_steps), C.byref(o)), "dephase")
        return rc, dict(outcome=o.outcome, to_state=o.to_state, t_steps=o.t_steps, n_branch=o.n_branch,
                        n_samples=o.n_samples, rhat=list(o.rhat)[: self.nobs])

    def dephase_fixed(self, t_phase, max_steps=1 << 62):
        """Original ParRep dephasing (Sec. 2.4.3): every replica stays t_phase in Omega."""
        o = _Dephase()
        rc = _check(lib().gro_dephase_fixed(self._h, int(t_phase), int(max_steps), C.byref(o)), "dephase_fixed")
        return rc, dict(outcome=o.outcome, to_state=o.to_state, t_steps=o.t_steps, n_branch=o.n_branch)

    def parallel_step(self, max_checks=1 << 62):
        o = _Exit()
        rc = _check(lib().gro_parallel_step(self._h, int(max_checks), C.byref(o)), "parallel_step")
        return rc, dict(M=o.M, k=o.k, to_state=o.to_state, tau_steps=o.tau_steps, tau=o.tau)

    def step_replicas(self, nsteps, r_lo, r_hi):
        _check(lib().gro_step_replicas(self._h, int(nsteps), int(r_lo), int(r_hi)), "step_replicas")

    def advance(self, nsteps):
        fec = np.zeros(self.R, np.int64)
        _check(lib().gro_advance(self._h, int(nsteps), fec.ctypes.data_as(C.POINTER(C.c_int64))), "advance")
        return fec


# ------------------------------------------------------------------ building blocks
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().gro_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def noise(seed, replica, step, stream, n_atoms):
    w = np.zeros((n_atoms, 4), np.uint32)
    g = np.zeros((n_atoms, 3))
    lib().gro_noise(int(seed) & 0xFFFFFFFFFFFFFFFF, replica, step, stream, n_atoms,
                    w.ctypes.data_as(C.POINTER(C.c_uint32)), _pd(g))
    return w, g


def fv_plan(seed, step, exited):
    ex = np.ascontiguousarray(exited, np.uint8)
    donor = np.zeros(len(ex), np.int32)
    _check(lib().gro_fv_plan(int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), len(ex),
                             ex.ctypes.data_as(C.POINTER(C.c_uint8)), _pi(donor)), "fv_plan")
    return donor


def rhat(n, S1, S2):
    S1 = _d(S1); S2 = _d(S2)
    nw, no = S1.shape
    out = np.zeros(no)
    _check(lib().gro_rhat(nw, no, int(n), _pd(S1), _pd(S2), _pd(out)), "rhat")
    return out


def exit_vote(first_exit_check, t_check):
    f = np.ascontiguousarray(first_exit_check, np.int64)
    M = C.c_int64(); k = C.c_int32(); tau = C.c_int64()
    rc = lib().gro_exit_vote(len(f), f.ctypes.data_as(C.POINTER(C.c_int64)), int(t_check),
                             C.byref(M), C.byref(k), C.byref(tau))
    if rc == BUDGET:
        return None
    return M.value, k.value, tau.value
