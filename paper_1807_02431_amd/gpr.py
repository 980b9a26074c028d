"""Python binding of the C ABI in include/gpr.h (libgpr_hip.so, gfx950).

Argument marshalling only: every step of the hot path runs in the HIP kernels behind the
C ABI.  Loading fails loudly when the library is missing; there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpr_hip.so")
PROBE_LIB_PATH = os.path.join(_HERE, "libgpr_hip_probe.so")   # the same sources with phase timers
PHASES = ("prologue", "integrate", "exchange", "rebuild", "forces", "tail", "epilogue")

OK, BUDGET = 0, 1
EINVAL, ENOMEM, EDEVICE, EPHASE, EUNSTABLE = -1, -2, -3, -4, -5
PATH_PLAIN, PATH_PERSISTENT = 0, 1
MAX_OBS = 8
MAX_BOXES = 8
NOALLOC_MAX_R = 16384     # GPR_NOALLOC_MAX_R: replicas gpr_fv_plan_noalloc takes


class GprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


class _State(C.Structure):
    _fields_ = [("kind", C.c_int32), ("atoms", C.c_int32 * 8), ("n_boxes", C.c_int32),
                ("box", (C.c_double * 4) * MAX_BOXES), ("n_group", C.c_int32),
                ("group", C.POINTER(C.c_int32)), ("center", C.c_double * 3), ("radius", C.c_double)]


class _Obs(C.Structure):
    _fields_ = [("kind", C.c_int32), ("atoms", C.c_int32 * 4), ("n_a", C.c_int32),
                ("group_a", C.POINTER(C.c_int32)), ("n_b", C.c_int32), ("group_b", C.POINTER(C.c_int32))]


_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)


class _Desc(C.Structure):
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
                ("n_branch", C.c_int64), ("n_samples", C.c_int64), ("rhat", C.c_double * MAX_OBS)]


class _Exit(C.Structure):
    _fields_ = [("M", C.c_int64), ("k", C.c_int32), ("to_state", C.c_int32),
                ("tau_steps", C.c_int64), ("tau", C.c_double)]


# every entry point of include/gpr.h with its ctypes signature
class _BatchOp(C.Structure):
    _fields_ = [("op", C.c_int32), ("status", C.c_int32), ("t_corr", C.c_int64), ("max_steps", C.c_int64),
                ("event", _Event), ("dephase", _Dephase), ("exit", _Exit)]


OP_DECORRELATE, OP_DEPHASE, OP_PARALLEL_STEP = 0, 1, 2

_VP = C.c_void_p
_P64 = C.POINTER(C.c_int64)
SIGNATURES = {
    "gpr_system_create": (C.c_int32, [C.POINTER(_Desc), C.POINTER(_VP)]),
    "gpr_system_destroy": (None, [_VP]),
    "gpr_last_error": (C.c_char_p, [_VP]),
    "gpr_set_stream": (C.c_int32, [_VP, _VP]),
    "gpr_set_path": (C.c_int32, [_VP, C.c_int32]),
    "gpr_set_launch": (C.c_int32, [_VP, C.c_int32, C.c_int32]),
    "gpr_energy_forces": (C.c_int32, [_VP, C.c_int32, C.c_int32, _PD, _PD]),
    "gpr_decorrelate": (C.c_int32, [_VP, C.c_int64, C.c_int64, C.POINTER(_Event)]),
    "gpr_dephase": (C.c_int32, [_VP, C.c_int64, C.POINTER(_Dephase)]),
    "gpr_parallel_step": (C.c_int32, [_VP, C.c_int64, C.POINTER(_Exit)]),
    "gpr_simulated_time": (C.c_double, [_VP]),
    "gpr_simulated_steps": (C.c_int64, [_VP]),
    "gpr_global_step": (C.c_int64, [_VP]),
    "gpr_current_state": (C.c_int32, [_VP]),
    "gpr_advance_steps": (C.c_int64, [_VP]),
    "gpr_get_state": (C.c_int32, [_VP, C.c_int32, _PD, _PD]),
    "gpr_set_state": (C.c_int32, [_VP, C.c_int32, _PD, _PD]),
    "gpr_advance": (C.c_int32, [_VP, C.c_int64, _P64]),
    "gpr_get_accumulators": (C.c_int32, [_VP, _P64, _PD, _PD, _PD]),
    "gpr_profile": (C.c_int32, [_VP, C.c_int32]),
    "gpr_profile_read": (C.c_int32, [_VP, _PD, _P64]),
    "gpr_phase_read": (C.c_int32, [_VP, _PD]),
    "gpr_observe": (C.c_int32, [_VP, _PD, _PI]),
    "gpr_philox_noise": (C.c_int32, [C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                     C.POINTER(C.c_uint32), C.POINTER(C.c_float)]),
    "gpr_fv_plan": (C.c_int32, [C.c_uint64, C.c_int64, C.c_int32, C.POINTER(C.c_uint8), _PI]),
    "gpr_fv_plan_noalloc": (C.c_int32, [C.c_uint64, C.c_int64, C.c_int32, C.POINTER(C.c_uint8), _PI]),
    "gpr_rhat": (C.c_int32, [C.c_int32, C.c_int32, C.c_int64, _PD, _PD, _PD]),
    "gpr_exit_vote": (C.c_int32, [C.c_int32, _P64, C.c_int64, _P64, C.POINTER(C.c_int32), _P64]),
    "gpr_dephase_fixed": (C.c_int32, [_VP, C.c_int64, C.c_int64, C.POINTER(_Dephase)]),
    "gpr_autotune": (C.c_int32, [_VP, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "gpr_set_graph": (C.c_int32, [_VP, C.c_int32]),
    "gpr_set_cycles": (C.c_int32, [_VP, C.c_int32]),
    "gpr_batch_advance": (C.c_int32, [C.POINTER(_VP), C.c_int32, C.c_int64, C.POINTER(_P64)]),
    "gpr_batch_run": (C.c_int32, [C.POINTER(_VP), C.c_int32, C.POINTER(_BatchOp)]),
    "gpr_set_params": (C.c_int32, [_VP, _PD, _PD, _PD, _PD]),
    "gpr_energy_forces_dev": (C.c_int32, [_VP, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gpr_energy_backward_dev": (C.c_int32, [_VP, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
}

_lib = None


def lib():
    """The loaded HIP library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgpr_hip.so is not built (run paper_1807_02431_amd/build.py); "
                              "the GPU library has no fallback path")
        # torch ships its own HIP runtime under the same soname as the system one; whichever is
        # loaded first serves the whole process, and torch fails to initialise on another
        # release's.  Load torch's first so that torch and this library share it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def use_probe_library():
    """Load the phase-timer build (libgpr_hip_probe.so) instead of the product library, for
    measurement; must come before the first call into the library."""
    global LIB_PATH
    if _lib is not None:
        raise RuntimeError("the library is already loaded")
    if not os.path.exists(PROBE_LIB_PATH):
        raise ImportError("libgpr_hip_probe.so is not built (run paper_1807_02431_amd/build.py --probe)")
    LIB_PATH = PROBE_LIB_PATH


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a):
    return a.ctypes.data_as(_PD) if a is not None and a.size else None


def _pi(a):
    return a.ctypes.data_as(_PI) if a is not None and a.size else None


def _check(rc, handle=None):
    if rc < 0:
        msg = lib().gpr_last_error(handle)
        raise GprError(rc, msg.decode() if msg else "error")
    return rc


class System:
    """A batch of replicas of one system on the current HIP device (see include/gpr.h)."""

    def __init__(self, spec: dict, path: int = PATH_PLAIN, stream=None):
        L = lib()
        keep = []
        n = int(spec["n_atoms"])
        self.n, self.R = n, int(spec["n_replicas"])
        self.nt = len(spec["torsions"]) if spec.get("torsions") is not None else 0
        self.nobs = len(spec.get("obs", []))
        d = _Desc()
        d.kind, d.n_atoms, d.n_replicas = int(spec["kind"]), n, self.R

        def D(key):
            v = spec.get(key)
            if v is None:
                return None
            a = _d(v)
            keep.append(a)
            return _pd(a)

        def I(key):
            v = spec.get(key)
            if v is None:
                return None
            a = _i(v)
            keep.append(a)
            return _pi(a)

        d.mass, d.pos, d.vel = D("mass"), D("pos"), D("vel")
        d.sigma, d.epsilon, d.charge = D("sigma"), D("epsilon"), D("charge")
        d.cutoff, d.eps_rf, d.skin = float(spec["cutoff"]), float(spec["eps_rf"]), float(spec["skin"])
        d.nlist_period = int(spec["nlist_period"])
        d.n_bonds, d.bond_atoms, d.bond_r0, d.bond_k = len(spec["bonds"]), I("bonds"), D("bond_r0"), D("bond_k")
        d.n_angles, d.angle_atoms = len(spec["angles"]), I("angles")
        d.angle_theta0, d.angle_k = D("angle_theta0"), D("angle_k")
        d.n_torsions, d.torsion_atoms, d.torsion_n = len(spec["torsions"]), I("torsions"), I("torsion_n")
        d.torsion_k, d.torsion_phi0 = D("torsion_k"), D("torsion_phi0")
        d.n_restraints, d.restraint_atom = len(spec["restraints"]), I("restraints")
        d.restraint_ref, d.restraint_k = D("restraint_ref"), D("restraint_k")
        d.n_pairs14, d.pair14_atoms, d.scale14 = len(spec["pairs14"]), I("pairs14"), float(spec["scale14"])
        d.n_exclusions, d.exclusion_atoms = len(spec["exclusions"]), I("exclusions")
        d.kT, d.gamma, d.dt = float(spec["kT"]), float(spec["gamma"]), float(spec["dt"])
        d.seed = int(spec["seed"]) & 0xFFFFFFFFFFFFFFFF
        d.t_gr, d.t_check_dephase = int(spec["t_gr"]), int(spec["t_check_dephase"])
        d.t_check_parallel, d.tol, d.t_min = int(spec["t_check_parallel"]), float(spec["tol"]), int(spec.get("t_min", 0))
        st = spec["state"]
        d.state.kind = int(st["kind"])
        for a, v in enumerate(st.get("atoms", [])):
            d.state.atoms[a] = int(v)
        boxes = st.get("boxes", [])
        d.state.n_boxes = len(boxes)
        for b, row in enumerate(boxes):
            for c in range(4):
                d.state.box[b][c] = float(row[c])
        if st.get("group") is not None:
            g = _i(st["group"])
            keep.append(g)
            d.state.n_group, d.state.group = len(g), _pi(g)
        for c, v in enumerate(st.get("center", [0.0, 0.0, 0.0])):
            d.state.center[c] = float(v)
        d.state.radius = float(st.get("radius", 0.0))
        obs = (_Obs * max(1, self.nobs))()
        for j, o in enumerate(spec.get("obs", [])):
            obs[j].kind = int(o["kind"])
            for a, v in enumerate(o.get("atoms", [])):
                obs[j].atoms[a] = int(v)
            for nm, cnt in (("group_a", "n_a"), ("group_b", "n_b")):
                if o.get(nm) is not None:
                    g = _i(o[nm])
                    keep.append(g)
                    setattr(obs[j], nm, _pi(g))
                    setattr(obs[j], cnt, len(g))
        d.n_obs, d.obs = self.nobs, obs
        h = C.c_void_p()
        _check(L.gpr_system_create(C.byref(d), C.byref(h)))
        self._h = h
        if stream is not None:
            self.set_stream(stream)
        if path != PATH_PLAIN:
            self.set_path(path)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().gpr_system_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def _c(self, rc):
        return _check(rc, self._h)

    # -------------------------------------------------------------- configuration
    def set_stream(self, stream):
        """stream: a torch.cuda.Stream or a raw hipStream_t value."""
        raw = getattr(stream, "cuda_stream", stream)
        self._c(lib().gpr_set_stream(self._h, C.c_void_p(int(raw))))

    def set_path(self, path):
        self._c(lib().gpr_set_path(self._h, int(path)))

    def set_graph(self, cycle_steps):
        self._c(lib().gpr_set_graph(self._h, int(cycle_steps)))

    def set_cycles(self, cycles):
        """Convergence and parallel steps as replays of `cycles` captured check cycles (0: off)."""
        self._c(lib().gpr_set_cycles(self._h, int(cycles)))

    def autotune(self, nsteps=200):
        """Times the persistent path's launch shapes and keeps the fastest; returns it."""
        bt, g = C.c_int32(), C.c_int32()
        self._c(lib().gpr_autotune(self._h, int(nsteps), C.byref(bt), C.byref(g)))
        return bt.value, g.value

    def set_launch(self, block_threads=0, groups_per_replica=0):
        self._c(lib().gpr_set_launch(self._h, int(block_threads), int(groups_per_replica)))

    def profile(self, enable=True):
        self._c(lib().gpr_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(summed ms, launches) of the dominant stepping kernel since profile() was called."""
        ms = C.c_double()
        n = C.c_int64()
        self._c(lib().gpr_profile_read(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def phase_read(self):
        """gpr_phase_read (timer build only): [R, 8, 11] per replica and workgroup, the
        microseconds in each of PHASES and the counts of steps and of pair-list rebuilds since
        the last read, then the start and end of the last launch (µs after its earliest start)."""
        out = np.zeros((self.R, 8, 11))
        self._c(lib().gpr_phase_read(self._h, out.ctypes.data_as(_PD)))
        return out

    # -------------------------------------------------------------- queries
    def energy_forces(self, r0=0, nr=None):
        nr = self.R - r0 if nr is None else nr
        E = np.zeros(nr)
        F = np.zeros((nr, 3, self.n))
        self._c(lib().gpr_energy_forces(self._h, r0, nr, _pd(E), _pd(F)))
        return E, F

    def get_state(self, r):
        q = np.zeros((3, self.n)); v = np.zeros((3, self.n))
        self._c(lib().gpr_get_state(self._h, r, _pd(q), _pd(v)))
        return q, v

    def set_state(self, r, q, v=None):
        q = _d(q).reshape(3, self.n)
        vv = None if v is None else _d(v).reshape(3, self.n)
        self._c(lib().gpr_set_state(self._h, r, _pd(q), _pd(vv)))

    # -------------------------------------------------------------- differentiation
    def set_params(self, epsilon=None, sigma=None, charge=None, torsion_k=None):
        arrs = [None if a is None else _d(a) for a in (epsilon, sigma, charge, torsion_k)]
        self._c(lib().gpr_set_params(self._h, *[_pd(a) if a is not None else None for a in arrs]))

    def energy_forces_dev(self, x_ptr, energy_ptr, forces_ptr):
        """Device pointers (ints): x float [R][3][n] in, energy double [R] and forces float
        [R][3][n] out (0 for none)."""
        self._c(lib().gpr_energy_forces_dev(self._h, C.c_void_p(x_ptr), C.c_void_p(energy_ptr or None),
                                            C.c_void_p(forces_ptr or None)))

    def energy_backward_dev(self, w_ptr, dx_ptr, d_eps_ptr, d_sigma_ptr, d_charge_ptr, d_tk_ptr):
        """Device pointers (ints, 0 for none): weights double [R] in; dx float [R][3][n] and the
        parameter gradients (double) out."""
        self._c(lib().gpr_energy_backward_dev(self._h, C.c_void_p(w_ptr), *[C.c_void_p(p or None) for p in
                                              (dx_ptr, d_eps_ptr, d_sigma_ptr, d_charge_ptr, d_tk_ptr)]))

    def simulated_time(self):
        return lib().gpr_simulated_time(self._h)

    def simulated_steps(self):
        return lib().gpr_simulated_steps(self._h)

    def global_step(self):
        return lib().gpr_global_step(self._h)

    def current_state(self):
        return lib().gpr_current_state(self._h)

    def observe(self):
        obs = np.zeros((self.R, max(1, self.nobs)))
        st = np.zeros(self.R, np.int32)
        self._c(lib().gpr_observe(self._h, _pd(obs), _pi(st)))
        return obs[:, : self.nobs], st

    def accumulators(self):
        n = C.c_int64()
        S1 = np.zeros((self.R, max(1, self.nobs)))
        S2 = np.zeros((self.R, max(1, self.nobs)))
        sh = np.zeros(max(1, self.nobs))
        self._c(lib().gpr_get_accumulators(self._h, C.byref(n), _pd(S1), _pd(S2), _pd(sh)))
        return n.value, S1[:, : self.nobs], S2[:, : self.nobs], sh[: self.nobs]

    # -------------------------------------------------------------- Gen.ParRep steps
    def decorrelate(self, t_corr, max_steps=1 << 62):
        ev = _Event()
        rc = self._c(lib().gpr_decorrelate(self._h, int(t_corr), int(max_steps), C.byref(ev)))
        return rc, dict(kind=ev.kind, from_state=ev.from_state, to_state=ev.to_state,
                        resident_steps=ev.resident_steps, steps_taken=ev.steps_taken)

    def dephase(self, max_steps=1 << 62):
        o = _Dephase()
        rc = self._c(lib().gpr_dephase(self._h, int(max_steps), C.byref(o)))
        return rc, dict(outcome=o.outcome, to_state=o.to_state, t_steps=o.t_steps, n_branch=o.n_branch,
                        n_samples=o.n_samples, rhat=list(o.rhat)[: self.nobs])

    def dephase_fixed(self, t_phase, max_steps=1 << 62):
        o = _Dephase()
        rc = self._c(lib().gpr_dephase_fixed(self._h, int(t_phase), int(max_steps), C.byref(o)))
        return rc, dict(outcome=o.outcome, to_state=o.to_state, t_steps=o.t_steps, n_branch=o.n_branch)

    def parallel_step(self, max_checks=1 << 62):
        o = _Exit()
        rc = self._c(lib().gpr_parallel_step(self._h, int(max_checks), C.byref(o)))
        return rc, dict(M=o.M, k=o.k, to_state=o.to_state, tau_steps=o.tau_steps, tau=o.tau)

    def advance_steps(self):
        """Steps taken by advance / batch_advance since creation (their schedule's position)."""
        return lib().gpr_advance_steps(self._h)

    def advance(self, nsteps, first_exit=True):
        """gpr_advance; returns the first exit checks, or None with first_exit=False (then
        they are not read back)."""
        if not first_exit:
            self._c(lib().gpr_advance(self._h, int(nsteps), None))
            return None
        fec = np.zeros(self.R, np.int64)
        self._c(lib().gpr_advance(self._h, int(nsteps), fec.ctypes.data_as(_P64)))
        return fec


def batch_advance(systems, nsteps):
    """gpr_advance of several systems whose persistent steps share launches; returns each
    system's first-exit-check array."""
    hs = (_VP * len(systems))(*[x._h for x in systems])
    fec = [np.zeros(x.R, np.int64) for x in systems]
    ptrs = (_P64 * len(systems))(*[f.ctypes.data_as(_P64) for f in fec])
    _check(lib().gpr_batch_advance(hs, len(systems), int(nsteps), ptrs), systems[0]._h)
    return fec


def _event_dict(ev):
    return dict(kind=ev.kind, from_state=ev.from_state, to_state=ev.to_state,
                resident_steps=ev.resident_steps, steps_taken=ev.steps_taken)


def _dephase_dict(o, nobs):
    return dict(outcome=o.outcome, to_state=o.to_state, t_steps=o.t_steps, n_branch=o.n_branch,
                n_samples=o.n_samples, rhat=list(o.rhat)[:nobs])


def _exit_dict(o):
    return dict(M=o.M, k=o.k, to_state=o.to_state, tau_steps=o.tau_steps, tau=o.tau)


def batch_run(systems, ops):
    """Gen.ParRep calls of several systems with their steps in shared persistent launches.
    ops[k]: dict(op=OP_DECORRELATE | OP_DEPHASE | OP_PARALLEL_STEP, t_corr=..., max_steps=...);
    returns [(status, result dict as the single-system call returns it)]."""
    hs = (_VP * len(systems))(*[x._h for x in systems])
    arr = (_BatchOp * len(systems))()
    for a, o in zip(arr, ops):
        a.op = int(o["op"])
        a.t_corr = int(o.get("t_corr", 0))
        a.max_steps = int(o.get("max_steps", 1 << 62))
    _check(lib().gpr_batch_run(hs, len(systems), arr), systems[0]._h)
    out = []
    for a, x in zip(arr, systems):
        if a.op == OP_DECORRELATE:
            res = _event_dict(a.event)
        elif a.op == OP_DEPHASE:
            res = _dephase_dict(a.dephase, x.nobs)
        else:
            res = _exit_dict(a.exit)
        out.append((a.status, res))
    return out


# ------------------------------------------------------------------ building blocks
def philox_noise(seed, replica, step, stream, n_atoms):
    w = np.zeros((n_atoms, 4), np.uint32)
    g = np.zeros((n_atoms, 3), np.float32)
    _check(lib().gpr_philox_noise(int(seed) & 0xFFFFFFFFFFFFFFFF, replica, int(step), stream, n_atoms,
                                  w.ctypes.data_as(C.POINTER(C.c_uint32)), g.ctypes.data_as(C.POINTER(C.c_float))))
    return w, g


def fv_plan(seed, step, exited):
    ex = np.ascontiguousarray(exited, np.uint8)
    donor = np.zeros(len(ex), np.int32)
    _check(lib().gpr_fv_plan(int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), len(ex),
                             ex.ctypes.data_as(C.POINTER(C.c_uint8)), _pi(donor)))
    return donor


def fv_plan_noalloc(seed, step, exited):
    """gpr_fv_plan staged through the library's static device array (no allocation)."""
    ex = np.ascontiguousarray(exited, np.uint8)
    donor = np.zeros(len(ex), np.int32)
    _check(lib().gpr_fv_plan_noalloc(int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), len(ex),
                                     ex.ctypes.data_as(C.POINTER(C.c_uint8)), _pi(donor)))
    return donor


def rhat(n, S1, S2):
    S1 = _d(S1); S2 = _d(S2)
    nw, no = S1.shape
    out = np.zeros(no)
    _check(lib().gpr_rhat(nw, no, int(n), _pd(S1), _pd(S2), _pd(out)))
    return out


def exit_vote(first_exit_check, t_check):
    f = np.ascontiguousarray(first_exit_check, np.int64)
    M = C.c_int64(); k = C.c_int32(); tau = C.c_int64()
    rc = _check(lib().gpr_exit_vote(len(f), f.ctypes.data_as(_P64), int(t_check), C.byref(M), C.byref(k), C.byref(tau)))
    if rc == BUDGET:
        return None
    return M.value, k.value, tau.value
