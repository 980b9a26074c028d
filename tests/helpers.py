"""Small hand-built systems shared by the tests (inputs only, no method arithmetic)."""
import numpy as np

import gpr_synth as G


def mini(pos, mass=None, sigma=0.3, epsilon=0.5, charge=0.0, R=2, **kw):
    """A molecular system with atoms at ``pos`` ([n][3]) and no terms unless given."""
    pos = np.asarray(pos, np.float64)
    n = len(pos)
    s = G._base(G.MOLECULAR, n, R)
    s.update(mass=np.full(n, 12.0) if mass is None else np.asarray(mass, np.float64),
             pos=pos.T.copy(), vel=np.zeros((3, n)),
             sigma=np.broadcast_to(np.asarray(sigma, np.float64), (n,)).copy(),
             epsilon=np.broadcast_to(np.asarray(epsilon, np.float64), (n,)).copy(),
             charge=np.broadcast_to(np.asarray(charge, np.float64), (n,)).copy(),
             kT=2.494, gamma=1.0, dt=0.001, t_gr=1, t_check_dephase=10, t_check_parallel=10,
             state=dict(kind=G.STATE_SIGN_X, atoms=[0]), obs=[])
    for k, v in kw.items():
        s[k] = v
    return s


def chain_terms(n):
    """Index lists of a linear chain of n atoms."""
    i = np.arange(n)
    return dict(bonds=np.stack([i[:-1], i[1:]], 1).astype(np.int32),
                angles=np.stack([i[:-2], i[1:-1], i[2:]], 1).astype(np.int32),
                torsions=np.stack([i[:-3], i[1:-2], i[2:-1], i[3:]], 1).astype(np.int32))


def gen_parrep_exits(sys, n_exits, t_corr):
    """Drives the Gen.ParRep loop of Fig. 1 (transient/decorrelation -> convergence ->
    parallel step) through a system object with the library's method names, and returns
    one record per exit event: (duration in steps since entering the state, from, to, how,
    tau_steps of the parallel step or 0)."""
    out = []
    last = sys.simulated_steps()
    omega = sys.current_state()
    while len(out) < n_exits:
        rc, ev = sys.decorrelate(t_corr)
        assert rc == 0
        if ev["kind"] == 1:
            now = sys.simulated_steps()
            out.append((now - last, ev["from_state"], ev["to_state"], "transient", 0))
            last, omega = now, ev["to_state"]
            continue
        rc, o = sys.dephase()
        assert rc == 0
        if o["outcome"] == 1:
            now = sys.simulated_steps()
            out.append((now - last, omega, o["to_state"], "dephase", 0))
            last, omega = now, o["to_state"]
            continue
        rc, e = sys.parallel_step()
        assert rc == 0
        now = sys.simulated_steps()
        out.append((now - last, omega, e["to_state"], "parallel", e["tau_steps"]))
        last, omega = now, e["to_state"]
    return out


def original_parrep_exits(sys, n_exits, t_corr, t_phase):
    """The original ParRep loop (Sec. 2.4.3): decorrelation with a fixed residence time
    t_corr, dephasing with a fixed time t_phase, then the parallel step; one record per exit
    as in gen_parrep_exits."""
    out = []
    last = sys.simulated_steps()
    omega = sys.current_state()
    while len(out) < n_exits:
        rc, ev = sys.decorrelate(t_corr)
        assert rc == 0
        if ev["kind"] == 1:
            now = sys.simulated_steps()
            out.append((now - last, ev["from_state"], ev["to_state"], "transient", 0))
            last, omega = now, ev["to_state"]
            continue
        rc, o = sys.dephase_fixed(t_phase)
        assert rc == 0 and o["outcome"] == 0
        rc, e = sys.parallel_step()
        assert rc == 0
        now = sys.simulated_steps()
        out.append((now - last, omega, e["to_state"], "parallel", e["tau_steps"]))
        last, omega = now, e["to_state"]
    return out


def direct_exits(sys, n_exits):
    """Brute-force direct simulation of the reference walker with the same exit-check
    period: decorrelation with an unbounded residence time never accepts a state, so
    every call returns at the next observed exit."""
    out = []
    last = sys.simulated_steps()
    while len(out) < n_exits:
        rc, ev = sys.decorrelate(1 << 62)
        assert rc == 0 and ev["kind"] == 1
        now = sys.simulated_steps()
        out.append((now - last, ev["from_state"], ev["to_state"], "direct", 0))
        last = now
    return out
