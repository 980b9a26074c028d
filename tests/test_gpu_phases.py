"""The phase-timer build of the library (libgpr_hip_probe.so: the same sources with the
persistent kernel's per-phase clocks) changes no result, and its timers add up: on the
300-atom receptor-ligand system (two workgroups per replica) the probe build's positions and
velocities after 120 steps are bit-identical to the product build's, every group counts every
step, and the summed phases of a launch stay within the kernel's own event timing.  The
product build refuses gpr_phase_read."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import gpr_synth as G

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, %(root)r)
import gpr_synth as G
import paper_1807_02431_amd.gpr as gb
gb.use_probe_library()
spec = G.config("rl300", n_replicas=8)
s = gb.System(spec, path=gb.PATH_PERSISTENT)
s.set_launch(0, 2)
s.profile(True)
s.advance(60, first_exit=False)
s.advance(60, first_exit=False)
kms, kn = s.profile_read()
ph = s.phase_read()
np.save(%(out)r, np.stack([np.concatenate([s.get_state(r)[0].ravel(), s.get_state(r)[1].ravel()]) for r in range(8)]))
np.save(%(ph)r, ph)
print(json.dumps({"kernel_ms": kms, "launches": kn}))
"""


def test_probe_build_same_results_and_timers_add_up(tmp_path):
    import paper_1807_02431_amd as gpr
    if not os.path.exists(gpr.gpr.PROBE_LIB_PATH):
        pytest.fail("libgpr_hip_probe.so is not built (__graft_entry__.build() builds it)")
    spec = G.config("rl300", n_replicas=8)
    s = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    s.set_launch(0, 2)
    s.advance(60, first_exit=False)
    s.advance(60, first_exit=False)
    ref = np.stack([np.concatenate([s.get_state(r)[0].ravel(), s.get_state(r)[1].ravel()]) for r in range(8)])
    with pytest.raises(gpr.GprError):
        s.phase_read()                                  # the product build has no timers

    out, phf = str(tmp_path / "state.npy"), str(tmp_path / "ph.npy")
    print("probe build, rl300 x 8, G = 2, two 60-step launches", flush=True)
    p = subprocess.run([sys.executable, "-c", _CHILD % dict(root=ROOT, out=out, ph=phf)],
                       capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-2000:]
    info = json.loads(p.stdout.strip().splitlines()[-1])
    got = np.load(out)
    assert np.array_equal(got, ref)
    ph = np.load(phf)                                   # [R, 8, 11]
    assert ph.shape == (8, 8, 11)
    assert np.all(ph[:, :2, 7] == 120) and np.all(ph[:, 2:, :] == 0)
    assert np.all(ph[:, :2, 8] >= 1)                    # the list is built at least once
    assert np.all(ph[:, :2, :7] >= 0)
    tot = ph[:, :2, :7].sum(axis=2)                     # µs per group over both launches
    kernel_us = 1000.0 * info["kernel_ms"]
    assert info["launches"] == 2
    # a group's phases lie inside its launches, and the slowest group fills most of them
    assert tot.max() <= kernel_us * 1.02 + 5.0, (tot.max(), kernel_us)
    assert tot.max() >= 0.5 * kernel_us, (tot.max(), kernel_us)
    # the last launch's start and end (µs after its earliest start) bound a 60-step launch
    st, en = ph[:, :2, 9], ph[:, :2, 10]
    assert st.min() == 0.0 and np.all(en > st)
    assert en.max() <= kernel_us, (en.max(), kernel_us)
