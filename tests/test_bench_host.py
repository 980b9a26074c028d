"""Host logic of bench.py (CPU): the in-cutoff pair count behind the roofline's algorithmic
FLOP figure against a brute-force count, the stored HBM traffic figure offered only for the
kernel sources it was measured on (and interpolated between measured launch lengths), the
samples and checks counted in a timed window, and the one-GPU guard."""
import os
import subprocess
import sys

import numpy as np
import pytest

import gpr_synth as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _brute_pairs(spec, q):
    x = q.T
    skip = {(min(a, b), max(a, b)) for a, b in np.concatenate([spec["exclusions"], spec["pairs14"]])}
    n, rc2 = spec["n_atoms"], spec["cutoff"] ** 2
    total = 0
    for i in range(n):
        for j in range(i + 1, n):
            if ((x[i] - x[j]) ** 2).sum() < rc2 and (i, j) not in skip:
                total += 1
    return total


@pytest.mark.parametrize("name", ["rl300"])
def test_in_cutoff_pairs_matches_brute_force(name):
    spec = G.config(name, n_replicas=2)
    q = np.asarray(spec["pos"], dtype=np.float64)
    got = bench.in_cutoff_pairs(spec, q)
    assert got == _brute_pairs(spec, q)
    assert got > 0


def test_flop_count_adds_up():
    spec = G.config("rl300", n_replicas=2)
    base = bench.flops_per_replica_step(spec, 0)
    assert bench.flops_per_replica_step(spec, 1000) - base == 1000 * bench.FLOP_PAIR
    assert base == (len(spec["bonds"]) * bench.FLOP_BOND + len(spec["angles"]) * bench.FLOP_ANGLE
                    + len(spec["torsions"]) * bench.FLOP_TORSION + len(spec["restraints"]) * bench.FLOP_RESTRAINT
                    + len(spec["pairs14"]) * bench.FLOP_PAIR14 + spec["n_atoms"] * bench.FLOP_ATOM_BAOAB)


def test_traffic_only_for_the_profiled_kernel_sources(tmp_path, monkeypatch):
    """A stored per-launch figure is offered only for the kernel sources it was measured on;
    for a launch length it was measured at it is returned as stored, for another length from
    the straight line through the two nearest measured lengths, and with one length only for
    that length."""
    sha = bench.kernel_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    f = prof / "k_persist_rl2432x64_hbm_traffic.md"
    f.write_text("machine-readable:\nsource_sha256 %s\nhbm_bytes_per_launch_1000 12345\n" % sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: sha)
    assert bench.measured_traffic(1000) == 12345
    assert bench.measured_traffic(500) is None
    f.write_text("machine-readable:\nsource_sha256 %s\nhbm_bytes_per_launch_20 3000\n"
                 "hbm_bytes_per_launch_1000 101000\n" % sha)
    assert bench.measured_traffic(20) == 3000
    assert bench.measured_traffic(1000) == 101000
    assert bench.measured_traffic(500) == pytest.approx(3000 + 100 * 480)
    assert bench.measured_traffic(2000) == pytest.approx(3000 + 100 * 1980)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic(1000) is None


def test_window_counts():
    assert bench.window_counts(5, 25, 50, 1000) == dict(samples=0, checks=0)
    assert bench.window_counts(1000, 11000, 50, 1000) == dict(samples=200, checks=10)
    assert bench.window_counts(990, 1010, 50, 1000) == dict(samples=1, checks=1)


def test_kernel_hash_covers_sources_and_flags():
    """The hash is over every kernel source and the build script (its compiler flags)."""
    import glob
    import hashlib
    pkg = os.path.join(ROOT, "paper_1807_02431_amd")
    files = sorted(glob.glob(os.path.join(pkg, "csrc", "*")) + [os.path.join(pkg, "build.py")])
    assert any(f.endswith(".hip") for f in files)
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    assert bench.kernel_source_hash() == h.hexdigest()


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_oracle_on_all_cores_reports_an_aggregate():
    r = bench.cpu_baseline_all_cores(seconds=1.0, max_workers=2)
    assert r is not None and r["kind"] == "oracle" and r["unit"] == "replica-steps/s"
    assert 1 <= r["cores"] <= 2 and r["value"] > 0
