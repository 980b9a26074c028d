"""Pins of the oracle's random numbers: Philox4x32-10 and the Box-Muller Gaussians.

Philox is fixed by its published definition (Salmon et al., SC'11): the oracle must
reproduce the Random123 known-answer vectors and agree word for word with rocRAND's
independent implementation.  The Gaussians are pinned by their distribution.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle.philox(ctr, key) == out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(tmp_path):
    exe = tmp_path / "prc"
    src = os.path.join(os.path.dirname(__file__), "philox_rocrand_check.cpp")
    subprocess.check_call(["hipcc", "-O1", "-x", "hip", "--offload-host-only", "-I/opt/rocm/include",
                           src, "-o", str(exe)], cwd=str(tmp_path))
    rng = np.random.default_rng(7)
    words = rng.integers(0, 2 ** 32, size=(500, 6), dtype=np.uint64)
    inp = "\n".join(" ".join(str(int(x)) for x in row) for row in words) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(words, out):
        ref = [int(x) for x in line.split()]
        assert oracle.philox(row[:4], row[4:6]) == ref


def test_noise_counter_layout():
    # word layout of the noise counter: (atom, step lo, replica, stream << 24 | step hi)
    seed = 0x1234_5678_9ABC_DEF0
    step = (5 << 32) + 17
    w, _ = oracle.noise(seed, 3, step, 2, 4)
    for atom in range(4):
        ref = oracle.philox([atom, 17, 3, (2 << 24) | 5], [0x9ABCDEF0, 0x12345678])
        assert list(w[atom]) == ref


def test_uniforms_exact_in_binary32():
    # u = (2 (w >> 9) + 1) 2^-24 is an odd multiple of 2^-24 below 1: exact in float32
    w = np.array([0, 1, 511, 512, 2 ** 32 - 1, 123456789], dtype=np.uint64)
    u = (2.0 * (w >> 9) + 1.0) * 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert u.min() > 0 and u.max() < 1


def test_gaussians_standard_normal():
    _, g = oracle.noise(99, 0, 0, 0, 200000)
    for c in range(3):
        x = g[:, c]
        assert abs(x.mean()) < 5 * (1 / np.sqrt(len(x)))
        assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / len(x))
        assert stats.kstest(x, "norm").pvalue > 1e-3
    # the three components are uncorrelated
    cc = np.corrcoef(g.T)
    assert np.all(np.abs(cc[np.triu_indices(3, 1)]) < 0.02)


def test_gaussians_independent_across_replicas_and_steps():
    _, a = oracle.noise(5, 0, 0, 0, 50000)
    _, b = oracle.noise(5, 1, 0, 0, 50000)
    _, c = oracle.noise(5, 0, 1, 0, 50000)
    _, d = oracle.noise(5, 0, 0, 1, 50000)
    for x in (b, c, d):
        assert abs(np.corrcoef(a[:, 0], x[:, 0])[0, 1]) < 0.03
        assert not np.allclose(a, x)
