"""The branching-plan entry point that allocates nothing (gpr_fv_plan_noalloc), through the
C ABI, against the allocating gpr_fv_plan: identical donors on two calls in a row, the second
with fewer replicas, and the size limit refused."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def test_fv_plan_noalloc_matches_allocating_entry_point():
    import paper_1807_02431_amd as gpr
    rng = np.random.default_rng(12)
    for R, p in ((5000, 0.3), (300, 0.6), (64, 1.0)):
        ex = (rng.random(R) < p).astype(np.uint8)
        step = int(rng.integers(0, 2 ** 40))
        print("noalloc plan R", R, flush=True)
        a = gpr.fv_plan(21, step, ex)
        b = gpr.fv_plan_noalloc(21, step, ex)
        assert np.array_equal(a, b), R
        assert np.array_equal(b, oracle.fv_plan(21, step, ex)), R
    big = np.zeros(gpr.NOALLOC_MAX_R + 1, np.uint8)
    with pytest.raises(gpr.GprError) as e:
        gpr.fv_plan_noalloc(21, 0, big)
    assert e.value.code == -1
    # the largest size passes
    ex = (rng.random(gpr.NOALLOC_MAX_R) < 0.5).astype(np.uint8)
    assert np.array_equal(gpr.fv_plan_noalloc(3, 77, ex), gpr.fv_plan(3, 77, ex))
