"""The allocation-free entry point lbm_coexistence_many_noalloc against
lbm_coexistence_many: bit for bit the same densities and statuses, on two
calls in a row (the second with fewer runs, so it runs on what the first
left in the library's fixed array), and its size limit."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_11792_amd import lbm as mod

    return mod


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y), equal_nan=True), (x, y)


def test_noalloc_matches_allocating_variant(lbm):
    G1 = [-5.5, -5.5, -5.3, -7.5, -6.0, -5.8]
    t1 = [1.0, 0.8, 0.6241, 0.5001, 1.2, 0.9]   # the 0.5001 run diverges
    first = lbm.lbm_coexistence_many_noalloc(G1, t1)
    _same(first, lbm.lbm_coexistence_many(G1, t1))
    assert first[2][3] == lbm.LBM_ERR_DIVERGED and math.isnan(first[0][3])
    G2, t2 = [-5.2, -6.0], [0.95, 0.75]
    second = lbm.lbm_coexistence_many_noalloc(G2, t2)
    _same(second, lbm.lbm_coexistence_many(G2, t2))
    assert list(second[2]) == [lbm.LBM_OK, lbm.LBM_OK]
    mrt = dict(lbm.MRT_DEFAULT)
    _same(lbm.lbm_coexistence_many_noalloc([-5.5], [0.9], mrt=mrt),
          lbm.lbm_coexistence_many([-5.5], [0.9], mrt=mrt))


def test_noalloc_rejects_too_many_runs(lbm):
    n = lbm.LBM_NOALLOC_MAX_RUNS + 1
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_coexistence_many_noalloc([-5.5] * n, [1.0] * n)
    assert e.value.status == lbm.LBM_ERR_INVALID_ARG
    full = lbm.LBM_NOALLOC_MAX_RUNS
    rl, rv, st = lbm.lbm_coexistence_many_noalloc([-5.5] * full, [1.0] * full)
    assert np.all(st == lbm.LBM_OK) and np.all(rl == rl[0]) and np.all(rv == rv[0])
