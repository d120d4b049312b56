"""The per-launch timing of lc_set_timing / lc_get_timing, which the
benchmark reads: every timed launch is counted once (also past the point
where the context folds its recorded events into running sums), the sums
are reset by each read, nothing is recorded while timing is off, and timing
does not change the results."""
import sys

import numpy as np
import pytest

from paper_1907_13415_amd import inputs
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

PARAMS = (1.0, 2.72, 0.05, 0.3, 0.7, 1.3)


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _solver(lc, shape, variant, seed):
    rng = np.random.default_rng(seed)
    s = lc.Solver("D3Q19", "fp32dev", shape, PARAMS)
    s.set_variant(variant)
    s.load(inputs.random_q5(shape, rng, amp=0.1))
    return s


@pytest.mark.parametrize("variant,kinds", [(2, (1, 1)), (3, (1, 0))])
def test_timed_launches_are_counted_past_the_fold(variant, kinds):
    """1500 steps record 1500 launches of each timed kind (3000 for the two
    sweeps, beyond the 1024 the context holds before folding)."""
    require_gpu()
    from paper_1907_13415_amd import lc
    _say("timing, variant %d" % variant)
    s = _solver(lc, (8, 10, 12), variant, 70)
    lc.lc_set_timing(s.ctx, True)
    s.step(1500)
    ms, n = lc.lc_get_timing(s.ctx)
    _say("launches %s, ms %s" % (n, ms))
    assert n == [1500 * k for k in kinds]
    for k in range(2):
        assert (ms[k] > 0) == (kinds[k] == 1)
        # a launch of this grid takes well under a millisecond
        assert ms[k] < 1500.0
    # the read resets the sums
    ms2, n2 = lc.lc_get_timing(s.ctx)
    assert n2 == [0, 0] and ms2 == [0.0, 0.0]
    # nothing is recorded with timing off
    lc.lc_set_timing(s.ctx, False)
    s.step(10)
    ms3, n3 = lc.lc_get_timing(s.ctx)
    assert n3 == [0, 0] and ms3 == [0.0, 0.0]


def test_timing_does_not_change_the_result():
    require_gpu()
    from paper_1907_13415_amd import lc
    out = []
    for timed in (False, True):
        s = _solver(lc, (9, 11, 13), 2, 71)
        lc.lc_set_timing(s.ctx, timed)
        s.step(20)
        out.append((s.export(lc.LC_FIELD_F), s.export(lc.LC_FIELD_Q)))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
