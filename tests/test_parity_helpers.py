"""CPU checks of the parity helpers the GPU tests rely on: the validity test
of a replayed cardinality support and of a replayed CG stopping decision."""
import numpy as np

from oracle import parsdmm as orc
from tests import gpu_util as gu


def test_support_report_accepts_tie_choices_and_rejects_wrong_ones():
    w = np.array([5.0, -3.0, 3.0, 1.0, -0.5, 3.0])
    # k = 3: 5 and two of the three entries of magnitude 3
    ok, ndiff, _ = gu.support_report(w, np.array([0, 1, 2]), 3)
    assert ok and ndiff == 0                       # the oracle's own choice (lower indices)
    ok, ndiff, dist = gu.support_report(w, np.array([0, 2, 5]), 3)
    assert ok and ndiff == 2 and dist == 0.0       # another tie choice
    ok, _, _ = gu.support_report(w, np.array([0, 1, 3]), 3)
    assert not ok                                  # keeps 1 while dropping a 3
    ok, _, _ = gu.support_report(w, np.array([0, 1]), 3)
    assert not ok                                  # too few while nonzeros were dropped
    z = np.array([2.0, 0.0, 0.0, 1.0])
    ok, _, _ = gu.support_report(z, np.array([0, 3]), 3)
    assert ok                                      # the third kept entry is an exact zero


def test_support_report_band():
    w = np.array([1.0, 0.99999, 0.5])
    ok, ndiff, dist = gu.support_report(w, np.array([1]), 1)
    assert ok and ndiff == 2 and 0 < dist <= gu.CARD_BAND    # within the tie band
    w = np.array([1.0, 0.9, 0.5])
    ok, _, _ = gu.support_report(w, np.array([1]), 1)
    assert not ok


def test_band_mask():
    w = np.array([4.0, -2.0, 2.0000001, 1.0, 3.0])
    mask = gu.band_mask(w, 3)                      # t_k = 2
    assert list(mask) == [True, False, False, True, True]


def test_cg_decision_ok():
    tr = [1.0, 0.5, 0.2, 0.09, 0.05]
    assert gu.cg_decision_ok(tr, 3, 0.1, 10)
    assert not gu.cg_decision_ok(tr, 2, 0.1, 10)   # stopped while still above cg_rel
    assert not gu.cg_decision_ok(tr, 4, 0.1, 10)   # ran past the first step below
    assert gu.cg_decision_ok([1.0, 0.5, 0.1000001, 0.05], 2, 0.1, 10)  # boundary within the band
    assert gu.cg_decision_ok([1.0, 0.5, 0.3], 2, 0.1, 2)               # the cap


def test_oracle_own_support_passes():
    rng = np.random.default_rng(1)
    w = rng.standard_normal(200)
    keep = orc.card_support(w, 17)
    ok, ndiff, _ = gu.support_report(w, keep, 17)
    assert ok and ndiff == 0


def test_cg_decision_when_the_oracle_reaches_zero_residual():
    assert gu.cg_decision_ok([1.0, 0.3, 0.0], 4, 0.1, 10)
    assert not gu.cg_decision_ok([1.0, 0.3], 4, 0.1, 10)
