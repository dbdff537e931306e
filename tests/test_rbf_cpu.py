"""Host checks of the RBF shape-parameter search (pdd_rbf_shape, no GPU)
against the oracle's own search, and of its argument checks."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd
from oracle.rbf import shape_for_condition, condition


@pytest.mark.parametrize("S,d,target", [(17, 1 / 16, 1e6), (33, 1 / 128, 1e10), (65, 1 / 1024, 1e10),
                                        (129, 200 / 640, 1e10), (5, 2.0, 1e3)])
def test_shape_matches_the_oracle(S, d, target):
    c = pdd.rbf_shape(S, d, target)
    assert c == pytest.approx(shape_for_condition(S, d, target), rel=1e-6)
    assert condition(np.arange(S) * d, c) == pytest.approx(target, rel=1e-4)


def test_shape_scales_with_the_spacing():
    """Phi(c; d) = Phi(c/d; 1) / d: the condition number depends on c/d only."""
    a = pdd.rbf_shape(33, 1.0, 1e8)
    b = pdd.rbf_shape(33, 1 / 64, 1e8)
    assert b == pytest.approx(a / 64, rel=1e-8)


@pytest.mark.parametrize("args", [(1, 0.1, 1e10), (257, 0.1, 1e10), (17, 0.0, 1e10), (17, -1.0, 1e10),
                                  (17, float("nan"), 1e10), (17, 0.1, 0.5), (17, 0.1, 1e40)])
def test_shape_rejects_bad_arguments(args):
    with pytest.raises(pdd.PddError) as e:
        pdd.rbf_shape(*args)
    assert e.value.status == pdd.EINVAL
