"""Pins of the oracle's Algorithm 2 (TT-ICE*, Sec. 3.3) on designed
increments with closed-form outcomes (tests/star_designs.py).

Each expected value below is worked out by hand from the design's norms:
the relative errors of eq:relerror, the relaxed tolerance of
eq:epsilonmodification and the SVD truncation parameter eps_upd ||D|| /
sqrt(d), the two skip rules (the mean of eq:relerror and
eq:batchrelativeerror), and the occupancy test of eq:coreoccupancy (">= tau"
in Algorithm 2).  Beside them, the error of the increment after the update
is measured by brute-force reconstruction and compared with the guarantee
the relaxed tolerance is derived for (the total error of the increment stays
within eps_des ||Y||)."""
import math

import numpy as np
import pytest

from oracle import TTICE
from star_designs import batch_rule_design, dc_share_design, occupancy_design


def _run(design, **kw):
    dims, eps, first, second = design
    o = TTICE(dims, eps, algo="star", **kw)
    o.update(first)
    assert o.ranks == [1, 1, 1]
    info = o.update(second)
    err2 = float(np.sum((second - o.reconstruct(1, second.shape[0])) ** 2))
    return o, info, err2


# Hand values of the D_C design (d = 2, eps = 0.1):
#   ||Y||^2 = 100 + 0.39 = 100.39, ||D||^2 = 0.39, error of D_C = 0.81
#   eps_upd^2 = (0.01 * 100.39 - 0.81) / 0.39 = 0.1939 / 0.39
#   eps_core^2 = eps_upd^2 ||D||^2 / 2 = 0.09695
# Level 1: the residual of D is D itself (orthogonal to e_1) with energies
# 0.3 and 0.09; 0.09 <= 0.09695 < 0.39, so one direction (e_2) is appended.
# Level 2: the new coefficients s_1 f_2 are orthogonal to the padded f_1, with
# energy 0.3 > 0.09695: one direction.  Ranks [1, 2, 2, 1].
# Error of the increment afterwards: 0.81 (frame 0's e_3 part) + 0.09 (frame
# 1's e_4 part) = 0.90 <= eps^2 ||Y||^2 = 1.0039.
DC_EPS_UPD2 = 0.1939 / 0.39
DC_EPS_CORE2 = 0.09695


@pytest.mark.parametrize("rule", ["mean", "batch", "none"])
def test_relaxed_tolerance_counts_the_discarded_frames_error(rule):
    """eq:epsilonmodification with a D_C frame of large norm share and
    relative error just under eps, and ||D|| << ||Y||."""
    o, info, err2 = _run(dc_share_design(), skip_rule=rule)
    assert info["rel_err_old"] == pytest.approx([0.09, 1.0], rel=1e-12)
    assert not info["skipped"] and info["used"] == 1
    assert info["eps_upd"] ** 2 == pytest.approx(DC_EPS_UPD2, rel=1e-12)
    assert info["eps_core"] ** 2 == pytest.approx(DC_EPS_CORE2, rel=1e-12)
    assert info["rR"] == [1, 1]
    assert o.ranks == [1, 2, 2]
    assert err2 == pytest.approx(0.90, rel=1e-12)
    assert err2 <= 0.01 * 100.39


def test_relaxed_tolerance_keeps_the_increment_within_eps():
    """The guarantee eq:epsilonmodification is derived for: with every
    frame's residual discarded or kept as the relaxed tolerance says, the
    increment's error stays within eps_des ||Y|| (brute force), and the
    slack left is exactly the energy of the directions not appended."""
    dims, eps, first, second = dc_share_design(seed=7)
    o, info, err2 = _run((dims, eps, first, second))
    ny2 = float(np.sum(second ** 2))
    assert err2 <= eps ** 2 * ny2
    assert eps ** 2 * ny2 - err2 == pytest.approx(1.0039 - 0.90, rel=1e-9)


# Hand values of the batch-rule design (eps = 0.1): relative errors 0.05 and
# 1, mean 0.525 > eps; eq:batchrelativeerror sqrt((0.25 + 0.01) / 100.01)
# = 0.05099 <= eps.

def test_batch_rule_skips_where_the_mean_rule_does_not():
    o, info, err2 = _run(batch_rule_design(), skip_rule="batch")
    assert info["rel_err_old"] == pytest.approx([0.05, 1.0], rel=1e-12)
    assert info["skipped"] and info["used"] == 0
    assert o.ranks == [1, 1, 1]
    # the skipped increment is stored with the old cores: its error is the
    # batch relative error's numerator, and within eps (the rule's guarantee)
    assert err2 == pytest.approx(0.26, rel=1e-12)
    assert math.sqrt(err2 / 100.01) == pytest.approx(0.050987, rel=1e-4)


def test_mean_rule_updates_on_the_batch_rule_design():
    """The mean rule (Algorithm 2) does not skip: D = {frame 1}, and
    eps_upd^2 = (0.01 * 100.01 - 0.25) / 0.01 = 75.01, so eps_core^2 =
    75.01 * 0.01 / 2 = 0.37505 exceeds frame 1's residual energy 0.01 at
    every core: no direction is appended."""
    o, info, err2 = _run(batch_rule_design(), skip_rule="mean")
    assert not info["skipped"] and info["used"] == 1
    assert info["eps_upd"] ** 2 == pytest.approx(75.01, rel=1e-12)
    assert info["eps_core"] ** 2 == pytest.approx(0.37505, rel=1e-12)
    assert o.ranks == [1, 1, 1]
    assert err2 == pytest.approx(0.26, rel=1e-12)


# Occupancy design: core 1 holds 4 of its 5 possible directions, occupancy
# exactly 4/5 = tau = 0.8.

def test_occupancy_at_exactly_tau_skips_the_core():
    """Algorithm 2 leaves a core whose occupancy is >= tau (eq:coreoccupancy):
    at exactly 0.8 core 1 is not updated, so the tensor outside its span
    adds no direction anywhere (core 2 sees zero coefficients)."""
    dims, eps, first, second = occupancy_design()
    o = TTICE(dims, eps, algo="star", tau=0.8)
    o.update(first)
    assert o.ranks == [1, 4, 4]
    info = o.update(second)
    assert not info["skipped"] and info["used"] == 1
    assert info["occupancy_skip"] == [True, False]
    assert o.ranks == [1, 4, 4]
    # the whole tensor is lost: its error equals its norm
    err2 = float(np.sum((second - o.reconstruct(4, 1)) ** 2))
    assert err2 == pytest.approx(1.0, rel=1e-12)


def test_occupancy_below_tau_updates_the_core():
    """The same stream with tau just above 0.8 updates core 1 (5 of 5
    directions) and core 2, and stores the tensor exactly."""
    dims, eps, first, second = occupancy_design()
    o = TTICE(dims, eps, algo="star", tau=0.8000001)
    o.update(first)
    info = o.update(second)
    assert info["occupancy_skip"] == [False, False]
    assert o.ranks == [1, 5, 5]
    np.testing.assert_allclose(o.reconstruct(4, 1), second, atol=1e-14)
