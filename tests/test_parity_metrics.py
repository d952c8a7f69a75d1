"""CPU pins of the parity tests' reach weights (tests/parity_metrics.py) on Kuhn, worked by hand."""
import numpy as np

import gamegen as gg
import oracle
from parity_metrics import rel_err, set_reach, slot_weights, weighted_err


def kuhn_reach(profile_of):
    g = gg.kuhn()
    o = oracle.Oracle(g)
    lay = o.layout()
    so = lay["slot_off"]
    prof = np.zeros(o.A)
    for i in range(o.I):
        prof[so[i]:so[i + 1]] = profile_of(i, so[i + 1] - so[i])
    return lay, set_reach(g, lay, prof)


def test_kuhn_uniform_reach_by_hand():
    """One deal node (six ordered deals, 1/6 each).  Player 1's first sets (one per card) hold two deals:
    reach 1/3.  Player 2's sets after a check (probability 1/2) hold two deals: 1/6; after a bet
    likewise 1/6.  Player 1's sets after check-bet: 1/3 * 1/2 * 1/2 = 1/12."""
    lay, r = kuhn_reach(lambda i, n: np.full(n, 1.0 / n))
    mo, mn, do = lay["mem_off"], lay["mem_node"], lay["depth_off"]
    depth = np.searchsorted(do, mn[mo[:-1]], side="right") - 1
    assert np.allclose(r[depth == 1], 1 / 3)
    assert np.allclose(r[depth == 2], 1 / 6)
    assert np.allclose(r[depth == 3], 1 / 12)
    assert r.size == 12


def test_kuhn_pure_profile_reach():
    """Always the first action (check, then check/call): player 2's sets after a bet are never reached."""
    lay, r = kuhn_reach(lambda i, n: np.eye(n)[0])
    mo, mn, do = lay["mem_off"], lay["mem_node"], lay["depth_off"]
    depth = np.searchsorted(do, mn[mo[:-1]], side="right") - 1
    assert np.allclose(r[depth == 1], 1 / 3)
    assert sorted(np.round(r[depth == 2], 12).tolist()) == [0.0] * 3 + [round(1 / 3, 12)] * 3
    assert np.allclose(r[depth == 3], 0.0)


def test_weighted_and_normwise_errors():
    lay, r = kuhn_reach(lambda i, n: np.full(n, 1.0 / n))
    w = slot_weights(lay, r)
    x = np.zeros(len(w))
    y = x.copy()
    y[0] = 0.5
    assert weighted_err(y, x, w) == 0.5 * w[0]
    assert rel_err(np.array([1.0, 2.0]), np.array([1.0, 4.0])) == 0.5
