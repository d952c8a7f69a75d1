"""GPU parity of the update rules and orders (paper Sec. 6, update rule and update order): CFR, CFR+,
DCFR and PCFR+, simultaneous and alternating, against the FP64 oracle's same rule after 100
free-running iterations, by the rule of free_run_compare (tests/parity_metrics.py): the method's bar
where the rule's own dynamics keep runs of one precision together, tolerances from the measured spread
of the oracle's own runs (kept below 1e-3, exploitability below 1e-5 pot) where they amplify rounding,
and an expected failure with the measured spread where they amplify it beyond that.  Some rules do:
the clamp and the discount switch on signs, and alternating updates feed one player's change straight
into the other's half.  Every cell is held to the 1e-5 bar at each of its 100 iterations by the
one-step test (tests/test_gpu_step_parity.py)."""
import sys

import numpy as np
import pytest

import gamegen as gg
import oracle
import paper_2609_11923_amd as cfr
from parity_metrics import CAP, MULT, free_run_compare, jitter, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-5
RULES = {"cfr": cfr.CFR_RULE_CFR, "cfr+": cfr.CFR_RULE_CFR_PLUS, "dcfr": cfr.CFR_RULE_DCFR,
         "pcfr+": cfr.CFR_RULE_PCFR_PLUS}
ORDERS = {"sim": cfr.CFR_ORDER_SIMULTANEOUS, "alt": cfr.CFR_ORDER_ALTERNATING}
PREC = {"fp64": cfr.CFR_PRECISION_FP64, "fp32": cfr.CFR_PRECISION_FP32}

# Kuhn and Leduc have exact symmetries that park some regrets exactly at zero, where regret matching
# (plus) switches between uniform and pure on the last bit (test_alternating_kuhn_divergence_is_the_
# discontinuity); generic payoffs (moved by up to 1e-3) avoid those ties.
GAMES = {
    "kuhn": lambda: jitter(gg.kuhn(), 1),
    "leduc3x2": lambda: jitter(gg.leduc(3, 2), 2),
    "random7": lambda: gg.random_game(7, 4, 3, 6),
    "random13": lambda: gg.random_game(13, 6, 6, 7, max_actions=5, max_chance=4),
}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver(game, rule, order, precision="fp64", **kw):
    return cfr.Solver(game, rule=RULES[rule], order=ORDERS[order], precision=PREC[precision], **kw)


def ref(game, rule, order, T, f32_state=False, reverse=False):
    o = oracle.Oracle(game, alternating=(order == "alt"), rule=rule, f32_state=f32_state, reverse=reverse)
    o.iterate(T)
    return o


def control_run(rule, order, T):
    def run(g, f32_state, reverse):
        return ref(g, rule, order, T, f32_state, reverse)
    return run


def compare(game, rule, order, precision, s, o, T):
    """Free-run comparison (free_run_compare in tests/parity_metrics.py); these games have generic
    payoffs, so the spread also samples payoffs moved at the rounding level."""
    free_run_compare(game, s, o, T, precision, control_run(rule, order, T), True, True, note)
    if rule in ("cfr+", "pcfr+"):
        assert (s.state()[0] >= 0).all()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(GAMES))
@pytest.mark.parametrize("order", list(ORDERS))
@pytest.mark.parametrize("rule", list(RULES))
def test_rule_parity(rule, order, name, precision):
    game = GAMES[name]()
    T = 100
    note(f"[rules] {rule} {order} {name} {precision}")
    s = solver(game, rule, order, precision)
    s.iterate(T)
    o = ref(game, rule, order, T)
    compare(game, rule, order, precision, s, o, T)


@pytest.mark.parametrize("rule,order", [("dcfr", "alt"), ("pcfr+", "sim"), ("pcfr+", "alt")])
def test_rule_parity_mid_game_full_size(rule, order):
    game = jitter(gg.leduc(13, 2), 3)
    note(f"[rules mid] {rule} {order}")
    s = solver(game, rule, order)
    s.iterate(100)
    o = ref(game, rule, order, 100)
    compare(game, rule, order, "fp64", s, o, 100)


def test_alternating_plan_has_two_halves():
    game = gg.leduc(3, 2)
    a = solver(game, "cfr+", "sim")
    b = solver(game, "cfr+", "alt")
    assert b.counts["kernels_per_iteration"] == 2 * a.counts["kernels_per_iteration"]


@pytest.mark.parametrize("rule,order", [("pcfr+", "sim"), ("dcfr", "alt"), ("pcfr+", "alt")])
def test_graph_equals_direct_and_reset_clears_the_prediction(rule, order):
    game = gg.random_game(7, 4, 3, 6)
    a = solver(game, rule, order)
    b = solver(game, rule, order, use_graph=False)
    a.iterate(30)
    b.iterate(30)
    assert np.array_equal(a.state()[0], b.state()[0]) and np.array_equal(a.state()[1], b.state()[1])
    a.reset()
    a.iterate(12)
    c = solver(game, rule, order)
    c.iterate(12)
    assert np.array_equal(a.state()[0], c.state()[0])
    assert np.array_equal(a.strategy(), c.strategy())


@pytest.mark.parametrize("rule,order", [("pcfr+", "alt"), ("dcfr", "sim")])
def test_persistent_and_batch_follow_the_rule(rule, order):
    """A batch under the persistent schedule reproduces the level launches bitwise, and each game
    matches its own oracle run."""
    games = [gg.subgame(**{k: v for k, v in sp.items() if k != "target"})
             for sp in gg.random_subgames(6, seed=4, lo=1e3, hi=2e4)] + [jitter(gg.leduc(3, 2), 4)]
    a = solver(games, rule, order, persistent=True, wg_nodes=4096)
    b = solver(games, rule, order)
    for n in (9, 31):
        a.iterate(n)
        b.iterate(n)
    Ra, Sa = a.state()
    assert np.array_equal(Ra, b.state()[0]) and np.array_equal(Sa, b.state()[1])
    base = b.slot_base
    avg = b.strategy(average=True)
    R = b.state()[0]
    for k, g in enumerate(games):
        o = ref(g, rule, order, 40)
        Ro, _, _, sao = o.state()
        c = ref(g, rule, order, 40, False, True)
        dR, davg = rel_err(c.state()[0], Ro), rel_err(c.state()[3], sao)
        tR, tavg = max(TOL, MULT * dR), max(TOL, MULT * davg)
        assert tR < CAP and tavg < CAP, k
        assert rel_err(R[base[k]:base[k + 1]], Ro) <= tR, k
        assert rel_err(avg[base[k]:base[k + 1]], sao) <= tavg, k


def test_unknown_rule_and_order_rejected():
    with pytest.raises(cfr.CfrError) as e:
        cfr.Solver(gg.kuhn(), rule=7)
    assert e.value.status == cfr.CFR_EINVAL
    with pytest.raises(cfr.CfrError) as e:
        cfr.Solver(gg.kuhn(), order=5)
    assert e.value.status == cfr.CFR_EINVAL


@pytest.mark.parametrize("rule", ["cfr+"])
def test_alternating_kuhn_divergence_is_the_discontinuity(rule):
    """On Kuhn itself (exact payoff symmetries), alternating CFR+ parts from the oracle.  The cause
    is classified, not waived: up to iteration 2 the regrets agree to rounding, and the current
    strategies differ only on sets whose regrets all sit at zero within rounding, where regret
    matching (plus) switches between uniform and a pure strategy on the sign of the last bit."""
    g = gg.kuhn()
    s = solver(g, rule, "alt")
    s.iterate(2)
    o = ref(g, rule, "alt", 2)
    R, _ = s.state()
    Ro, _, sco, _ = o.state()
    assert np.abs(R - Ro).max() <= 1e-12
    cur = s.strategy()
    so = o.layout()["slot_off"]
    at_zero, differ = [], []
    for i in range(len(so) - 1):
        sl = slice(so[i], so[i + 1])
        if np.abs(cur[sl] - sco[sl]).max() > 1e-6:
            differ.append(i)
        if np.abs(Ro[sl]).max() <= 1e-12 and np.abs(R[sl]).max() <= 1e-12:
            at_zero.append(i)
    note(f"[discontinuity] {rule}: strategies differ on sets {differ}; sets with all regrets at zero {at_zero}")
    assert set(differ) <= set(at_zero)

