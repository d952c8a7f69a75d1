"""GPU tests of the LDS-resident schedule for tiny standalone games: one workgroup runs whole
iterations with the game's state in LDS (no launch per level), which removes the per-iteration
launch floor that small games cannot fill (paper Sec. Results, cross-framework timing).  The
arithmetic and its order are those of the level launches, so the iterates must be bitwise equal;
against the oracle the usual parity bar applies."""
import dataclasses
import sys

import numpy as np
import pytest

import gamegen as gg
import oracle
import paper_2609_11923_amd as cfr

pytestmark = pytest.mark.gpu

PREC = {"fp64": cfr.CFR_PRECISION_FP64, "fp32": cfr.CFR_PRECISION_FP32}
RULES = {"cfr+": (cfr.CFR_RULE_CFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS),
         "cfr": (cfr.CFR_RULE_CFR, cfr.CFR_ORDER_SIMULTANEOUS),
         "dcfr-alt": (cfr.CFR_RULE_DCFR, cfr.CFR_ORDER_ALTERNATING),
         "pcfr+": (cfr.CFR_RULE_PCFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS),
         "cfr+-alt": (cfr.CFR_RULE_CFR_PLUS, cfr.CFR_ORDER_ALTERNATING)}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def jitter(game, seed, eps=1e-3):
    rng = np.random.default_rng(seed)
    pay = np.array(game.payoff, np.float64)
    term = np.asarray(game.type) == 3
    pay[term] += eps * rng.uniform(-1, 1, int(term.sum()))
    return dataclasses.replace(game, payoff=pay)


GAMES = {
    "kuhn": lambda: gg.kuhn(),
    "random7": lambda: gg.random_game(7, 4, 3, 6),
    "random_wide": lambda: gg.random_game(21, 5, 4, 5, max_actions=8, max_chance=3),
}


def pair(game, precision, rule, **kw):
    r, o = RULES[rule]
    a = cfr.Solver(game, rule=r, order=o, precision=PREC[precision], persistent=cfr.CFR_SCHEDULE_LDS, **kw)
    b = cfr.Solver(game, rule=r, order=o, precision=PREC[precision], **kw)
    return a, b


def same_state(a, b):
    Ra, Sa = a.state()
    Rb, Sb = b.state()
    return np.array_equal(Ra, Rb) and np.array_equal(Sa, Sb) and np.array_equal(a.strategy(), b.strategy())


@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("precision", list(PREC))
@pytest.mark.parametrize("name", list(GAMES))
def test_lds_schedule_equals_level_launches(name, precision, rule):
    game = GAMES[name]()
    note(f"[lds] {name} {precision} {rule}")
    a, b = pair(game, precision, rule)
    for n in (1, 7, 30, 7):   # a new n captures a new graph; the counter carries over
        a.iterate(n)
        b.iterate(n)
    assert a.iterations == b.iterations == 45
    assert same_state(a, b)
    assert a.exploitability() == b.exploitability()


@pytest.mark.parametrize("layout", ["public", "bfs"])
def test_lds_schedule_direct_launches_and_layouts(layout):
    lay = cfr.CFR_LAYOUT_PUBLIC if layout == "public" else cfr.CFR_LAYOUT_BFS
    game = gg.random_game(7, 4, 3, 6)
    a, b = pair(game, "fp64", "cfr+", layout=lay, use_graph=False)
    a.iterate(23)
    b.iterate(23)
    assert same_state(a, b)


def test_lds_schedule_leduc_fp32_when_it_fits():
    """Leduc with 3 ranks (9,457 nodes) needs about 146 KiB in FP32: it runs when the device gives a
    workgroup that much LDS, and is refused with a clear error otherwise."""
    game = gg.leduc(3, 2)
    try:
        a, b = pair(game, "fp32", "cfr+")
    except cfr.CfrError as e:
        assert e.status == cfr.CFR_EINVAL and "LDS" in str(e)
        pytest.skip(f"device LDS per workgroup too small: {e}")
    a.iterate(20)
    b.iterate(20)
    assert same_state(a, b)


def test_lds_schedule_parity_with_the_oracle():
    g = jitter(gg.kuhn(), 1)
    s = cfr.Solver(g, precision=cfr.CFR_PRECISION_FP64, persistent=cfr.CFR_SCHEDULE_LDS)
    s.iterate(100)
    o = oracle.Oracle(g)
    o.iterate(100)
    Ro, _, _, sao = o.state()
    R = s.state()[0]
    eR = np.abs(R - Ro).max() / np.abs(Ro).max()
    eavg = np.abs(s.strategy(average=True) - sao).max() / np.abs(sao).max()
    note(f"[lds] kuhn parity: R {eR:.2e} avg {eavg:.2e}")
    assert eR <= 1e-5 and eavg <= 1e-5
    assert abs(s.exploitability()[0] - o.exploitability()[0]) <= 1e-6 * g.pot


def test_switching_schedules_keeps_the_state():
    game = gg.random_game(7, 4, 3, 6)
    a = cfr.Solver(game, precision=cfr.CFR_PRECISION_FP64)
    b = cfr.Solver(game, precision=cfr.CFR_PRECISION_FP64)
    a.iterate(10)
    a.set_schedule(cfr.CFR_SCHEDULE_LDS)
    a.iterate(10)
    a.set_schedule(cfr.CFR_SCHEDULE_LEVEL)
    a.iterate(5)
    b.iterate(25)
    assert same_state(a, b)


def test_lds_schedule_refusals():
    big = gg.leduc(13, 2)
    with pytest.raises(cfr.CfrError) as e:
        cfr.Solver(big, persistent=cfr.CFR_SCHEDULE_LDS)
    assert e.value.status == cfr.CFR_EINVAL and "LDS" in str(e.value)
    batch = [gg.kuhn(), gg.kuhn()]
    with pytest.raises(cfr.CfrError) as e:
        cfr.Solver(batch, persistent=cfr.CFR_SCHEDULE_LDS)
    assert e.value.status == cfr.CFR_EINVAL and "batch" in str(e.value)
    s = cfr.Solver(big)
    with pytest.raises(cfr.CfrError):
        s.set_schedule(cfr.CFR_SCHEDULE_LDS)
    s.iterate(2)   # the level schedule stays in place
    with pytest.raises(cfr.CfrError) as e:
        cfr.Solver(gg.kuhn(), persistent=3)
    assert e.value.status == cfr.CFR_EINVAL


def test_autotune_picks_the_lds_schedule_for_kuhn():
    s = cfr.Solver(gg.kuhn())
    r = s.autotune(50)
    note(f"[lds] autotune on kuhn: {r}")
    assert r["persistent"] == cfr.CFR_SCHEDULE_LDS and r["blocks"] == 1
    s.iterate(10)
    t = cfr.Solver(gg.kuhn())
    t.iterate(10)
    assert same_state(s, t)
