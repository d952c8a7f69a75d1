"""GPU tests of the in-place re-solve (paper Appendix H, set_payoffs / set_root_chance / set_root_ranges; Table
'tab:lifecycle'): rewriting a compiled game's payoffs or root chance reproduces a fresh compile of
the changed game, without reallocating and with the captured graph still replaying."""
import dataclasses
import sys

import numpy as np
import pytest

import gamegen as gg
import oracle
import paper_2609_11923_amd as cfr

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(x, ref):
    return float(np.abs(np.asarray(x, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-30))


def specs(n, seed):
    out = []
    for sp in gg.random_subgames(n, seed, lo=1e3, hi=3e4):
        sp = dict(sp)
        sp.pop("target")
        out.append(sp)
    return out


def new_ranges(sp, seed):
    rng = np.random.default_rng(seed)
    sp = dict(sp)
    sp["r1"] = rng.dirichlet(np.ones(len(sp["hands1"])))
    sp["r2"] = rng.dirichlet(np.ones(len(sp["hands2"])))
    return sp


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("layout", ["public", "bfs"])
def test_set_root_ranges_equals_a_fresh_compile(precision, layout):
    """New ranges for every subgame of a batch, written after a solve whose graph was captured: a
    reset and a new solve then equal, bitwise, a batch compiled from the new subgames."""
    sps = specs(6, 2)
    games = [gg.subgame(**sp) for sp in sps]
    p = cfr.CFR_PRECISION_FP64 if precision == "fp64" else cfr.CFR_PRECISION_FP32
    lay = cfr.CFR_LAYOUT_PUBLIC if layout == "public" else cfr.CFR_LAYOUT_BFS
    s = cfr.Solver(games, precision=p, layout=lay, lifecycle=True)
    s.iterate(15)   # captures the graph
    sps2 = [new_ranges(sp, 10 + k) for k, sp in enumerate(sps)]
    games2 = [gg.subgame(**sp) for sp in sps2]
    for k, (g, sp) in enumerate(zip(games, sps2)):
        s.set_root_ranges(sp["r1"], sp["r2"], game=k)
    s.reset()
    s.iterate(40)
    t = cfr.Solver(games2, precision=p, layout=lay)
    t.iterate(40)
    assert np.array_equal(s.state()[0], t.state()[0]) and np.array_equal(s.state()[1], t.state()[1])
    assert np.array_equal(s.batch_exploitability()[0], t.batch_exploitability()[0])


def test_set_payoffs_equals_a_fresh_compile_on_subgames():
    sps = specs(4, 3)
    games = [gg.subgame(**sp) for sp in sps]
    s = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64, lifecycle=True)
    s.iterate(5)
    rng = np.random.default_rng(0)
    games2 = []
    for k, g in enumerate(games):
        pay = np.array(g.payoff, np.float64)
        term = np.asarray(g.type) == 3
        pay[term] = rng.uniform(-1, 1, int(term.sum()))
        games2.append(dataclasses.replace(g, payoff=pay))
        s.set_payoffs(pay, game=k)
    s.reset()
    s.iterate(30)
    t = cfr.Solver(games2, precision=cfr.CFR_PRECISION_FP64)
    t.iterate(30)
    assert np.array_equal(s.state()[0], t.state()[0])
    assert np.array_equal(s.batch_exploitability()[0], t.batch_exploitability()[0])


@pytest.mark.parametrize("name", ["leduc3x2", "random13"])
def test_set_payoffs_with_chance_below_the_root_matches_the_oracle(name):
    """Chance nodes below the root: the rewritten template groups the chance product as
    root * (rest), a compile multiplies along the path, so they agree to rounding; the solve
    matches the oracle of the changed game to the parity bar."""
    g = gg.leduc(3, 2) if name == "leduc3x2" else gg.random_game(13, 6, 6, 7, max_actions=5, max_chance=4)
    s = cfr.Solver(g, precision=cfr.CFR_PRECISION_FP64, lifecycle=True)
    s.iterate(10)
    rng = np.random.default_rng(1)
    pay = np.array(g.payoff, np.float64)
    term = np.asarray(g.type) == 3
    pay[term] = np.round(rng.uniform(-2, 2, int(term.sum())), 3)
    g2 = dataclasses.replace(g, payoff=pay)
    s.set_payoffs(pay)
    s.reset()
    s.iterate(100)
    o = oracle.Oracle(g2)
    o.iterate(100)
    Ro, _, _, sao = o.state()
    note(f"[lifecycle] {name}: R {rel_err(s.state()[0], Ro):.2e} avg {rel_err(s.strategy(average=True), sao):.2e}")
    assert rel_err(s.state()[0], Ro) <= 1e-5
    assert rel_err(s.strategy(average=True), sao) <= 1e-5
    assert abs(s.exploitability()[0] - o.exploitability()[0]) <= 1e-6 * g2.pot


def test_resolve_continues_from_the_previous_solution():
    """Without a reset the solver continues from its regrets and strategy sums under the new
    template; exploitability is measured against the new game."""
    sp = specs(1, 4)[0]
    g = gg.subgame(**sp)
    s = cfr.Solver(g, precision=cfr.CFR_PRECISION_FP64, lifecycle=True)
    s.iterate(300)
    sp2 = new_ranges(sp, 7)
    s.set_root_ranges(sp2["r1"], sp2["r2"])
    e_before = s.exploitability()[0]
    _, S_before = s.state()
    s.iterate(300)
    e_after = s.exploitability()[0]
    note(f"[lifecycle] re-solve from the old solution: expl {e_before:.3e} -> {e_after:.3e}")
    # the state was kept (the counter continues; linear averaging still weighs the first 300
    # iterations by about a quarter, so the average is biased toward the old game)
    assert s.iterations == 600 and S_before.sum() > 0
    assert e_after < 0.5 * e_before


def test_lifecycle_errors():
    g = gg.kuhn()
    s = cfr.Solver(g)
    with pytest.raises(cfr.CfrError) as e:
        s.set_payoffs(np.asarray(g.payoff))
    assert e.value.status == cfr.CFR_ESTATE
    s = cfr.Solver(g, lifecycle=True)
    with pytest.raises(cfr.CfrError) as e:
        s.set_payoffs(np.asarray(g.payoff)[:-1])
    assert e.value.status == cfr.CFR_EINVAL
    with pytest.raises(cfr.CfrError) as e:
        s.set_root_chance(np.full(6, 0.2))
    assert e.value.status == cfr.CFR_EINVAL
    with pytest.raises(cfr.CfrError) as e:
        s.set_root_chance(np.full(6, 1 / 6), game=1)
    assert e.value.status == cfr.CFR_EINVAL
    d = cfr.Solver(gg.degenerate("single_action"), lifecycle=True)
    with pytest.raises(cfr.CfrError) as e:
        d.set_root_chance(np.ones(1))
    assert e.value.status == cfr.CFR_EINVAL and "chance" in str(e.value)


def test_set_root_ranges_errors():
    g = gg.kuhn()   # a sequential deal: no joint-deal hand map at the root
    s = cfr.Solver(g, lifecycle=True)
    with pytest.raises(cfr.CfrError) as e:
        s.set_root_ranges(np.ones(3), np.ones(3))
    assert e.value.status == cfr.CFR_ESTATE
    sp = specs(1, 5)[0]
    sub = gg.subgame(**sp)
    t = cfr.Solver(sub)   # no lifecycle records
    with pytest.raises(cfr.CfrError) as e:
        t.set_root_ranges(sp["r1"], sp["r2"])
    assert e.value.status == cfr.CFR_ESTATE
    u = cfr.Solver(sub, lifecycle=True)
    n1, n2 = len(sp["hands1"]), len(sp["hands2"])
    for r1, r2 in ((np.ones(n1 + 1), np.ones(n2)), (np.zeros(n1), np.ones(n2)), (np.full(n1, -1.0), np.ones(n2)),
                   (np.full(n1, np.nan), np.ones(n2))):
        with pytest.raises(cfr.CfrError) as e:
            u.set_root_ranges(r1, r2)
        assert e.value.status == cfr.CFR_EINVAL
    u.set_root_ranges(np.ones(n1), np.ones(n2))   # uniform ranges are valid
