"""GPU tests of the affine child addressing of the update pass: in a public-state layout where child a
of every member h of an information set is h + offset(set, a), the fused backward/update level reads
one offset per slot instead of the explicit child list.  The arithmetic and its order are those of
the explicit path, so every iterate must be bitwise equal to it; a layout without the property
falls back to the child list by itself and keeps parity with the oracle."""
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
         "dcfr-alt": (cfr.CFR_RULE_DCFR, cfr.CFR_ORDER_ALTERNATING),
         "pcfr+": (cfr.CFR_RULE_PCFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS)}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def subgames(n, seed):
    return [gg.subgame(**{k: v for k, v in sp.items() if k != "target"})
            for sp in gg.random_subgames(n, seed=seed, lo=1e3, hi=3e4)]


GAMES = {
    "kuhn": lambda: gg.kuhn(),
    "leduc3x2": lambda: gg.leduc(3, 2),
    "leduc13x2": lambda: gg.leduc(13, 2),
    "random13": lambda: gg.random_game(13, 6, 6, 7, max_actions=5, max_chance=4),
    "random_wide": lambda: gg.random_game(21, 5, 4, 5, max_actions=8, max_chance=3),
    "subgames6": lambda: subgames(6, 5),
}


def run(game, precision, rule, affine, n=37, **kw):
    r, o = RULES[rule]
    s = cfr.Solver(game, rule=r, order=o, precision=PREC[precision], affine=affine, **kw)
    s.iterate(n)
    return s


@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("precision", list(PREC))
@pytest.mark.parametrize("name", list(GAMES))
def test_affine_equals_explicit_bitwise(name, precision, rule):
    game = GAMES[name]()
    note(f"[affine] {name} {precision} {rule}")
    a = run(game, precision, rule, True)
    b = run(game, precision, rule, False)
    assert a.counts["child_addressing"] == 2, "card-game layouts have per-slot child offsets"
    assert b.counts["child_addressing"] == 1
    Ra, Sa = a.state()
    Rb, Sb = b.state()
    assert np.array_equal(Ra, Rb) and np.array_equal(Sa, Sb)
    assert np.array_equal(a.strategy(), b.strategy())
    if isinstance(game, list):
        assert np.array_equal(a.batch_exploitability()[0], b.batch_exploitability()[0])
    else:
        assert a.exploitability() == b.exploitability()


@pytest.mark.parametrize("precision", list(PREC))
def test_affine_persistent_batch_equals_level_launches(precision):
    """The persistent kernel on the affine path reproduces the level launches bitwise (and the
    explicit path)."""
    games = subgames(9, 6) + [gg.leduc(3, 2)]
    a = cfr.Solver(games, precision=PREC[precision], persistent=True, wg_nodes=4096)
    b = cfr.Solver(games, precision=PREC[precision])
    c = cfr.Solver(games, precision=PREC[precision], persistent=True, wg_nodes=4096, affine=False)
    assert a.counts["child_addressing"] == 2 and c.counts["child_addressing"] == 1
    for n in (5, 28):
        a.iterate(n)
        b.iterate(n)
        c.iterate(n)
    for x in (b, c):
        assert np.array_equal(a.state()[0], x.state()[0]) and np.array_equal(a.state()[1], x.state()[1])


def test_layout_without_offsets_falls_back_to_the_child_list():
    """Every node its own public state: the public-state sort then leaves the members of a set and
    their children without a common offset, so the compile keeps the explicit child list; parity
    with the oracle still holds at the bar."""
    g = gg.leduc(3, 2)
    g2 = dataclasses.replace(g, pub=np.arange(len(g.type), dtype=np.int64)[::-1].copy())
    s = cfr.Solver(g2, precision=cfr.CFR_PRECISION_FP64)
    assert s.counts["child_addressing"] == 1
    s.iterate(100)
    o = oracle.Oracle(g)
    o.iterate(100)
    Ro, _, _, sao = o.state()
    R = s.state()[0]
    err = np.abs(R - Ro).max() / np.abs(Ro).max()
    eavg = np.abs(s.strategy(average=True) - sao).max() / np.abs(sao).max()
    note(f"[affine] fallback: R {err:.2e} avg {eavg:.2e}")
    assert err <= 1e-5 and eavg <= 1e-5
    assert abs(s.exploitability()[0] - o.exploitability()[0]) <= 1e-6 * g.pot


def test_bfs_layout_reports_implicit_children():
    s = cfr.Solver(gg.leduc(3, 2), layout=cfr.CFR_LAYOUT_BFS)
    assert s.counts["child_addressing"] == 0


@pytest.mark.parametrize("rule", ["cfr+", "dcfr-alt", "pcfr+"])
@pytest.mark.parametrize("precision", list(PREC))
def test_node_order_groups_equal_the_child_list_path(precision, rule):
    """Subgames with many hands per player: player-2 sets interleave inside a public-state block, so the
    compile lists some update groups' members in node order (with their set-major positions).  Those
    groups reproduce the explicit child-list path bitwise, under the level launches and the persistent
    launch."""
    games = [gg.subgame(**{k: v for k, v in sp.items() if k != "target"})
             for sp in gg.random_subgames(4, seed=8, lo=1e5, hi=3e5)]
    r, o = RULES[rule]
    a = cfr.Solver(games, rule=r, order=o, precision=PREC[precision])
    b = cfr.Solver(games, rule=r, order=o, precision=PREC[precision], affine=False)
    c = cfr.Solver(games, rule=r, order=o, precision=PREC[precision], persistent=True, wg_nodes=16384)
    note(f"[node order] {precision} {rule}: {a.counts['node_order_groups']} groups, "
         f"{a.counts['node_order_members']} members of {a.counts['decision_nodes']}")
    assert a.counts["node_order_groups"] > 0 and a.counts["node_order_members"] > 0
    assert b.counts["node_order_groups"] == 0
    for s in (a, b, c):
        s.iterate(23)
    Ra, Sa = a.state()
    for x in (b, c):
        Rx, Sx = x.state()
        assert np.array_equal(Ra, Rx) and np.array_equal(Sa, Sx)
    assert np.array_equal(a.batch_exploitability()[0], b.batch_exploitability()[0])


@pytest.mark.parametrize("precision", list(PREC))
@pytest.mark.parametrize("name", ["leduc13x2", "random_wide", "subgames6", "cards_k2"])
def test_group_set_bound_leaves_iterates_unchanged(name, precision):
    """Update groups hold at most 128 or 256 sets: chosen from the game's group counts under both
    bounds (128 unless it makes more than 30 % more groups), or forced.  The bound decides which
    workgroup updates a set and how much LDS the affine rows take, never a set's arithmetic, so every
    bound gives bitwise equal iterates, under the level launches and the persistent launch."""
    if name == "cards_k2":
        # two hands per player: about two members per set, so 128-set groups would split most groups
        h1, h2 = gg.sample_hands(2, 0)
        game = gg.large(2, seed=0, hands=(h1, h2))
    else:
        game = GAMES[name]()
    r, o = RULES["dcfr-alt"]
    sol = {}
    for gs in (0, 128, 256):
        sol[gs] = cfr.Solver(game, rule=r, order=o, precision=PREC[precision], group_sets=gs)
    c = {gs: s.counts for gs, s in sol.items()}
    note(f"[group sets] {name} {precision}: auto {c[0]['group_sets']}, groups {c[128]['update_groups']} "
         f"(128) / {c[256]['update_groups']} (256)")
    assert c[128]["group_sets"] == 128 and c[256]["group_sets"] == 256
    assert c[128]["update_groups"] >= c[256]["update_groups"]
    auto = 128 if c[128]["update_groups"] * 10 <= c[256]["update_groups"] * 13 else 256
    assert c[0]["group_sets"] == auto and c[0]["update_groups"] == c[auto]["update_groups"]
    if name == "cards_k2":
        assert auto == 256
    if name == "leduc13x2":
        assert auto == 128
    pers = {gs: cfr.Solver(game, rule=r, order=o, precision=PREC[precision], group_sets=gs, persistent=True,
                           wg_nodes=16384) for gs in (128, 256)}
    for s in list(sol.values()) + list(pers.values()):
        s.iterate(9)
    R0, S0 = sol[0].state()
    for s in [sol[128], sol[256], pers[128], pers[256]]:
        R, S = s.state()
        assert np.array_equal(R, R0) and np.array_equal(S, S0)
    for s in list(sol.values()) + list(pers.values()):
        s.close()
