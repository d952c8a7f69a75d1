"""GPU tests of the batched form: many independent games (subgames with their own root ranges)
compiled into one handle and advanced together.  Each game is checked against its own FP64
oracle run (the same bar as single games), and a batch must reproduce, bitwise, what each game
gives when compiled alone (same kernels, same per-set reduction order)."""
import sys

import numpy as np
import pytest

import gamegen as gg
import oracle
import paper_2609_11923_amd as cfr

pytestmark = pytest.mark.gpu

TOL = 1e-5


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(x, ref):
    if ref.size == 0:
        return 0.0
    return float(np.abs(np.asarray(x, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-30))


def subgames(n, seed, lo=300.0, hi=3000.0):
    return [gg.subgame(**{k: v for k, v in spec.items() if k != "target"})
            for spec in gg.random_subgames(n, seed, lo=lo, hi=hi)]


def mixed_batch():
    return [gg.kuhn(), gg.leduc(3, 2), gg.random_game(7, 4, 3, 6), gg.example11(),
            gg.random_game(13, 6, 6, 7, max_actions=5, max_chance=4)] + subgames(6, seed=1)


@pytest.mark.parametrize("layout", ["public", "bfs"])
def test_batch_matches_oracle_per_game(layout):
    games = mixed_batch()
    note(f"[batch] {len(games)} games, nodes {[g.n_nodes for g in games]}")
    lay = cfr.CFR_LAYOUT_PUBLIC if layout == "public" else cfr.CFR_LAYOUT_BFS
    s = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64, layout=lay)
    assert s.n_games == len(games)
    T = 100
    s.iterate(T)
    R, S = s.state()
    avg = s.strategy(average=True)
    e, b1, b2, v = s.batch_exploitability()
    base = s.slot_base
    for k, g in enumerate(games):
        o = oracle.Oracle(g)
        o.iterate(T)
        Ro, _, _, sao = o.state()
        lo, hi = base[k], base[k + 1]
        assert hi - lo == o.A
        assert rel_err(R[lo:hi], Ro) <= TOL, k
        assert rel_err(avg[lo:hi], sao) <= TOL, k
        eo, _, _, vo = o.exploitability()
        assert abs(e[k] - eo) <= 1e-6 * g.pot, k
        assert abs(v[k] - vo) <= 1e-6 * g.pot, k


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_separate_solves_bitwise(precision):
    games = subgames(8, seed=3) + [gg.leduc(3, 2)]
    p = cfr.CFR_PRECISION_FP32 if precision == "fp32" else cfr.CFR_PRECISION_FP64
    b = cfr.Solver(games, precision=p)
    b.iterate(40)
    Rb, Sb = b.state()
    cur_b = b.strategy()
    eb = b.batch_exploitability()[0]
    base = b.slot_base
    for k, g in enumerate(games):
        s = cfr.Solver(g, precision=p)
        s.iterate(40)
        R, S = s.state()
        assert np.array_equal(R, Rb[base[k]:base[k + 1]]), k
        assert np.array_equal(S, Sb[base[k]:base[k + 1]]), k
        assert np.array_equal(s.strategy(), cur_b[base[k]:base[k + 1]]), k
        assert s.exploitability()[0] == pytest.approx(eb[k], abs=1e-12)


def test_batch_warm_start_and_reset():
    games = subgames(4, seed=5)
    s = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64)
    rng = np.random.default_rng(0)
    R0 = np.round(rng.random(s.A) * 2.0, 3).astype(np.float32)
    s.set_regrets(R0)
    s.iterate(30)
    R, _ = s.state()
    base = s.slot_base
    for k, g in enumerate(games):
        o = oracle.Oracle(g)
        o.set_state(R=R0[base[k]:base[k + 1]].astype(np.float64), sbar=np.zeros(o.A), t=0)
        o.iterate(30)
        assert rel_err(R[base[k]:base[k + 1]], o.state()[0]) <= TOL
    s.reset()
    s.iterate(10)
    t = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64)
    t.iterate(10)
    assert np.array_equal(s.state()[0], t.state()[0])


def test_batch_rejects_invalid_game_with_index():
    games = [gg.kuhn(), gg.from_arrays([0, 3, 3], [[1, 2], [], []], [[0.5, 0.6], None, None], [-1] * 3, [0, 1, 2])]
    with pytest.raises(cfr.CfrError) as e:
        cfr.Solver(games)
    assert e.value.status == cfr.CFR_EINVAL and "game 1" in str(e.value)


@pytest.mark.parametrize("wg_nodes", [1024, 4096, 1 << 20])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_persistent_equals_level_synchronous(wg_nodes, precision):
    """One persistent launch per call (per-game barriers between levels; small wg_nodes gives each game
    several workgroups) reproduces the level-synchronous launches bitwise."""
    games = subgames(12, seed=7, lo=1e3, hi=3e4) + [gg.leduc(3, 2)]
    p = cfr.CFR_PRECISION_FP32 if precision == "fp32" else cfr.CFR_PRECISION_FP64
    note(f"[persistent] {len(games)} games, {sum(g.n_nodes for g in games)} nodes, wg_nodes={wg_nodes}")
    a = cfr.Solver(games, precision=p, persistent=True, wg_nodes=wg_nodes)
    b = cfr.Solver(games, precision=p)
    for n in (7, 25):
        a.iterate(n)
        b.iterate(n)
    assert a.iterations == b.iterations == 32
    Ra, Sa = a.state()
    Rb, Sb = b.state()
    assert np.array_equal(Ra, Rb) and np.array_equal(Sa, Sb)
    assert np.array_equal(a.strategy(), b.strategy())
    assert np.array_equal(a.batch_exploitability()[0], b.batch_exploitability()[0])


def test_persistent_single_game():
    g = gg.leduc(13, 2)
    a = cfr.Solver(g, persistent=True, wg_nodes=65536)
    b = cfr.Solver(g)
    a.iterate(20)
    b.iterate(20)
    assert np.array_equal(a.state()[0], b.state()[0])


def test_autotune_picks_a_schedule_and_resets(tmp_path):
    games = subgames(16, seed=9, lo=1e3, hi=2e4)
    s = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64)
    cache = str(tmp_path / "tune.txt")
    r = s.autotune(10, cache_path=cache)
    note(f"[autotune] {r}")
    assert r["candidates"] >= 2 and r["ms_per_iteration"] > 0
    assert s.iterations == 0
    s.iterate(30)
    ref = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64)
    ref.iterate(30)
    assert np.array_equal(s.state()[0], ref.state()[0])
    # second call reads the cache
    t = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64)
    r2 = t.autotune(10, cache_path=cache)
    assert r2["candidates"] == 0 and r2["persistent"] == r["persistent"]


@pytest.mark.parametrize("order", ["sim", "alt"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_retired_games_keep_their_state_and_the_rest_are_unchanged(precision, order):
    """cfr_set_active: after 12 iterations games 1, 4 and 6 retire; 20 more iterations leave their
    regrets, strategy sums and strategy bitwise where they were, while the active games' iterates equal
    those of an uninterrupted run of the whole batch bitwise (games are independent; the shared
    counter advances alike).  Brought back, a retired game iterates again; cfr_reset brings every game
    back; the persistent schedule is refused while a game is retired."""
    games = mixed_batch()
    p = cfr.CFR_PRECISION_FP32 if precision == "fp32" else cfr.CFR_PRECISION_FP64
    o = cfr.CFR_ORDER_ALTERNATING if order == "alt" else cfr.CFR_ORDER_SIMULTANEOUS
    a = cfr.Solver(games, precision=p, order=o, iters_per_graph=5)
    b = cfr.Solver(games, precision=p, order=o)
    base = a.slot_base
    for s in (a, b):
        s.iterate(12)
    R12, S12 = a.state()
    cur12 = a.strategy()
    retired = [1, 4, 6]
    mask = np.ones(len(games), np.uint8)
    mask[retired] = 0
    a.set_active(mask)
    with pytest.raises(cfr.CfrError) as e:
        a.set_schedule(cfr.CFR_SCHEDULE_PERSISTENT, 4096)
    assert e.value.status == cfr.CFR_ESTATE
    a.iterate(20)
    b.iterate(20)
    Ra, Sa = a.state()
    Rb, Sb = b.state()
    cura, curb = a.strategy(), b.strategy()
    for k in range(len(games)):
        sl = slice(base[k], base[k + 1])
        if k in retired:
            assert np.array_equal(Ra[sl], R12[sl]) and np.array_equal(Sa[sl], S12[sl]), k
            assert np.array_equal(cura[sl], cur12[sl]), k
        else:
            assert np.array_equal(Ra[sl], Rb[sl]) and np.array_equal(Sa[sl], Sb[sl]), k
            assert np.array_equal(cura[sl], curb[sl]), k
    ea = a.batch_exploitability()[0]
    assert np.isfinite(ea).all()
    a.set_active(np.ones(len(games), np.uint8))
    a.iterate(3)
    R3, _ = a.state()
    assert not np.array_equal(R3[base[1]:base[2]], R12[base[1]:base[2]])
    a.set_active(mask)
    a.reset()
    a.iterate(5)
    c = cfr.Solver(games, precision=p, order=o)
    c.iterate(5)
    assert np.array_equal(a.state()[0], c.state()[0])


def test_single_game_cannot_be_retired():
    s = cfr.Solver(gg.kuhn())
    s.set_active([1])
    with pytest.raises(cfr.CfrError) as e:
        s.set_active([0])
    assert e.value.status == cfr.CFR_EUNSUPPORTED
    with pytest.raises(cfr.CfrError) as e:
        s.set_active([1, 1])
    assert e.value.status == cfr.CFR_EINVAL


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("rule", ["cfr+", "pcfr+", "dcfr-alt"])
def test_a_game_moves_out_of_the_batch_bitwise(precision, rule):
    """cfr_get_game_state returns each game's slice of the batch state (and the PCFR+ prediction)
    bitwise.  Set on a handle of that game alone (cfr_set_state, the batch's iteration count), on the
    LDS-resident schedule, the game then iterates bitwise as it does in the batch."""
    rules = {"cfr+": (cfr.CFR_RULE_CFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS),
             "pcfr+": (cfr.CFR_RULE_PCFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS),
             "dcfr-alt": (cfr.CFR_RULE_DCFR, cfr.CFR_ORDER_ALTERNATING)}
    r, o = rules[rule]
    p = cfr.CFR_PRECISION_FP32 if precision == "fp32" else cfr.CFR_PRECISION_FP64
    pred = rule == "pcfr+"
    games = mixed_batch()
    a = cfr.Solver(games, rule=r, order=o, precision=p)
    a.iterate(14)
    R, S = a.state()
    P = a.prediction() if pred else None
    base = a.slot_base
    for k in range(len(games)):
        sl = slice(base[k], base[k + 1])
        st = a.game_state(k, prediction=pred)
        assert np.array_equal(st[0], R[sl]) and np.array_equal(st[1], S[sl]), k
        if pred:
            assert np.array_equal(st[2], P[sl]), k
    movers = [0, 2, 3]   # Kuhn, a small random game, the worked example: all fit the LDS schedule
    hs = {}
    for k in movers:
        st = a.game_state(k, prediction=pred)
        h = cfr.Solver(games[k], rule=r, order=o, precision=p, persistent=cfr.CFR_SCHEDULE_LDS)
        h.set_state(st[0], st[1], a.iterations, st[2] if pred else None)
        hs[k] = h
    a.iterate(9)
    R2, S2 = a.state()
    for k, h in hs.items():
        h.iterate(9)
        Rh, Sh = h.state()
        sl = slice(base[k], base[k + 1])
        assert h.iterations == a.iterations
        assert np.array_equal(Rh, R2[sl]) and np.array_equal(Sh, S2[sl]), k
        h.close()
    with pytest.raises(cfr.CfrError) as e:
        a.game_state(len(games))
    assert e.value.status == cfr.CFR_EINVAL
    with pytest.raises(cfr.CfrError) as e:
        cfr.cfr_get_game_state(a.h, 0, int(base[1] - base[0]) + 1)
    assert e.value.status == cfr.CFR_EINVAL
    if not pred:
        with pytest.raises(cfr.CfrError) as e:
            a.game_state(0, prediction=True)
        assert e.value.status == cfr.CFR_EINVAL


def test_retiring_solve_moves_its_tail_with_the_same_crossings():
    """A retiring solve (games retired at the checkpoint where they reach the target) moves its last
    <= 8 games to LDS-resident handles of their own: the exploitability at every checkpoint, hence every
    crossing iteration, equals that of the same solve kept in the batch; afterwards the batch has every
    game active again."""
    import torch
    from paper_2609_11923_amd.warm import crossing_iterations, geometric_checkpoints, retiring_solve
    games = subgames(14, seed=3)
    pots = np.array([g.pot for g in games])
    thr = 1e-3 * pots.min()
    cps = geometric_checkpoints(3000)
    s = cfr.Solver(games)
    stream = torch.cuda.Stream()
    e1, u1, seg1, rec = retiring_solve(s, games, torch, cps, thr, stream)
    s.reset()
    e2, u2, seg2, rec2 = retiring_solve(s, games, torch, cps, thr, stream, move_tail=False)
    note(f"[tail] moved {rec}; segments {[round(x, 2) for x in seg1]} vs {[round(x, 2) for x in seg2]}")
    assert rec is not None and rec2 is None and 0 < len(rec["games"]) <= 8
    assert u1 == u2
    np.testing.assert_allclose(e1, e2, rtol=1e-12, atol=0)
    c1, c2 = crossing_iterations(u1, e1, thr), crossing_iterations(u2, e2, thr)
    assert np.isfinite(c1).all() and np.allclose(c1, c2, rtol=0, atol=1e-9)
    s.reset()
    s.iterate(4)
    t = cfr.Solver(games)
    t.iterate(4)
    assert np.array_equal(s.state()[0], t.state()[0])
