"""One-step parity along the oracle's own trajectory: the GPU iteration map against the FP64 oracle.

For t = 0 .. T-1 the oracle's state after t iterations (cumulative regrets, strategy sums and, under
PCFR+, the prediction) is loaded into the GPU solver with cfr_set_state, which rounds it to the state
type; the GPU runs iteration t + 1 and its state is compared with the oracle's after t + 1 iterations.
The bar is the method's: normwise relative error <= 1e-5 on the regrets, the strategy sums, the
normalised average strategy and the PCFR+ prediction (the iteration's instantaneous regret).

Why both this and the free-running comparison (tests/test_gpu_parity.py, test_gpu_rules.py).  After
100 free-running iterations two correct implementations whose arithmetic differs at the last bit can
part by far more than 1e-5: regret matching (plus) switches a set between a pure and a mixed strategy
when a regret crosses zero, and the alternating and discounted rules amplify such changes from
iteration to iteration (the oracle's own FP32 build, and its FP64 build summing children in reverse
order, show it).  Loading the reference state before every iteration removes that amplification, so every
one of the 100 iterations is held to the bar, in FP32 state as in FP64."""
import sys

import numpy as np
import pytest

import gamegen as gg
import oracle
import paper_2609_11923_amd as cfr
from parity_metrics import rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-5
RULES = {"cfr": cfr.CFR_RULE_CFR, "cfr+": cfr.CFR_RULE_CFR_PLUS, "dcfr": cfr.CFR_RULE_DCFR,
         "pcfr+": cfr.CFR_RULE_PCFR_PLUS}
ORDERS = {"sim": cfr.CFR_ORDER_SIMULTANEOUS, "alt": cfr.CFR_ORDER_ALTERNATING}
PREC = {"fp64": cfr.CFR_PRECISION_FP64, "fp32": cfr.CFR_PRECISION_FP32}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def step_parity(game, rule="cfr+", order="sim", precision="fp32", T=100, steps=None, **solver_kw):
    """Worst per-step errors over the checked steps (all of 0..T-1 unless `steps` is given); solver_kw
    go to the solver (layout, child addressing)."""
    steps = set(range(T)) if steps is None else set(steps)
    o = oracle.Oracle(game, alternating=(order == "alt"), rule=rule)
    s = cfr.Solver(game, rule=RULES[rule], order=ORDERS[order], precision=PREC[precision], **solver_kw)
    worst = dict(R=0.0, S=0.0, avg=0.0, pred=0.0)
    for t in range(T):
        if t in steps:
            R, S, _, _ = o.state()
            pred = o.prediction() if rule == "pcfr+" else None
            s.set_state(R, S, t, pred)
            s.iterate(1)
        o.iterate(1)
        if t not in steps:
            continue
        Ro, So, _, sao = o.state()
        Rg, Sg = s.state()
        e = dict(R=rel_err(Rg, Ro), S=rel_err(Sg, So), avg=rel_err(s.strategy(average=True), sao))
        if rule == "pcfr+":
            e["pred"] = rel_err(s.prediction(), o.prediction())
        for k, x in e.items():
            worst[k] = max(worst[k], x)
        if max(e.values()) > TOL:
            note(f"[step] {game.name} {rule} {order} {precision}: step {t + 1} errors {e}")
            break
    note(f"[step] {game.name} {rule} {order} {precision} ({len(steps)} steps): worst " +
         " ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    return worst


SMALL = {
    "kuhn": gg.kuhn,
    "leduc3x2": lambda: gg.leduc(3, 2),
    "random13": lambda: gg.random_game(13, 6, 6, 7, max_actions=5, max_chance=4),
}


@pytest.mark.parametrize("precision", list(PREC))
@pytest.mark.parametrize("order", list(ORDERS))
@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("name", list(SMALL))
def test_step_parity_small(name, rule, order, precision):
    w = step_parity(SMALL[name](), rule, order, precision)
    assert max(w.values()) <= TOL


@pytest.mark.parametrize("precision", list(PREC))
@pytest.mark.parametrize("rule,order", [("cfr+", "sim"), ("cfr+", "alt"), ("dcfr", "alt"), ("pcfr+", "sim"),
                                        ("pcfr+", "alt")])
def test_step_parity_mid_game_full_size(rule, order, precision):
    """The mid game at its full size (13 ranks x 2 suits, 1,179,777 nodes), every one of 100 steps."""
    w = step_parity(gg.leduc(13, 2), rule, order, precision)
    assert max(w.values()) <= TOL


@pytest.mark.parametrize("layout", ["public", "bfs"])
@pytest.mark.parametrize("precision", list(PREC))
def test_step_parity_large_game_generator(precision, layout):
    """The large game's generator at two hands per player (about 10M nodes): the oracle runs all 100
    iterations and the GPU map is checked at steps 1-5 and every tenth step up to 100."""
    steps = list(range(5)) + list(range(9, 100, 10))
    lay = cfr.CFR_LAYOUT_PUBLIC if layout == "public" else cfr.CFR_LAYOUT_BFS
    w = step_parity(gg.large(2, seed=0), "cfr+", "sim", precision, steps=steps, layout=lay)
    assert max(w.values()) <= TOL


def test_step_parity_fp32_batch_per_subgame():
    """A 12-subgame FP32 batch (sizes 1e3-1e5 edges): each game's oracle state is loaded into its slot
    range, one batched iteration runs, and every game's state matches its own oracle's next state."""
    specs = gg.random_subgames(12, seed=3, lo=1e3, hi=1e5)
    games = [gg.subgame(**{k: v for k, v in sp.items() if k != "target"}) for sp in specs]
    s = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP32)
    base = s.slot_base
    ors = [oracle.Oracle(g) for g in games]
    worst = 0.0
    for t in range(40):
        st = [o.state() for o in ors]
        s.set_state(np.concatenate([x[0] for x in st]), np.concatenate([x[1] for x in st]), t)
        s.iterate(1)
        for o in ors:
            o.iterate(1)
        R, S = s.state()
        avg = s.strategy(average=True)
        for k, o in enumerate(ors):
            Ro, So, _, sao = o.state()
            sl = slice(base[k], base[k + 1])
            e = max(rel_err(R[sl], Ro), rel_err(S[sl], So), rel_err(avg[sl], sao))
            worst = max(worst, e)
            assert e <= TOL, (t, k, e)
    note(f"[step] FP32 batch of 12 subgames, 40 steps: worst {worst:.2e}")
