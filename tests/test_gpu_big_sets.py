"""GPU parity on the update paths that ordinary games leave unused: information sets with more members
than one LDS staging chunk of the fused backward/update level (1,024 members with FP32 state and at
most 4 actions, 512 with FP64, 256 with more than 4 actions), and sets with more than 16 actions (the
64-action instantiation).  Each game runs under the three child-addressing modes of the update (affine
offsets, the explicit child list, breadth-first implicit children), against the FP64 oracle: every one of
30 steps of the one-step test at 1e-5, and a free run of 100 iterations (FP64 state: the full bar; FP32
state: exploitability and the reach-weighted errors)."""
import numpy as np
import pytest

import gamegen as gg
import oracle
import paper_2609_11923_amd as cfr
from parity_metrics import rel_err, set_reach, slot_weights, weighted_err
from test_gpu_step_parity import step_parity

pytestmark = pytest.mark.gpu

TOL = 1e-5


def wide_game(n1, n2, a1, a2, seed):
    """A joint deal of (i, j) over n1 x n2 private types with seeded weights; player 1 acts with a1
    actions knowing i (n1 sets of n2 members each); player 2 answers each action with a2 actions knowing
    (action, j) (a1 n2 sets of n1 members); seeded terminal payoffs in [-1, 1].  Public states: the deal,
    player 1's node, player 2's node after each action, each terminal sequence."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.1, 1.0, n1 * n2)
    w /= w.sum()
    type_, kids, probs, key, pay, pub = [0], [[]], [list(w)], [-1], [0.0], [0]
    for i in range(n1):
        for j in range(n2):
            p1 = len(type_)
            kids[0].append(p1)
            type_.append(1); kids.append([]); probs.append(None); key.append(i); pay.append(0.0); pub.append(1)
            for a in range(a1):
                p2 = len(type_)
                kids[p1].append(p2)
                type_.append(2); kids.append([]); probs.append(None); key.append(1_000_000 + a * n2 + j)
                pay.append(0.0); pub.append(2 + a)
                for b in range(a2):
                    z = len(type_)
                    kids[p2].append(z)
                    type_.append(3); kids.append([]); probs.append(None); key.append(-1)
                    pay.append(float(rng.uniform(-1.0, 1.0))); pub.append(2 + a1 + a * a2 + b)
    return gg.from_arrays(type_, kids, probs, key, pay, pub=pub, pot=1.0, name=f"wide_{n1}x{n2}_{a1}x{a2}")


GAMES = {
    # FP32 chunk 1024, FP64 chunk 512 (at most 4 actions): three sets of 1,100 members
    "members1100_actions3": lambda: wide_game(3, 1100, 3, 2, 1),
    # more than 4 actions: chunk 256, three sets of 300 members with 6 actions
    "members300_actions6": lambda: wide_game(3, 300, 6, 2, 2),
    # more than 16 actions (the 64-action instantiation), 300 members
    "members300_actions20": lambda: wide_game(2, 300, 20, 2, 3),
}
MODES = {"affine": dict(layout=cfr.CFR_LAYOUT_PUBLIC, affine=True),
         "explicit": dict(layout=cfr.CFR_LAYOUT_PUBLIC, affine=False),
         "bfs": dict(layout=cfr.CFR_LAYOUT_BFS)}
PREC = {"fp64": cfr.CFR_PRECISION_FP64, "fp32": cfr.CFR_PRECISION_FP32}


@pytest.mark.parametrize("precision", list(PREC))
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("name", list(GAMES))
def test_big_sets(name, mode, precision):
    game = GAMES[name]()
    kw = MODES[mode]
    s = cfr.Solver(game, precision=PREC[precision], **kw)
    want = {"affine": 2, "explicit": 1, "bfs": 0}[mode]
    assert s.counts["child_addressing"] == want
    s.close()
    w = step_parity(game, "cfr+", "sim", precision, T=30, **kw)
    assert max(w.values()) <= TOL
    s = cfr.Solver(game, precision=PREC[precision], **kw)
    s.iterate(100)
    o = oracle.Oracle(game)
    o.iterate(100)
    R, _ = s.state()
    Ro, _, sco, sao = o.state()
    avg = s.strategy(average=True)
    e = s.exploitability()[0]
    eo = o.exploitability()[0]
    lay = o.layout()
    wt = slot_weights(lay, set_reach(game, lay, sao))
    print(f"[big sets] {name} {mode} {precision}: R {rel_err(R, Ro):.2e} avg {rel_err(avg, sao):.2e} "
          f"weighted avg {weighted_err(avg, sao, wt):.2e} expl {e:.9e} vs {eo:.9e}", flush=True)
    assert abs(e - eo) <= 1e-6 * game.pot
    assert weighted_err(avg, sao, wt) <= TOL
    assert weighted_err(R, Ro, wt, max(np.abs(Ro).max(), 1e-30)) <= TOL
    if precision == "fp64":
        assert rel_err(R, Ro) <= TOL and rel_err(avg, sao) <= TOL
