"""GPU parity on the large game at its full size: 36-card deck, K = 10 two-card hands per player (seed 0),
220,492,889 nodes -- the benchmark's headline game -- in FP64 state for 3 iterations against the FP64
oracle at the method's bar (normwise relative error <= 1e-5 on the regrets and the average strategy,
exploitability within 1e-6 pot).  The oracle holds the whole tree on the host (about 55 GB)."""
import sys

import numpy as np
import pytest

import gamegen as gg
import oracle
import paper_2609_11923_amd as cfr
from parity_metrics import rel_err

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(900)
def test_large_game_full_size_fp64_three_iterations():
    h1, h2 = gg.sample_hands(10, 0)
    game = gg.large(10, seed=0, hands=(h1, h2))
    note(f"[full] large game K=10: {game.n_nodes} nodes")
    s = cfr.Solver(game, precision=cfr.CFR_PRECISION_FP64)
    s.iterate(3)
    R, _ = s.state()
    avg = s.strategy(average=True)
    e, b1, b2, v = s.exploitability()
    s.close()
    note(f"[full] gpu done: expl {e:.9e}")
    o = oracle.Oracle(game)
    o.iterate(3)
    Ro, _, _, sao = o.state()
    eo, _, _, vo = o.exploitability()
    eR, eavg = rel_err(R, Ro), rel_err(avg, sao)
    note(f"[full] R {eR:.2e} avg {eavg:.2e} expl gpu {e:.9e} oracle {eo:.9e}")
    assert eR <= 1e-5 and eavg <= 1e-5
    assert abs(e - eo) <= 1e-6 * game.pot and abs(v - vo) <= 1e-6 * game.pot
    assert (R >= 0).all()
