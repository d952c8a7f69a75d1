"""What the trained warm-start network gains over the method without it (GPU, end to end).

Train the network on the average strategies the solver produced for one set of subgames (their
own payoff seed), then solve held-out subgames (another payoff seed) three ways on one compiled
batch: cold (plain CFR+ from zero regrets), warm (the first `PROBE` iterations of the solve, then
regrets from the trained network), and the same warm start with the untrained network.  Exact
exploitability (the device best response) decides.  The network's regrets are added to the
probe's (scale 0.5 iterations' worth).  Every step is seeded and every reduction has
a fixed order, so the outcome is reproducible; the gain itself is not pinned by the paper (it has
no learned part)."""
import sys

import numpy as np
import pytest
import torch

import gamegen as gg
import paper_2609_11923_amd as cfr
from paper_2609_11923_amd import warm

pytestmark = pytest.mark.gpu

PROBE = 16


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_trained_network_beats_cold_start_and_untrained_network():
    tr = gg.random_subgames(800, seed=11, lo=1e3, hi=1e5, game_seed=5)
    X, T, W, N, st = warm.make_training_set(tr, 400, torch, probe=PROBE, log=note)
    note(f"[warm test] {st['rows']} rows, target entropy {st['target_entropy']:.3f}")
    sizes = [(cfr.CFR_FEATURES, 256), (256, 256), (256, 256), (256, cfr.CFR_MLP_OUT)]
    theta0 = gg.mlp_init(sizes, seed=1)
    net = cfr.Mlp()
    net.set_params(theta0)
    hist = warm.train(net, X, T, W, N, torch, epochs=8, lr=2e-3, log=note)
    assert hist[-1]["train_loss_sample"] < hist[0]["train_loss_sample"]
    ctl = cfr.Mlp()
    ctl.set_params(theta0)
    test = warm.subgames(gg.random_subgames(64, seed=12, lo=1e3, hi=1e5, game_seed=6))
    ev = warm.evaluate(test, torch, net, 0.5, 3000, control=ctl, probe=PROBE, add=True, log=note, retire=True)
    cold, wst, unt = ev["cold"]["_cross"], ev["warm"]["_cross"], ev["control_untrained_net"]["_cross"]
    note(f"[warm test] median iterations: cold {np.median(cold):.1f}, warm {np.median(wst):.1f}, "
         f"untrained {np.median(unt):.1f}; warm faster on {np.mean(wst < cold):.2f} of games")
    # (a game that never reaches the threshold counts as infinitely slow)
    assert np.isfinite(cold).mean() >= 0.9 and np.isfinite(wst).mean() >= 0.9
    assert np.median(wst) < 0.95 * np.median(cold)
    assert np.median(wst) < np.median(unt)
    # wall time includes the feature pass, probe, network and injection
    assert ev["warm"]["time_ms_median"] < ev["cold"]["time_ms_median"]
    for arm in ("cold", "warm"):
        # retiring each game at the checkpoint where it reached the target changes no crossing and,
        # when every game got there, shortens the time until the last one did
        rt = ev[arm]["retiring"]
        assert rt["crossings_equal"]
        if rt["time_ms_all"] is not None and ev[arm]["time_ms_all"] is not None:
            note(f"[warm test] {arm}: all at the target after {ev[arm]['time_ms_all']:.1f} ms, "
                 f"{rt['time_ms_all']:.1f} ms retiring")
            assert rt["time_ms_all"] <= ev[arm]["time_ms_all"] * 1.02
        sw = ev[arm].get("stopwatch")
        if sw is not None:
            # run straight through past the last crossing, every game is at the threshold, within a few
            # per cent of the interpolated crossing
            note(f"[warm test] {arm} stopwatch: {sw}")
            assert sw["ms_events"] > 0 and sw["reached"] == sw["games"]
            assert sw["iterations"] <= sw["interpolated_iterations"] * 1.1 + 6
