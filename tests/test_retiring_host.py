"""Host logic of the retiring solve (no GPU): when the last games leave the batch for handles of their
own, which games, on which streams, and how the time and the exploitability rows are assembled.  A
fake batch solver, fake per-game handles and fake streams and events stand in for the device: each
game's exploitability falls as rate / t, so every crossing iteration is known in closed form."""
import types

import numpy as np
import pytest

import paper_2609_11923_amd as cfr
from paper_2609_11923_amd import warm

MS_PER_ITER = 0.25       # fake batch: milliseconds per iteration while any game is active
MS_PER_ITER_TAIL = 0.01  # fake own handles: milliseconds per iteration


class FakeStream:
    """A stream is its own clock: work on it advances t, waiting on an event moves t up to it."""

    def __init__(self):
        self.t = 0.0

    def wait_event(self, ev):
        self.t = max(self.t, ev.t)


class FakeEvent:
    def __init__(self, enable_timing=False):
        self.t = 0.0

    def record(self, stream):
        self.t = stream.t

    def synchronize(self):
        pass

    def elapsed_time(self, other):
        return other.t - self.t


def fake_torch():
    return types.SimpleNamespace(cuda=types.SimpleNamespace(Event=FakeEvent, Stream=FakeStream))


class FakeGame:
    def __init__(self, n_nodes, rate, fits=True):
        self.n_nodes, self.rate, self.fits = n_nodes, rate, fits


class FakeBatch:
    """Batch solver: every active game advances; exploitability of game i after t iterations is
    rate_i / t."""

    def __init__(self, games):
        self.games = games
        self.n_games = len(games)
        self.t = 0
        self.active = np.ones(self.n_games, np.uint8)
        self.set_active_calls = []
        self.options = types.SimpleNamespace(rule=cfr.CFR_RULE_CFR_PLUS, averaging=0, order=0, precision=0,
                                             device=0)
        self.game_t = np.zeros(self.n_games)

    @property
    def iterations(self):
        return self.t

    def iterate(self, n, stream=None):
        stream.t += n * MS_PER_ITER
        self.t += n
        self.game_t[self.active.astype(bool)] += n

    def batch_exploitability(self, stream=None):
        return (np.array([g.rate / max(t, 1) for g, t in zip(self.games, self.game_t)]),)

    def set_active(self, mask, stream=None):
        self.active = np.array(mask, np.uint8)
        self.set_active_calls.append(self.active.copy())

    def game_state(self, i, prediction=False, stream=None):
        return (np.full(3, float(self.game_t[i])), np.zeros(3))


class FakeHandle:
    """A game on a handle of its own: continues from the batch's count for that game."""
    made = []

    def __init__(self, game, **kw):
        if not game.fits:
            raise cfr.CfrError(cfr.CFR_EINVAL, "the game does not fit in LDS")
        assert kw["persistent"] == cfr.CFR_SCHEDULE_LDS
        self.game, self.t, self.closed, self.streams = game, 0.0, False, []
        FakeHandle.made.append(self)

    def set_state(self, regrets, strategy_sum, t, prediction=None):
        self.t = float(regrets[0])   # the fake batch puts the game's own count there

    def iterate(self, n, stream=None):
        stream.t += n * MS_PER_ITER_TAIL
        self.streams.append(stream)
        self.t += n

    def exploitability(self, stream=None):
        return (self.game.rate / self.t, 0.0, 0.0, 0.0)

    def close(self):
        self.closed = True


@pytest.fixture
def fakes(monkeypatch):
    FakeHandle.made = []
    monkeypatch.setattr(warm, "Solver", FakeHandle)
    return fake_torch(), FakeStream()


def solve(games, fakes, move=True, cps=(10, 20, 40, 80, 160, 320, 640)):
    torch, stream = fakes
    s = FakeBatch(games)
    thr = 1.0
    e, used, seg, rec = warm.retiring_solve(s, games, torch, list(cps), thr, stream, move_tail=move)
    return s, e, used, seg, rec


def test_the_last_games_move_and_every_checkpoint_is_unchanged(fakes):
    # exploitability rate / t: game i crosses the threshold 1 at t = rate_i (15 to 600)
    rates = [15, 18, 25, 30, 35, 50, 70, 90, 150, 300, 450, 600]
    games = [FakeGame(n_nodes=1000 + 100 * k, rate=r) for k, r in enumerate(rates)]
    s, e, used, seg, rec = solve(games, fakes)
    s2, e2, used2, seg2, rec2 = solve(games, fakes, move=False)
    assert rec2 is None and rec is not None
    # after 40 iterations the seven games with rate > 40 remain (at most eight): they move then
    assert rec["at_iteration"] == 40 and rec["games"] == [5, 6, 7, 8, 9, 10, 11]
    assert used == used2 and np.allclose(e, e2)
    cross = warm.crossing_iterations(used, e, 1.0)
    assert np.allclose(cross, warm.crossing_iterations(used2, e2, 1.0))
    assert np.allclose(cross, rates)
    # after the move the batch is no longer iterated; it is all active again at the end
    assert s.t == 40 and s.active.all()
    # four streams, largest game first onto the least loaded: games 11, 10, 9, 8 open one each, then
    # 7 joins game 8's, 6 game 9's and 5 game 10's
    lanes = {h.game.rate: h.streams[0] for h in FakeHandle.made}
    assert len({id(x) for x in lanes.values()}) == 4
    assert lanes[90] is lanes[150] and lanes[70] is lanes[300] and lanes[50] is lanes[450]
    assert all(lanes[600] is not lanes[r] for r in (50, 70, 90, 150, 300, 450))
    assert all(h.closed for h in FakeHandle.made)
    # the segment after the move: the busiest stream (two games, 40 iterations each) plus, once, the
    # move's host time
    assert seg[:3] == seg2[:3]
    assert seg[3] == pytest.approx(2 * 40 * MS_PER_ITER_TAIL + rec["move_host_ms"])
    assert seg2[3] == pytest.approx(40 * MS_PER_ITER)


def test_a_game_that_does_not_fit_stays_in_the_batch(fakes):
    rates = [15, 18, 25, 30, 35, 50, 70, 90, 150, 300, 450, 600]
    games = [FakeGame(n_nodes=1000, rate=r, fits=(k != 11)) for k, r in enumerate(rates)]
    s, e, used, seg, rec = solve(games, fakes)
    # the largest-rate game never fits: nothing moves, the batch runs to the end, handles made on the
    # way are closed, and the attempt is not repeated at later checkpoints
    assert rec is None and s.t == used[-1]
    assert all(h.closed for h in FakeHandle.made)
    assert len(FakeHandle.made) == 6   # games 5..10 were made before game 11 failed, once
    s2, e2, used2, _, _ = solve(games, fakes, move=False)
    assert used == used2 and np.allclose(e, e2)


def test_no_move_while_more_than_eight_games_remain(fakes):
    games = [FakeGame(n_nodes=500, rate=1000 + k) for k in range(10)]
    s, e, used, seg, rec = solve(games, fakes, cps=(100, 200, 400, 800, 1600))
    # all ten cross together between 800 and 1600: never at most eight left before the end
    assert rec is None and FakeHandle.made == []
    assert np.isfinite(warm.crossing_iterations(used, e, 1.0)).all()


def test_stopwatch_reruns_until_every_game_is_there(monkeypatch):
    """stopwatch_to_all starts at the interpolated last crossing and reruns the whole timed solve with
    2 % more iterations (plus one) until every game is below the threshold, at most `runs` times."""
    calls = []

    def fake_stopwatch(s, rows, torch, n, **kw):
        calls.append(n)
        return {"iterations": n, "ms_events": n * 0.25, "reached": 256 if n >= 2300 else 255, "games": 256}

    monkeypatch.setattr(warm, "stopwatch", fake_stopwatch)
    sw = warm.stopwatch_to_all(None, None, None, 2235)
    assert calls == [2235, 2281, 2328]        # ceil(n * 1.02) + 1 each time
    assert sw["reached"] == 256 and sw["iterations"] == 2328
    assert sw["interpolated_iterations"] == 2235 and sw["runs"] == 3
    calls.clear()
    sw = warm.stopwatch_to_all(None, None, None, 100, runs=2)
    assert calls == [100, 103] and sw["runs"] == 2 and sw["reached"] == 255   # capped: reported as is
