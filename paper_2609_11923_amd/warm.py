"""Learned warm start for batches of subgames (host-side driver of the library's kernels).

The paper has no learned part.  This module trains the warm-start network (cfr_mlp) on average
strategies the solver itself produced, and measures what it buys: iterations and wall time to
exploitability <= 1e-3 pot for the warm-started batch against plain cold-start CFR+ on the same
GPU, with an untrained network as a control.  Exact exploitability (the device best response)
decides; scale 0 (the cold start) is the fallback.

Everything numeric runs in libcfr.so: the solver, the feature rows, the network's forward,
backward and Adam steps, the warm-start injection.  torch holds device memory and streams;
numpy shuffles indices and assembles targets on the host.
"""
from __future__ import annotations

import time

import numpy as np

from . import (CFR_FEATURES, CFR_PRECISION_FP32, CFR_RULE_PCFR_PLUS, CFR_SCHEDULE_LDS, CfrError, Mlp, Solver)

THRESHOLD = 1e-3  # of the pot


def crossing_iterations(checkpoints, expl, thr):
    """Per game, the iteration at which exploitability first reaches thr, log-log interpolated
    between the bracketing checkpoints (the paper's time-to-target methodology); inf if never."""
    checkpoints = np.asarray(checkpoints, float)
    expl = np.asarray(expl, float)          # [checkpoints, games]
    out = np.full(expl.shape[1], np.inf)
    for g in range(expl.shape[1]):
        e = expl[:, g]
        hit = np.nonzero(e <= thr)[0]
        if hit.size == 0:
            continue
        k = hit[0]
        if k == 0 or e[k - 1] <= 0 or e[k] <= 0:
            out[g] = checkpoints[k]
            continue
        x0, x1 = np.log(checkpoints[k - 1]), np.log(checkpoints[k])
        y0, y1 = np.log(e[k - 1]), np.log(e[k])
        f = (np.log(thr) - y0) / (y1 - y0) if y1 != y0 else 1.0
        out[g] = float(np.exp(x0 + f * (x1 - x0)))
    return out


def subgames(specs, threads=8):
    """The subgames of `specs` (input generation: the generator's C code runs on several threads)."""
    import gamegen as gg
    from concurrent.futures import ThreadPoolExecutor
    one = lambda sp: gg.subgame(**{k: v for k, v in sp.items() if k != "target"})   # noqa: E731
    if threads <= 1 or len(specs) < 2:
        return [one(sp) for sp in specs]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, specs))


class Rows:
    """Device inputs of cfr_features for a list of games (canonical set order, games in order)."""

    def __init__(self, games, torch, device="cuda:0"):
        import gamegen as gg
        self.games = games
        bs, hs, ss, na = [], [], [], []
        self.game_off = [0]
        for g in games:
            first, _ = gg.first_members(g)
            b, h, s = gg.warm_descriptors(g, first=first)
            bs.append(b); hs.append(h); ss.append(s)
            na.append(np.asarray(g.n_children)[first])
            self.game_off.append(self.game_off[-1] + len(first))
        self.nact = np.concatenate(na).astype(np.int64)
        self.I = len(self.nact)
        self.bucket = torch.tensor(np.concatenate(bs), device=device)
        self.history = torch.tensor(np.concatenate(hs), device=device)
        self.scalars = torch.tensor(np.concatenate(ss), device=device)
        self.x = torch.empty(self.I, CFR_FEATURES, dtype=torch.bfloat16, device=device)

    def features(self, solver, probe=0, stream=None):
        assert solver.n_infosets == self.I
        solver.features(self.bucket, self.history, self.scalars, self.x, probe_iters=probe, stream=stream)


def make_training_set(specs, iters, torch, probe=0, chunk=256, precision=CFR_PRECISION_FP32, solver_kw=None,
                      log=print):
    """Solve the subgames of `specs` in batches of `chunk` for `iters` CFR+ iterations and keep,
    per information set with at most 4 actions, its feature row and the solver's average
    strategy as the target.  Row weights are the sets' regret units m(I) (which grow with the
    opponent's and chance's reach of the set), normalised to sum to 1 over each subgame.
    Returns device tensors X [n, 128] bf16, T [n, 4] f32, W [n] f32, nact [n] u8, and stats."""
    Xs, Ts, Ws, Ns = [], [], [], []
    ent = 0.0
    t0 = time.perf_counter()
    stats = dict(subgames=0, edges=0, rows=0, gen_s=0.0, compile_s=0.0, solve_s=0.0)
    for c0 in range(0, len(specs), chunk):
        ta = time.perf_counter()
        games = subgames(specs[c0:c0 + chunk])
        tb = time.perf_counter()
        s = Solver(games, precision=precision, iters_per_graph=10, **(solver_kw or {}))
        rows = Rows(games, torch)
        tc = time.perf_counter()
        rows.features(s, probe=probe)       # the probe is the first `probe` iterations of this solve
        unit = torch.empty(rows.I, dtype=torch.float32, device=rows.x.device)
        s.regret_unit(unit)
        s.iterate(iters - probe)
        avg = s.strategy(average=True)        # host copy, synchronises
        td = time.perf_counter()
        off = np.concatenate([[0], np.cumsum(rows.nact)])
        keep = np.flatnonzero(rows.nact <= 4)
        T = np.zeros((len(keep), 4), np.float32)
        for a in range(4):
            has = rows.nact[keep] > a
            T[has, a] = avg[off[keep[has]] + a]
        u = unit.cpu().numpy().astype(np.float64)
        W = np.zeros(rows.I)
        for k, (lo, hi) in enumerate(zip(rows.game_off[:-1], rows.game_off[1:])):
            tot = u[lo:hi].sum()
            W[lo:hi] = u[lo:hi] / tot if tot > 0 else 1.0 / max(hi - lo, 1)
        Wk = W[keep]
        Tp = np.where(T > 0, T, 1.0)
        ent += float((Wk * -(T * np.log(Tp)).sum(axis=1)).sum())
        Xs.append(rows.x[torch.tensor(keep, device=rows.x.device)])
        Ts.append(torch.tensor(T, device=rows.x.device))
        Ws.append(torch.tensor(Wk.astype(np.float32), device=rows.x.device))
        Ns.append(torch.tensor(rows.nact[keep].astype(np.uint8), device=rows.x.device))
        stats["subgames"] += len(games)
        stats["edges"] += int(sum(g.n_edges for g in games))
        stats["rows"] += len(keep)
        stats["gen_s"] += tb - ta
        stats["compile_s"] += tc - tb
        stats["solve_s"] += td - tc
        s.close()
        del games
        log(f"[warm] data {stats['subgames']}/{len(specs)} subgames, {stats['rows']} rows, "
            f"{time.perf_counter() - t0:.1f} s")
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    W = torch.cat(Ws)
    N = torch.cat(Ns)
    # the weighted target entropy: the loss a perfect predictor would reach
    stats["target_entropy"] = ent / max(float(W.sum().item()), 1e-30)
    return X, T, W, N, stats


def train(mlp: Mlp, X, T, W, N, torch, epochs=4, batch=4096, lr=1e-3, lr_min=1e-4, seed=0, val=None, log=print):
    """Adam on shuffled minibatches of weighted rows, cosine learning-rate decay.  val: an optional
    (X, T, W, N) whose loss is reported after every epoch."""
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * max(1, n // batch)
    step = 0
    hist = []
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n).astype(np.int32), device=X.device)
        for k in range(0, n - batch + 1 if n >= batch else 1, batch):
            idx = perm[k:k + batch]
            rows = int(idx.shape[0])
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * step / max(1, steps)))
            mlp.train_step(X, T, W, N, rows, lr_t, idx=idx, n_data=n, stream=stream)
            step += 1
        torch.cuda.synchronize()
        rec = dict(epoch=ep + 1, steps=step, s=time.perf_counter() - t0)
        if val is not None:
            rec["val_loss"] = loss_of(mlp, *val, torch=torch)
        m = min(n, 65536)
        rec["train_loss_sample"] = loss_of(mlp, X[:m], T[:m], W[:m], N[:m], torch=torch)
        hist.append(rec)
        log(f"[warm] epoch {rec}")
    return hist


def loss_of(mlp: Mlp, X, T, W, N, torch):
    """Weighted mean cross entropy over rows (chunks of max_rows); the gradient buffer is
    overwritten, the parameters are not."""
    n = X.shape[0]
    cap = mlp.desc.max_rows
    tot, wt = 0.0, 0.0
    for k in range(0, n, cap):
        r = min(cap, n - k)
        wk = float(W[k:k + r].sum().item())
        tot += wk * mlp.backward(X[k:k + r], T[k:k + r], W[k:k + r], N[k:k + r], r)
        wt += wk
    return tot / max(wt, 1e-30)


def solve_curves(s: Solver, rows: Rows, torch, checkpoints, mlp=None, scale=0.0, probe=0, add=False, log=None,
                 retire_thr=None, seg_ms=None, tail_out=None):
    """One batch solve from scratch on solver s, with exploitability checkpoints at absolute
    iteration counts (a warm start's probe iterations count).  Timed on the stream with events:
    the warm start (feature pass, probe iterations, network, injection) and the iterations; the
    best-response evaluations at the checkpoints are not timed.  With retire_thr, a game whose
    exploitability is at most retire_thr at a checkpoint is retired (cfr_set_active) and no longer
    iterated, and the last few games finish on handles of their own (retiring_solve); seg_ms (a list)
    then receives the measured milliseconds of every segment between checkpoints and tail_out (a dict)
    the record of that move.  Returns (expl [checkpoints, games], warm_ms, iter_ms, the checkpoints
    used)."""
    stream = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    warm_ms = 0.0
    s.reset()
    torch.cuda.synchronize()
    if mlp is not None:
        ev[0].record(stream)
        rows.features(s, probe=probe, stream=stream)
        s.warm_start(mlp, rows.x, scale, add=add, stream=stream)
        ev[1].record(stream)
        ev[1].synchronize()
        warm_ms = ev[0].elapsed_time(ev[1])
    done = probe if mlp is not None else 0
    checkpoints = [int(c) for c in checkpoints if c > done]
    if retire_thr is not None:
        expl, used, seg, rec = retiring_solve(s, rows.games, torch, checkpoints, retire_thr, stream, start=done,
                                              log=log)
        if seg_ms is not None:
            seg_ms.extend(seg)
        if tail_out is not None and rec is not None:
            tail_out.update(rec)
        return expl, warm_ms, float(sum(seg)), used
    expl, iter_ms = [], 0.0
    for c in checkpoints:
        ev[0].record(stream)
        s.iterate(int(c) - done, stream=stream)
        ev[1].record(stream)
        ev[1].synchronize()
        ms = ev[0].elapsed_time(ev[1])
        iter_ms += ms
        if seg_ms is not None:
            seg_ms.append(ms)
        done = int(c)
        expl.append(s.batch_exploitability(stream=stream)[0])
        if log is not None:
            log(f"[warm]   iteration {done}: median expl {np.median(expl[-1]):.3e}")
    return np.array(expl), warm_ms, iter_ms, checkpoints[:len(expl)]


# a retiring solve moves its last games to handles of their own once at most this many are left and
# every one fits the LDS-resident schedule; they run on up to TAIL_STREAMS streams at once
TAIL_GAMES = 8
TAIL_STREAMS = 4


class TinyTail:
    """The last games of a retiring batch solve, each on a handle of its own on the LDS-resident
    schedule (one workgroup runs whole iterations with the game's state in LDS: no launch per depth,
    where the batch's level launches would run near-empty).  Each game's state (cfr_get_game_state) and
    the batch's iteration count go into its handle (cfr_set_state), so it continues bitwise as it would
    in the batch.  The handles iterate concurrently on a few streams forked from and joined back into
    the caller's stream.  Raises CfrError (after adding the game to `too_big` and closing the handles made)
    when a game does not fit or cannot take the state."""

    def __init__(self, s: Solver, games, idx, torch, stream, too_big: set):
        o = s.options
        pred = o.rule == CFR_RULE_PCFR_PLUS
        t = s.iterations
        self.h = {}
        self.torch = torch
        for i in (int(x) for x in idx):
            try:
                h = Solver(games[i], rule=o.rule, averaging=o.averaging, order=o.order, precision=o.precision,
                           persistent=CFR_SCHEDULE_LDS, device=o.device)
                self.h[i] = h
                st = s.game_state(i, prediction=pred, stream=stream)
                h.set_state(st[0], st[1], t, st[2] if pred else None)
            except CfrError:
                too_big.add(i)   # not movable: the solve keeps it in the batch
                self.close()
                raise
        self.streams = [torch.cuda.Stream() for _ in range(min(TAIL_STREAMS, len(self.h)))]
        # largest game first onto the least loaded stream: games that share a stream run one after the other
        load = [0] * len(self.streams)
        self.lane = {}
        for i in sorted(self.h, key=lambda j: -games[j].n_nodes):
            q = int(np.argmin(load))
            self.lane[i] = q
            load[q] += games[i].n_nodes

    def iterate(self, n: int, stream):
        torch = self.torch
        fork = torch.cuda.Event()
        fork.record(stream)
        for st in self.streams:
            st.wait_event(fork)
        for i, h in self.h.items():
            h.iterate(n, stream=self.streams[self.lane[i]])
        for st in self.streams:
            join = torch.cuda.Event()
            join.record(st)
            stream.wait_event(join)

    def exploitability(self, stream) -> dict:
        return {i: h.exploitability(stream=stream)[0] for i, h in self.h.items()}

    def retire(self, i: int):
        self.h.pop(i).close()

    def close(self):
        for h in self.h.values():
            h.close()
        self.h = {}


def retiring_solve(s: Solver, games, torch, checkpoints, thr, stream, start=0, move_tail=True, log=None):
    """Iterate the batch on solver s from iteration `start` to each checkpoint, retiring (cfr_set_active)
    every game whose exploitability is at most thr at a checkpoint.  With move_tail, once at most
    TAIL_GAMES games are left and all fit the LDS-resident schedule they move to TinyTail handles and
    finish there (same iterates, no launch per depth).  Each segment between checkpoints is event-timed
    on `stream`; the host time of the move (compiles, state copies) is added to the segment after it.
    Best responses are not timed.  The batch's games are all active again on return, its state is that
    of the batch (a moved game's later iterations are not in it).  Returns (expl [checkpoints, games],
    checkpoints used, segment ms, record of the move or None)."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    active = np.ones(s.n_games, np.uint8)
    expl, used, seg = [], [], []
    tail, rec, too_big, pending_ms = None, None, set(), 0.0
    done = int(start)
    try:
        for c in (int(x) for x in checkpoints if x > start):
            ev[0].record(stream)
            if tail is not None:
                tail.iterate(c - done, stream)
            else:
                s.iterate(c - done, stream=stream)
            ev[1].record(stream)
            ev[1].synchronize()
            seg.append(ev[0].elapsed_time(ev[1]) + pending_ms)
            pending_ms = 0.0
            done = c
            used.append(c)
            if tail is None:
                e = np.array(s.batch_exploitability(stream=stream)[0])
            else:
                e = expl[-1].copy()
                for i, x in tail.exploitability(stream).items():
                    e[i] = x
            expl.append(e)
            active &= (e > thr).astype(np.uint8)
            if log is not None:
                log(f"[warm]   iteration {done}: median expl {np.median(e):.3e}, {int(active.sum())} games iterating"
                    + (" (moved to LDS-resident handles)" if tail is not None else ""))
            if not active.any():
                break
            if tail is not None:
                for i in [i for i in tail.h if not active[i]]:
                    tail.retire(i)
                continue
            idx = np.flatnonzero(active)
            if move_tail and len(idx) <= TAIL_GAMES and not too_big.intersection(int(i) for i in idx):
                t0 = time.perf_counter()
                try:
                    tail = TinyTail(s, games, idx, torch, stream, too_big)
                except CfrError:
                    tail = None
                if tail is not None:
                    pending_ms = (time.perf_counter() - t0) * 1e3
                    rec = {"at_iteration": done, "games": [int(i) for i in idx], "move_host_ms": pending_ms}
                    continue
            s.set_active(active, stream=stream)
    finally:
        if tail is not None:
            tail.close()
        s.set_active(np.ones(s.n_games, np.uint8), stream=stream)
    return np.array(expl), used, seg, rec


def retiring_time_to_all(cross, checkpoints, seg_ms, warm_ms, skip=0):
    """Wall time until the last game reaches the threshold when games retire at the checkpoint where
    they reached it: the warm start, the measured segments before the last game's bracketing segment
    and, of that segment, the share up to the last game's (interpolated) crossing iteration.  None if
    a game never got there."""
    if not np.isfinite(cross).all() or not len(seg_ms):
        return None
    last = float(np.max(cross))
    starts = [skip] + list(checkpoints[:-1])
    t = warm_ms
    for a, b, ms in zip(starts, checkpoints, seg_ms):
        if last >= b:
            t += ms
        else:
            t += ms * max(last - a, 0.0) / max(b - a, 1)
            break
    return float(t)


def stopwatch(s: Solver, rows: Rows, torch, iters, mlp=None, scale=0.0, probe=0, add=False, thr=None):
    """One uninterrupted solve from scratch to `iters` iterations counted from the start (a warm start's
    probe included), timed as a whole: on the stream with events and on the host clock from the first
    launch to the stream's end.  Exploitability is evaluated once, after the timed region, to count the
    games that reached `thr`."""
    stream = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    done = 0
    if mlp is not None:
        rows.features(s, probe=probe, stream=stream)
        s.warm_start(mlp, rows.x, scale, add=add, stream=stream)
        done = probe
    if iters > done:
        s.iterate(int(iters) - done, stream=stream)
    ev[1].record(stream)
    ev[1].synchronize()
    host_ms = (time.perf_counter() - t0) * 1e3
    e = s.batch_exploitability(stream=stream)[0]
    out = dict(iterations=int(iters), ms_events=float(ev[0].elapsed_time(ev[1])), ms_host=float(host_ms))
    if thr is not None:
        out["reached"] = int((np.asarray(e) <= thr).sum())
        out["games"] = int(np.asarray(e).size)
    return out


def stopwatch_to_all(s: Solver, rows: Rows, torch, iters, runs=6, **kw):
    """stopwatch() from `iters` (the last game's crossing, interpolated between checkpoints): while some
    game is still above the threshold at the end, the whole timed solve runs again from scratch with 2 %
    more iterations (the iterates are reproducible bitwise, so each run repeats the previous one and
    goes on), at most `runs` times.  The result records the interpolated start and the runs taken."""
    n = int(iters)
    for k in range(1, runs + 1):
        sw = stopwatch(s, rows, torch, n, **kw)
        if sw.get("reached", 0) >= sw.get("games", 0) or k == runs:
            break
        n = int(np.ceil(n * 1.02)) + 1
    sw["interpolated_iterations"] = int(iters)
    sw["runs"] = k
    return sw


LEVEL_SYNC = {"persistent": 0, "wg_nodes": 0}


def batch_solver(games, torch, schedule=LEVEL_SYNC, precision=CFR_PRECISION_FP32, tune_iters=20, solver_kw=None,
                 log=print):
    """A compiled batch on the given schedule (None: autotuned).  Warm and cold arms share the
    handle, so they always run the same schedule and rule (solver_kw: rule, order)."""
    log(f"[warm] compiling {len(games)} games")
    # ten iterations per captured graph (remainders run the one-iteration graph)
    s = Solver(games, precision=precision, iters_per_graph=10, **(solver_kw or {}))
    if schedule is None:
        schedule = s.autotune(tune_iters, stream=torch.cuda.Stream())
        log(f"[warm] autotune: {schedule}")
    else:
        s.set_schedule(bool(schedule["persistent"]), int(schedule.get("wg_nodes", 0)))
    return s, schedule


def summarize(cross, ms_per_iter, warm_ms, skip=0):
    """Iterations to the threshold count from the start; wall time is the warm start (which holds
    the first `skip` iterations) plus the remaining iterations at the measured rate."""
    fin = np.isfinite(cross)
    t = lambda it: float(warm_ms + max(it - skip, 0.0) * ms_per_iter)  # noqa: E731
    q = lambda a, p: float(np.percentile(a, p)) if a.size else None  # noqa: E731
    return dict(
        reached=int(fin.sum()), games=int(cross.size),
        iterations_median=float(np.median(cross)),
        iterations_iqr=[float(np.percentile(cross, 25)), float(np.percentile(cross, 75))],
        time_ms_median=t(np.median(cross)),
        time_ms_iqr=[t(np.percentile(cross, 25)), t(np.percentile(cross, 75))],
        time_ms_all=t(np.max(cross)) if fin.all() else None,
        probe_iterations=int(skip),
        reached_iterations_median=q(cross[fin], 50),
        warm_ms=float(warm_ms), ms_per_iteration=float(ms_per_iter),
    )


def geometric_checkpoints(t_max, first=8):
    c, k = [], first
    while k < t_max:
        c.append(k)
        k = int(np.ceil(k * 1.5))
    return c + [t_max]


def choose_scale(games, torch, mlp, scales, t_max, probe=0, schedule=LEVEL_SYNC, solver_kw=None, add=False,
                 log=print):
    """The scale whose warm start reaches the threshold in the fewest iterations (median over the
    validation games; ties and unreached games broken by the geometric mean of the final
    exploitability)."""
    cps = geometric_checkpoints(t_max)
    pots = np.array([g.pot for g in games])
    s, _ = batch_solver(games, torch, schedule=schedule, solver_kw=solver_kw, log=log)
    rows = Rows(games, torch)
    best = None
    table = []
    for c in scales:
        log(f"[warm] validation solve at scale {c}")
        e, _, _, used = solve_curves(s, rows, torch, cps, mlp=mlp, scale=c, probe=probe, add=add, log=log)
        cross = crossing_iterations(used, e, THRESHOLD * pots.min())
        score = (float(np.median(cross)), float(np.exp(np.mean(np.log(np.maximum(e[-1], 1e-12))))))
        table.append(dict(scale=c, median_iterations=score[0], final_expl_geomean=score[1]))
        log(f"[warm] scale {c}: median iterations {score[0]:.1f}, final expl geomean {score[1]:.3e}")
        if best is None or score < best[0]:
            best = (score, c)
    s.close()
    return best[1], table


def evaluate(games, torch, mlp, scale, t_max, control=None, probe=0, schedule=LEVEL_SYNC, solver_kw=None, add=False,
             log=print, retire=False):
    """Cold, warm and (optional) control-network solves of the same batch with the same compiled
    handle and schedule; per-game iterations and wall time to exploitability <= 1e-3 pot."""
    s, schedule = batch_solver(games, torch, schedule=schedule, solver_kw=solver_kw, log=log)
    rows = Rows(games, torch)
    cps = geometric_checkpoints(t_max)
    pots = np.array([g.pot for g in games])
    thr = THRESHOLD * pots.min()
    out = {"schedule": schedule}
    arms = [("cold", None, 0.0), ("warm", mlp, scale)]
    if control is not None:
        arms.append(("control_untrained_net", control, scale))
    for name, net, c in arms:
        log(f"[warm] test solve: {name}")
        e, warm_ms, iter_ms, used = solve_curves(s, rows, torch, cps, mlp=net, scale=c, probe=probe, add=add, log=log)
        cross = crossing_iterations(used, e, thr)
        # iterations count from the start (probe included); the probe's time is inside warm_ms
        skip = probe if net is not None else 0
        out[name] = summarize(cross, iter_ms / (used[-1] - skip), warm_ms, skip)
        if retire and not schedule.get("persistent"):
            # the same solve, each game retired at the checkpoint where it reached the threshold
            s.reset()
            seg, tail = [], {}
            e2, warm2, _, used2 = solve_curves(s, rows, torch, cps, mlp=net, scale=c, probe=probe, add=add,
                                              log=log, retire_thr=thr, seg_ms=seg, tail_out=tail)
            cross2 = crossing_iterations(used2, e2, thr)
            out[name]["retiring"] = {
                "time_ms_all": retiring_time_to_all(cross2, used2, seg, warm2, skip),
                "crossings_equal": bool(np.allclose(cross2, cross, rtol=0, atol=1e-9, equal_nan=True)),
                "segment_ms": [float(x) for x in seg], "checkpoints": [int(x) for x in used2],
                "tail_moved": tail or None}
        out[name]["expl_final_median"] = float(np.median(e[-1]))
        out[name]["_cross"] = cross
        if np.isfinite(cross).all():
            # the same solve run straight through to the last game's crossing, timed as a whole
            out[name]["stopwatch"] = stopwatch_to_all(s, rows, torch, int(np.ceil(cross.max())), mlp=net,
                                                      scale=c, probe=probe, add=add, thr=thr)
        log(f"[warm] {name}: {({k: v for k, v in out[name].items() if not k.startswith('_')})}")
    s.close()
    return out


# above this many nodes a game cannot fit one workgroup's 160 KB of LDS (three 4-byte values per node
# alone): not worth a compile to find out
LDS_NODES_MAX = 16384


def alone_ms_per_iteration(games, torch, iters=50, log=print, lds=None):
    """Milliseconds per iteration of each game solved on its own: hipGraph replay of ten iterations per
    graph (as the batch runs), or, where the game fits one workgroup's LDS and it is faster, the
    LDS-resident schedule -- the per-game cost of plain one-at-a-time solving with the better of the
    two.  A batch reproduces each game's iterates bitwise, so its crossing iterations carry over
    unchanged.  lds (a list), if given, receives the indices of the games the LDS schedule won."""
    out = np.zeros(len(games))
    stream = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(s):
        s.iterate(13, stream=stream)      # direct iteration + capture of the graphs
        ev[0].record(stream)
        s.iterate(iters, stream=stream)
        ev[1].record(stream)
        ev[1].synchronize()
        s.close()
        return ev[0].elapsed_time(ev[1]) / iters

    for k, g in enumerate(games):
        out[k] = timed(Solver(g, iters_per_graph=10))
        s = None
        if g.n_nodes <= LDS_NODES_MAX:
            try:
                s = Solver(g, persistent=CFR_SCHEDULE_LDS)
            except CfrError:
                s = None                  # does not fit one workgroup's LDS
        if s is not None:
            ms = timed(s)
            if ms < out[k]:
                out[k] = ms
                if lds is not None:
                    lds.append(k)
        if (k + 1) % 64 == 0:
            log(f"[warm] timed {k + 1}/{len(games)} games alone")
    return out

