"""Benchmark: CFR iterations per second of one compiled game on one MI355X.

A step is one complete CFR+ iteration (regret matching, forward reach pass, backward value
pass, regret and average updates), replayed from one hipGraph, with the game already resident
in HBM.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|mid|tiny|batch|batch-steps|mlp|warm]

Workloads (seeded, synthetic):
  large  36-card deck, K=10 two-card hands per player, two public rounds of pot betting,
         hashed payoffs in [-1, 1] (about 2.2e8 nodes; the largest single game)
  mid    Leduc-rule game with 13 ranks x 2 suits (1,179,777 nodes)
  tiny   Kuhn poker (55 nodes)
The roofline object reports the dominant kernel (largest share of iteration time) from
per-launch HIP events recorded on the stream the kernels run on (cfr_profile).  The
cpu_baseline object times the FP64 oracle on a bounded sample of the same workload on one host
core and scales it to the whole game.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CFR iters/sec + HBM GB/s; time to exploitability 1e-3 pot, warm vs cold"
HBM_PEAK_GBPS = 8000.0


def make_workload(name, K, seed):
    import gamegen as gg
    if name == "large":
        h1, h2 = gg.sample_hands(K, seed)
        g = gg.large(K, seed=seed, hands=(h1, h2))
        desc = f"large synthetic card game: 36-card deck, K={K} two-card hands per player (seed {seed}), " \
               f"2 public rounds, pot betting <=3 raises/round, hashed payoffs"
        # sample for the CPU baseline: the subtree of one compatible hand pair of the same game
        j = next(j for j, b in enumerate(h2) if not set(h1[0]) & set(b))
        sample = lambda: gg.large(1, seed=seed, hands=([h1[0]], [h2[j]]))
        return g, desc, sample, "one hand pair of the same game (its whole subtree), scaled by node count"
    if name == "mid":
        g = gg.leduc(13, 2)
        return g, "Leduc-rule game, 13 ranks x 2 suits, two limit rounds", (lambda: g), "the whole game"
    if name == "tiny":
        g = gg.kuhn()
        return g, "Kuhn poker", (lambda: g), "the whole game"
    raise SystemExit(f"unknown workload {name}")


def kernels_digest():
    """sha256 of the kernel source, to tie stored profiler counts to the kernels they measured."""
    import hashlib
    path = os.path.join(ROOT, "paper_2609_11923_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def stored_traffic(kernel, workload, precision, launches, path=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, when it was
    taken on the same kernel source, workload and precision; None otherwise."""
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path)).get(f"{kernel}/{workload}/{precision}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernels_sha256") != kernels_digest():
        return None
    return (rec["fetch_bytes_per_iteration"] + rec["write_bytes_per_iteration"]) / launches


def physical_rate(bytes_per_iteration, ms_per_iteration, peak=HBM_PEAK_GBPS):
    """GB/s of `bytes_per_iteration` moved in `ms_per_iteration`; raises if that exceeds the HBM peak,
    which bytes a kernel really moves cannot do."""
    rate = bytes_per_iteration / (ms_per_iteration * 1e-3) / 1e9
    if rate > peak * 1.0001:
        raise ValueError(f"{bytes_per_iteration:.4g} bytes in {ms_per_iteration:.4g} ms is {rate:.0f} GB/s, above "
                         f"the {peak:.0f} GB/s peak: these are not bytes the kernels move")
    return rate


def roofline_record(kernels, traffic_fn):
    """The roofline object of the dominant kernel (largest share of the iteration's time).
    achieved = the kernel's design bytes per launch (every index, state and value element it must
    read or write in this layout, counted once) over its mean launch duration; the method's per-unit
    byte figures are reported beside it for reference (they count reads this design never makes: a
    child pointer per edge, a template read per terminal, a separate regret pass), and the
    counter-measured traffic when profiles/ holds it for the current kernel source."""
    dom = max(kernels, key=lambda k: k["ms_per_iteration"])
    nl = dom["launches_per_iteration"]
    per_launch_ms = dom["ms_per_iteration"] / nl
    design = dom["bytes_per_iteration"] / nl
    method = dom["method_bytes_per_iteration"] / nl
    achieved = physical_rate(design, per_launch_ms)
    traffic = traffic_fn(dom["name"], nl)
    return {
        "bound": "hbm", "kernel": dom["name"], "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
        "bytes": "design bytes per launch: each index, state and value element the kernel must touch, once",
        "launches_per_iteration": nl, "ms_per_launch": per_launch_ms, "design_bytes_per_launch": design,
        "method_bytes_per_launch": method,
        "achieved_method_bytes": method / (per_launch_ms * 1e-3) / 1e9,
        "achieved_traffic": None if traffic is None else traffic / (per_launch_ms * 1e-3) / 1e9,
        "traffic_over_design": None if traffic is None else traffic / design,
    }


def time_to_target(solver, torch, pot, log, max_iters=20000, thr=1e-3, label=""):
    """Solve from a reset with exploitability checkpoints on a geometric schedule.  The training
    segments between checkpoints are timed with events on the solve's stream (best-response time is
    not training time); the crossing iteration is log-log interpolated between the bracketing
    checkpoints and its time interpolated on the measured cumulative training time."""
    from paper_2609_11923_amd.warm import crossing_iterations, geometric_checkpoints
    stream = torch.cuda.Stream()
    solver.reset()
    cps = geometric_checkpoints(max_iters)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    done, ms, times, expl = 0, 0.0, [], []
    for c in cps:
        ev0.record(stream)
        solver.iterate(c - done, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        ms += ev0.elapsed_time(ev1)
        done = c
        times.append(ms)
        expl.append(solver.exploitability(stream=stream)[0])
        log(f"[bench] {label} iteration {done}: expl {expl[-1]:.4e} ({expl[-1] / pot:.3e} pot), {ms:.1f} ms")
        if expl[-1] <= thr * pot:
            break
    n = len(expl)
    cross = float(crossing_iterations(cps[:n], np.asarray(expl)[:, None], thr * pot)[0])
    out = dict(threshold_pot=thr, reached=bool(np.isfinite(cross)), checkpoints=cps[:n],
               exploitability=[float(x) for x in expl], training_ms=times)
    if np.isfinite(cross):
        k = int(np.searchsorted(cps[:n], cross))
        c0, t0 = (cps[k - 1], times[k - 1]) if k > 0 else (0, 0.0)
        c1, t1 = cps[k], times[k]
        out["iterations"] = cross
        out["ms"] = t0 + (cross - c0) * (t1 - t0) / max(c1 - c0, 1)
    log(f"[bench] {label} time to {thr:g} pot: {out.get('iterations')} iterations, {out.get('ms')} ms")
    return out


def batch_games(n, seed):
    import gamegen as gg
    specs = gg.random_subgames(n, seed, lo=1e3, hi=1e6, game_seed=0)
    return [gg.subgame(**{k: v for k, v in sp.items() if k != "target"}) for sp in specs], specs


# iterations per captured graph for the batch's solves (10: 2 % faster than 1 per iteration on the
# 256-subgame batch; remainders run the one-iteration graph)
BATCH_ITERS_PER_GRAPH = 10


def run_batch(cfr, torch, games, iters, precision, log, tune_iters=20, warm=None, max_iters=4000):
    """Solve a batch of subgames: autotuned schedule, `iters` iterations timed in one call, then a
    fresh solve with exploitability checkpoints (not timed) for time to 1e-3 pot.  warm: optional
    initial regrets (canonical slot order) for the warm-started form."""
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    s = cfr.Solver(games, precision=precision, iters_per_graph=BATCH_ITERS_PER_GRAPH)
    t_compile = time.perf_counter() - t0
    s_counts = s.counts
    tune = s.autotune(tune_iters, stream=stream)
    log(f"[bench] batch autotune: {tune}")
    if warm is not None:
        s.set_regrets(warm, stream=stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.iterate(iters, stream=stream)
    ev1.record(stream)
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    e_final = s.batch_exploitability(stream=stream)[0]
    # per-kernel design bytes and durations of the level kernels (direct launches) for the roofline
    kernels = s.profile(5, stream=stream)
    design_iter = sum(k["bytes_per_iteration"] for k in kernels)
    roof = roofline_record(kernels, lambda name, nl: stored_traffic(name, "batch", "fp32", nl))
    # checkpointed solve for time to threshold
    s.reset()
    if warm is not None:
        s.set_regrets(warm, stream=stream)
    from paper_2609_11923_amd.warm import crossing_iterations, geometric_checkpoints, alone_ms_per_iteration
    checkpoints, expl = geometric_checkpoints(max_iters), []
    done = 0
    for c in checkpoints:
        s.iterate(c - done, stream=stream)
        done = c
        expl.append(s.batch_exploitability(stream=stream)[0])
        log(f"[bench] batch iteration {done}: median expl {np.median(expl[-1]):.3e}")
    pots = np.array([g.pot for g in games])
    cross = crossing_iterations(checkpoints, expl, 1e-3 * pots.min())
    ms_it = ms / iters
    # the same solve with every game retired at the checkpoint where it reached the threshold
    # (training segments event-timed, best responses excluded), the last few games moved to handles of
    # their own on the LDS-resident schedule; and without that move
    from paper_2609_11923_amd.warm import retiring_solve, retiring_time_to_all
    s.set_schedule(cfr.CFR_SCHEDULE_LEVEL, 0)   # retiring games needs the level-synchronous schedule
    retiring = {}
    for move in (True, False):
        s.reset()
        if warm is not None:
            s.set_regrets(warm, stream=stream)
        expl_r, used, seg, rec = retiring_solve(s, games, torch, checkpoints, 1e-3 * pots.min(), stream,
                                                move_tail=move)
        cross_r = crossing_iterations(used, expl_r, 1e-3 * pots.min())
        r = {"time_to_1e3pot_all_ms": retiring_time_to_all(cross_r, used, seg, 0.0),
             "crossings_equal": bool(np.allclose(cross_r, cross, rtol=0, atol=1e-9, equal_nan=True)),
             "segment_ms": seg, "checkpoints": used}
        if move:
            retiring = dict(r, tail_moved=rec,
                            what="each game retired (cfr_set_active) at the checkpoint where it reached 1e-3 pot; "
                                 "the last <= 8 games, once all fit, finish on LDS-resident handles of their own "
                                 "(host time of that move included)")
        else:
            retiring["without_tail_move"] = r
    log(f"[bench] batch with retiring games: all at 1e-3 pot after {retiring['time_to_1e3pot_all_ms']} ms "
        f"({retiring['without_tail_move']['time_to_1e3pot_all_ms']} ms without moving the tail)")
    s.close()
    lds_won = []
    alone = alone_ms_per_iteration(games, torch, log=log, lds=lds_won)
    fin = np.isfinite(cross)
    seq_ms = float(np.sum(cross[fin] * alone[fin]))
    bat_ms = float(np.max(cross[fin]) * ms_it) if fin.any() else None
    return dict(
        compile_s=t_compile, schedule=tune, group_sets=int(s_counts["group_sets"]),
        update_groups=int(s_counts["update_groups"]), iterations=iters, ms_total=ms, ms_per_iteration=ms_it,
        roofline=roof, design_bytes_per_iteration=design_iter,
        hbm_gbps_design_bytes=physical_rate(design_iter, ms_it),
        frac_design_bytes=physical_rate(design_iter, ms_it) / HBM_PEAK_GBPS, kernels=kernels,
        edges=int(sum(g.n_edges for g in games)),
        edge_iterations_per_s=sum(g.n_edges for g in games) * iters / (ms * 1e-3),
        expl_final_median=float(np.median(e_final)), expl_final_max=float(np.max(e_final)),
        reached_1e3pot=int(np.isfinite(cross).sum()),
        iterations_to_1e3pot_median=float(np.median(cross)),
        time_to_1e3pot_all_ms=float(np.max(cross) * ms_it) if np.isfinite(cross).all() else None,
        time_to_1e3pot_median_ms=float(np.median(cross) * ms_it),
        checkpoint_iterations=int(max_iters),
        retiring=retiring,
        one_at_a_time={
            "what": "each game alone on its own handle (hipGraph replay, ten iterations per graph, or the "
                    "LDS-resident schedule where the game fits and it is faster), run to its own crossing "
                    "iteration; the batch reproduces each game's iterates bitwise, so crossing iterations are "
                    "shared",
            "games_on_lds_schedule": len(lds_won),
            "ms_per_iteration_median": float(np.median(alone)), "ms_per_iteration_sum": float(np.sum(alone)),
            "games_counted": int(fin.sum()),
            "time_to_1e3pot_all_ms": seq_ms,
            "batched_time_to_1e3pot_same_games_ms": bat_ms,
            "wall_time_reduction": (1.0 - bat_ms / seq_ms) if bat_ms and seq_ms > 0 else None,
        },
    ), cross


def run_batch_steps(cfr, torch, args, log):
    """The 256-subgame batch under one schedule (level launches or the persistent launch): `warmup`
    then `steps` timed iterations, and for the level schedule the per-kernel roofline.  A light mode for
    profilers (no checkpointed solves)."""
    games, _ = batch_games(args.batch_games, args.seed)
    log(f"[bench] batch of {len(games)} subgames, {sum(g.n_edges for g in games)} edges, {args.batch_schedule}")
    s = cfr.Solver(games, use_graph=not args.direct, iters_per_graph=args.iters_per_graph)
    if args.batch_schedule == "persistent":
        s.set_schedule(cfr.CFR_SCHEDULE_PERSISTENT, args.wg_nodes)
    stream = torch.cuda.Stream()
    s.iterate(max(args.warmup, 1), stream=stream)
    stream.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    s.iterate(args.steps, stream=stream)
    ev1.record(stream)
    ev1.synchronize()
    ms_it = ev0.elapsed_time(ev1) / args.steps
    out = dict(schedule=args.batch_schedule, iters_per_graph=args.iters_per_graph, ms_per_iteration=ms_it, n_games=len(games),
               edges=int(sum(g.n_edges for g in games)), group_sets=int(s.counts["group_sets"]),
               update_groups=int(s.counts["update_groups"]))
    if args.batch_schedule == "level":
        kernels = s.profile(args.profile_iters, stream=stream)
        design_iter = sum(k["bytes_per_iteration"] for k in kernels)
        out.update(kernels=kernels, design_bytes_per_iteration=design_iter,
                   roofline=roofline_record(kernels, lambda name, nl: stored_traffic(name, "batch", "fp32", nl)),
                   frac_design_bytes=physical_rate(design_iter, ms_it) / HBM_PEAK_GBPS)
    log(f"[bench] batch {args.batch_schedule}: {ms_it:.4f} ms/iteration")
    s.close()
    return out


def run_mlp(cfr, torch, args, log, rows=1 << 18):
    """The warm-start network's kernels alone: inference over `rows` feature rows and Adam training steps
    on minibatches of 4,096 (seeded synthetic rows and targets), with the hidden GEMMs' rate against the
    BF16 matrix-core peak."""
    import gamegen as gg
    torch.manual_seed(0)
    sizes = [(cfr.CFR_FEATURES, 256), (256, 256), (256, 256), (256, cfr.CFR_MLP_OUT)]
    net = cfr.Mlp(max_rows=4096)
    net.set_params(gg.mlp_init(sizes, seed=1))
    x = torch.randn(rows, cfr.CFR_FEATURES, device="cuda").to(torch.bfloat16)
    z = torch.empty(rows, 4, dtype=torch.float32, device="cuda")
    flops_row = 2 * sum(a * b for a, b in sizes)
    net.forward(x, rows, z)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    ev0.record()
    for _ in range(reps):
        net.forward(x, rows, z)
    ev1.record()
    ev1.synchronize()
    ms_inf = ev0.elapsed_time(ev1) / reps
    B = 4096
    t = torch.softmax(torch.randn(rows, 4, device="cuda"), dim=1).float().contiguous()
    w = torch.ones(rows, device="cuda")
    nact = torch.full((rows,), 4, dtype=torch.uint8, device="cuda")
    steps = 50
    net.train_step(x, t, w, nact, B, 1e-3)
    torch.cuda.synchronize()
    ev0.record()
    for k in range(steps):
        off = (k * B) % (rows - B)
        net.train_step(x[off:], t[off:], w[off:], nact[off:], B, 1e-3)
    ev1.record()
    ev1.synchronize()
    ms_step = ev0.elapsed_time(ev1) / steps
    out = dict(rows=rows, inference_ms=ms_inf, inference_tflops=flops_row * rows / (ms_inf * 1e-3) / 1e12,
               train_batch=B, train_step_ms=ms_step,
               train_tflops=3 * flops_row * B / (ms_step * 1e-3) / 1e12, peak_tflops=2500.0,
               what="128 -> 3 x 256 -> 4 ReLU network, BF16 matrix cores, FP32 accumulation; training counts "
                    "forward, data and weight gradients (3x the forward flops)")
    log(f"[bench] mlp: {out}")
    net.close()
    return out


def run_rules(cfr, torch, games, log, max_iters=4000):
    """Time to exploitability <= 1e-3 pot of the batch under each update rule and order (the same
    games, compiled per rule, level-synchronous graph, FP32 state).  Iterations count full
    iterations (an alternating one runs both players' halves); wall time uses each rule's own
    measured time per iteration."""
    from paper_2609_11923_amd.warm import (crossing_iterations, geometric_checkpoints, retiring_solve,
                                           retiring_time_to_all)
    pots = np.array([g.pot for g in games])
    cps = geometric_checkpoints(max_iters)
    out = {}
    for name, rule, order in [("CFR+", cfr.CFR_RULE_CFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS),
                              ("CFR+ alternating", cfr.CFR_RULE_CFR_PLUS, cfr.CFR_ORDER_ALTERNATING),
                              ("DCFR", cfr.CFR_RULE_DCFR, cfr.CFR_ORDER_SIMULTANEOUS),
                              ("DCFR alternating", cfr.CFR_RULE_DCFR, cfr.CFR_ORDER_ALTERNATING),
                              ("PCFR+", cfr.CFR_RULE_PCFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS),
                              ("PCFR+ alternating", cfr.CFR_RULE_PCFR_PLUS, cfr.CFR_ORDER_ALTERNATING)]:
        s = cfr.Solver(games, rule=rule, order=order, iters_per_graph=BATCH_ITERS_PER_GRAPH)
        stream = torch.cuda.Stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        expl, done, ms = [], 0, 0.0
        for c in cps:
            ev0.record(stream)
            s.iterate(c - done, stream=stream)
            ev1.record(stream)
            ev1.synchronize()
            ms += ev0.elapsed_time(ev1)
            done = c
            expl.append(s.batch_exploitability(stream=stream)[0])
        cross = crossing_iterations(cps, expl, 1e-3 * pots.min())
        # the same solve with each game retired at the checkpoint where it reached the target (the last
        # few games finish on LDS-resident handles of their own)
        s.reset()
        expl_r, used, seg, _ = retiring_solve(s, games, torch, cps, 1e-3 * pots.min(), stream)
        s.close()
        cross_r = crossing_iterations(used, expl_r, 1e-3 * pots.min())
        ms_it = ms / cps[-1]
        fin = np.isfinite(cross)
        out[name] = dict(ms_per_iteration=ms_it, reached=int(fin.sum()), iterations_median=float(np.median(cross)),
                         time_to_1e3pot_median_ms=float(np.median(cross) * ms_it),
                         time_to_1e3pot_all_ms=float(np.max(cross) * ms_it) if fin.all() else None,
                         time_to_1e3pot_all_ms_retiring=retiring_time_to_all(cross_r, used, seg, 0.0),
                         expl_at_max_median=float(np.median(expl[-1])))
        log(f"[bench] rule {name}: {out[name]}")
    return out


def run_lifecycle(cfr, torch, games, specs, log, solves=5):
    """Reuse versus rebuild (the paper's lifecycle comparison) for new root ranges of every game
    of the batch: rewriting the root chance in place and resetting, against compiling the changed
    batch and running its first iteration (which captures the graph)."""
    import gamegen as gg
    rng = np.random.default_rng(123)
    s = cfr.Solver(games, lifecycle=True)
    s.iterate(2)
    reuse, rebuild = [], []
    for _ in range(solves):
        ranges = []
        new_specs = []
        for g, sp in zip(games, specs):
            r1 = rng.dirichlet(np.ones(len(sp["hands1"])))
            r2 = rng.dirichlet(np.ones(len(sp["hands2"])))
            ranges.append((r1, r2))
            new_specs.append(dict({k: v for k, v in sp.items() if k != "target"}, r1=r1, r2=r2))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, (r1, r2) in enumerate(ranges):
            s.set_root_ranges(r1, r2, game=k)
        s.reset()
        s.iterate(1)
        torch.cuda.synchronize()
        reuse.append(time.perf_counter() - t0)
        new_games = [gg.subgame(**sp) for sp in new_specs]     # input generation: not timed
        t0 = time.perf_counter()
        t = cfr.Solver(new_games)
        t.iterate(1)
        torch.cuda.synchronize()
        rebuild.append(time.perf_counter() - t0)
        t.close()
    s.close()
    out = dict(solves=solves, reuse_ms_median=1e3 * float(np.median(reuse)),
               rebuild_ms_median=1e3 * float(np.median(rebuild)),
               what="new root ranges for all games: cfr_set_root_ranges + reset + first iteration, versus "
                    "compile + first iteration (graph capture); game generation excluded")
    out["speedup"] = out["rebuild_ms_median"] / out["reuse_ms_median"]
    log(f"[bench] lifecycle: {out}")
    return out


def measure_game(cfr, torch, game, args, precision, log, iters_per_graph=None, then=None, profile=True):
    """Compile one game, replay `warmup` then time `steps` iterations (hip events on the stream the
    graph is launched on), then per-kernel durations and bytes (cfr_profile) and the roofline of
    the dominant kernel; the handle is released before returning."""
    t0 = time.perf_counter()
    prec = cfr.CFR_PRECISION_FP64 if precision == "fp64" else cfr.CFR_PRECISION_FP32
    ipg = args.iters_per_graph if iters_per_graph is None else iters_per_graph
    solver = cfr.Solver(game, iters_per_graph=ipg, precision=prec, use_graph=not args.direct)
    t_compile = time.perf_counter() - t0
    c = solver.counts
    log(f"[bench] {precision}: compiled in {t_compile:.1f} s: {c}")
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    solver.iterate(max(args.warmup, 1), stream=stream)   # the first call also captures the graph
    stream.synchronize()
    t_warm = time.perf_counter() - t0
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    solver.iterate(args.steps, stream=stream)
    ev1.record(stream)
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / args.steps
    log(f"[bench] {precision}: {args.steps} iterations in {ms:.2f} ms ({ms_step:.4f} ms/iteration)")
    if not profile:
        res = dict(counts=c, compile_s=t_compile, warmup_s=t_warm, ms_per_iteration=ms_step,
                   iterations_per_s=args.steps / (ms * 1e-3), iters_per_graph=ipg)
        if then is not None:
            res.update(then(solver))
        solver.close()
        return res
    kernels = solver.profile(args.profile_iters, stream=stream)
    bytes_iter = sum(k["bytes_per_iteration"] for k in kernels)
    method_iter = sum(k["method_bytes_per_iteration"] for k in kernels)
    workload = getattr(args, "traffic_workload", args.workload)
    roof = roofline_record(kernels, lambda name, nl: stored_traffic(name, workload, precision, nl))
    log(f"[bench] {precision}: kernels {kernels}")
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calibrate_copy} MiB done")
        del src, dst
    e, b1, b2, v = solver.exploitability(stream=stream)
    res = dict(
        counts=c, compile_s=t_compile, warmup_s=t_warm, ms_per_iteration=ms_step,
        iterations_per_s=args.steps / (ms * 1e-3), iters_per_graph=ipg,
        # the whole iteration's design bytes over the measured iteration time (checked physical)
        hbm_gbps_design_bytes=physical_rate(bytes_iter, ms_step), design_bytes_per_iteration=bytes_iter,
        frac_design_bytes=physical_rate(bytes_iter, ms_step) / HBM_PEAK_GBPS,
        # the method's per-unit figures, for reference only (reads this design never makes)
        gbps_method_bytes=method_iter / (ms_step * 1e-3) / 1e9, method_bytes_per_iteration=method_iter,
        roofline=roof,
        kernels=kernels,
        exploitability_after={"iterations": solver.iterations, "expl": e, "pot": float(c["pot"])},
    )
    if then is not None:
        res.update(then(solver))
    solver.close()
    del solver
    torch.cuda.empty_cache()
    return res


WARM_RULES = {}


def run_tiny(cfr, torch, log, iters=2000):
    """Tiny standalone games under the level schedule (graph replay, one launch per depth level) and
    the LDS schedule (one workgroup, the whole iteration in LDS, one launch per call): time per
    iteration over `iters` iterations on a fresh handle after a warm-up call of the same length."""
    import gamegen as gg
    games = [("kuhn", gg.kuhn(), cfr.CFR_PRECISION_FP32), ("kuhn", gg.kuhn(), cfr.CFR_PRECISION_FP64),
             ("leduc3x2", gg.leduc(3, 2), cfr.CFR_PRECISION_FP32), ("random7", gg.random_game(7, 4, 3, 6),
                                                                   cfr.CFR_PRECISION_FP32)]
    out = []
    for name, g, prec in games:
        row = {"game": name, "precision": "fp64" if prec == cfr.CFR_PRECISION_FP64 else "fp32",
               "nodes": int(len(g.type))}
        for sched, key in ((cfr.CFR_SCHEDULE_LEVEL, "level"), (cfr.CFR_SCHEDULE_LDS, "lds")):
            try:
                s = cfr.Solver(g, precision=prec, persistent=sched)
            except cfr.CfrError as e:
                row[key + "_ms_per_iteration"] = None
                row[key + "_error"] = str(e)
                continue
            st = torch.cuda.Stream()
            s.iterate(iters, stream=st)
            st.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            s.iterate(iters, stream=st)
            e1.record(st)
            e1.synchronize()
            row[key + "_ms_per_iteration"] = e0.elapsed_time(e1) / iters
            s.close()
        if row.get("level_ms_per_iteration") and row.get("lds_ms_per_iteration"):
            row["speedup"] = row["level_ms_per_iteration"] / row["lds_ms_per_iteration"]
        log(f"[tiny] {row}")
        out.append(row)
    return out


def run_warm(cfr, torch, args, log):
    """Learned warm start: train the network on average strategies of solved subgames (their own
    payoff seeds, so nothing about the test payoffs can be memorised), pick the regret scale on a
    validation batch, then solve the held-out test batch cold, warm and with the untrained
    network."""
    import gamegen as gg
    from paper_2609_11923_amd import warm
    rule, order = WARM_RULES[args.warm_rule]
    kw = dict(rule=rule, order=order)
    t0 = time.perf_counter()
    tr_specs = gg.random_subgames(args.warm_train_games, seed=1, lo=1e3, hi=args.warm_train_hi, game_seed=1)
    X, T, W, N, dstats = warm.make_training_set(tr_specs, args.warm_target_iters, torch, probe=args.warm_probe,
                                                solver_kw=kw, log=log)
    va_specs = gg.random_subgames(args.warm_val_games, seed=2, lo=1e3, hi=1e6, game_seed=2)
    Xv, Tv, Wv, Nv, vstats = warm.make_training_set(va_specs, args.warm_target_iters, torch, probe=args.warm_probe,
                                                    solver_kw=kw, log=log)
    t_data = time.perf_counter() - t0
    sizes = [(cfr.CFR_FEATURES, 256), (256, 256), (256, 256), (256, cfr.CFR_MLP_OUT)]
    theta0 = gg.mlp_init(sizes, seed=0)
    mlp = cfr.Mlp()
    mlp.set_params(theta0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"[warm] weighted target entropy (the loss floor): train {dstats['target_entropy']:.4f}, "
        f"validation {vstats['target_entropy']:.4f}")
    hist = warm.train(mlp, X, T, W, N, torch, epochs=args.warm_epochs, lr=args.warm_lr, val=(Xv, Tv, Wv, Nv), log=log)
    t_train = time.perf_counter() - t1
    steps = hist[-1]["steps"] if hist else 0
    del X, T, W, N
    log("[warm] choosing the regret scale on the validation batch")
    val_games = warm.subgames(va_specs)
    scale, table = warm.choose_scale(val_games, torch, mlp, args.warm_scales, args.warm_val_iters,
                                     probe=args.warm_probe, solver_kw=kw, add=args.warm_add, log=log)
    control = cfr.Mlp()
    control.set_params(theta0)
    log("[warm] evaluating on the held-out test batch")
    test_games, _ = batch_games(args.batch_games, args.seed)
    ev = warm.evaluate(test_games, torch, mlp, scale, args.warm_max_iters, control=control, probe=args.warm_probe,
                       solver_kw=kw, add=args.warm_add, log=log, retire=True)
    cold, wst = ev["cold"]["_cross"], ev["warm"]["_cross"]
    both = np.isfinite(cold) & np.isfinite(wst)
    # throughput of the network on the matrix cores: one forward over every test set's row
    log("[warm] timing inference")
    rows = warm.Rows(test_games, torch)
    s = cfr.Solver(test_games, **kw)
    rows.features(s, probe=args.warm_probe)
    z = torch.empty(rows.I, 4, dtype=torch.float32, device="cuda")
    mlp.forward(rows.x, rows.I, z)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        mlp.forward(rows.x, rows.I, z)
    e1.record()
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 5
    hidden_flops = 2.0 * rows.I * sum(fi * fo for fi, fo in sizes[:-1])
    s.close()
    out = {
        "threshold": "exploitability <= 1e-3 pot (device best response, FP64)",
        "test": f"{len(test_games)} held-out subgames (the batched workload), up to {args.warm_max_iters} iterations",
        "network": "128 -> 3 x 256 ReLU -> 4, BF16 MFMA, FP32 accumulation, Adam on FP32 master weights",
        "probe_iterations": args.warm_probe,
        "rule": args.warm_rule,
        "injection": "added to the probe's regrets" if args.warm_add else "replaces the probe's regrets",
        "train": {"subgames": dstats["subgames"], "edges": dstats["edges"], "rows": dstats["rows"],
                  "target_entropy": dstats["target_entropy"], "val_target_entropy": vstats["target_entropy"],
                  "lr": args.warm_lr, "weights": "regret unit m(I), normalised per subgame",
                  "target_iterations": args.warm_target_iters, "epochs": args.warm_epochs, "steps": steps,
                  "batch": 4096, "data_s": t_data, "train_s": t_train, "history": hist,
                  "train_tflops": 3 * 2.0 * steps * 4096 * sum(fi * fo for fi, fo in sizes) / max(t_train, 1e-9) / 1e12},
        "scale": scale, "scale_search": table,
        "cold": {k: v for k, v in ev["cold"].items() if not k.startswith("_")},
        "warm": {k: v for k, v in ev["warm"].items() if not k.startswith("_")},
        "control_untrained_net": {k: v for k, v in ev["control_untrained_net"].items() if not k.startswith("_")},
        "schedule": ev["schedule"],
        "paired": {"games_both_reached": int(both.sum()),
                   "iteration_ratio_median": float(np.median(wst[both] / cold[both])) if both.any() else None,
                   "warm_faster_fraction": float(np.mean(wst[both] < cold[both])) if both.any() else None},
        "inference": {"rows": rows.I, "ms": fwd_ms, "hidden_tflops": hidden_flops / (fwd_ms * 1e-3) / 1e12,
                      "peak_tflops_bf16": 2500.0},
    }
    c_t, w_t = out["cold"]["time_ms_median"], out["warm"]["time_ms_median"]
    out["wall_time_reduction_median"] = (1.0 - w_t / c_t) if np.isfinite(c_t) and np.isfinite(w_t) else None
    return out


def cpu_baseline(sample_fn, n_full, seconds):
    import oracle
    g = sample_fn()
    o = oracle.Oracle(g)
    o.iterate(1)
    n = 0
    t0 = time.perf_counter()
    while True:
        o.iterate(1)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    it_s_sample = n / el
    return dict(value=it_s_sample * g.n_nodes / n_full, unit="iterations/s", cores=1, kind="oracle",
                sample=f"{n} FP64 oracle iterations on {g.n_nodes} nodes in {el:.1f} s, scaled by "
                       f"{g.n_nodes}/{n_full} nodes", host=host_cpu())


def host_cpu():
    """The host's CPU model and core counts (the oracle is single-threaded: it uses one of them)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return dict(cpu_model=model, nproc=os.cpu_count(), usable_cpus=usable, oracle_threads=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--K", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--profile-iters", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iters-per-graph", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp32")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-state run of the same game")
    ap.add_argument("--direct", action="store_true", help="launch kernels directly instead of replaying a graph")
    ap.add_argument("--batch-games", type=int, default=256)
    ap.add_argument("--batch-iters", type=int, default=500)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-subgame measurement")
    ap.add_argument("--batch-schedule", choices=["level", "persistent"], default="level",
                    help="schedule of --workload batch-steps")
    ap.add_argument("--wg-nodes", type=int, default=0, help="persistent schedule: target nodes per workgroup")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm-start measurement")
    ap.add_argument("--no-rules", action="store_true", help="skip the update-rule comparison on the batch")
    ap.add_argument("--no-tiny", action="store_true", help="skip the tiny-game schedule comparison")
    ap.add_argument("--warm-train-games", type=int, default=10000)
    ap.add_argument("--warm-train-hi", type=float, default=1e6, help="largest training subgame (edges)")
    ap.add_argument("--warm-target-iters", type=int, default=500)
    ap.add_argument("--warm-val-games", type=int, default=64)
    ap.add_argument("--warm-val-iters", type=int, default=1000)
    ap.add_argument("--warm-epochs", type=int, default=8)
    ap.add_argument("--warm-lr", type=float, default=2e-3)
    ap.add_argument("--warm-probe", type=int, default=16, help="probe iterations whose strategies feed the network")
    ap.add_argument("--warm-replace", dest="warm_add", action="store_false",
                    help="replace the probe's regrets by the network's instead of adding to them")
    ap.add_argument("--warm-rule", default="cfr+", choices=["cfr+", "cfr+-alt", "dcfr-alt", "pcfr+"],
                    help="update rule of the warm-start experiment (training targets, probe and solves)")
    ap.add_argument("--warm-max-iters", type=int, default=4000)
    ap.add_argument("--warm-scales", type=float, nargs="+", default=[0.25, 0.5, 1.0, 2.0, 4.0, 8.0])
    ap.add_argument("--no-time-to-target", action="store_true", help="skip the single game's time to 1e-3 pot")
    ap.add_argument("--ttt-max-iters", type=int, default=20000)
    ap.add_argument("--no-sweep", action="store_true", help="skip the K sweep of the large game's generator")
    ap.add_argument("--sweep-K", type=int, nargs="+", default=[4, 6, 8])
    ap.add_argument("--no-mid", action="store_true", help="skip the mid game's measurements")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration for profilers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (several GPUs are a design "
              f"only: sharding by the first public card, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_11923_amd as cfr
    WARM_RULES.update({"cfr+": (cfr.CFR_RULE_CFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS),
                       "cfr+-alt": (cfr.CFR_RULE_CFR_PLUS, cfr.CFR_ORDER_ALTERNATING),
                       "dcfr-alt": (cfr.CFR_RULE_DCFR, cfr.CFR_ORDER_ALTERNATING),
                       "pcfr+": (cfr.CFR_RULE_PCFR_PLUS, cfr.CFR_ORDER_SIMULTANEOUS)})

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.workload == "warm":
        res = run_warm(cfr, torch, args, log)
        print(json.dumps({"workload": "warm", **res}), flush=True)
        return
    if args.workload == "batch-steps":
        print(json.dumps({"workload": "batch-steps", **run_batch_steps(cfr, torch, args, log)}), flush=True)
        return
    if args.workload == "mlp":
        print(json.dumps({"workload": "mlp", **run_mlp(cfr, torch, args, log)}), flush=True)
        return
    if args.workload == "batch":
        games, _ = batch_games(args.batch_games, args.seed)
        log(f"[bench] batch of {len(games)} subgames, {sum(g.n_edges for g in games)} edges")
        prec = cfr.CFR_PRECISION_FP64 if args.precision == "fp64" else cfr.CFR_PRECISION_FP32
        res, _ = run_batch(cfr, torch, games, args.batch_iters, prec, log)
        print(json.dumps({"workload": "batch", "n_games": len(games), "precision": args.precision, **res}), flush=True)
        return

    t0 = time.perf_counter()
    game, desc, sample_fn, sample_desc = make_workload(args.workload, args.K, args.seed)
    t_gen = time.perf_counter() - t0
    log(f"[bench] generated {args.workload}: {game.n_nodes} nodes in {t_gen:.1f} s")
    n_nodes = game.n_nodes
    torch.cuda.set_device(0)
    pot = float(game.pot)
    ttt = None if args.no_time_to_target else \
        (lambda sv: {"time_to_target": time_to_target(sv, torch, pot, log, args.ttt_max_iters, label=args.workload)})
    m = measure_game(cfr, torch, game, args, args.precision, log, then=ttt)
    c = m["counts"]
    out = {
        "metric": METRIC,
        "value": m["iterations_per_s"],
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_iteration"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": desc, "nodes": int(c["nodes"]), "edges": int(c["edges"]), "infosets": int(c["infosets"]),
            "slots": int(c["slots"]), "blocks": int(c["blocks"]), "update_groups": int(c["update_groups"]),
            "group_sets": int(c["group_sets"]), "rule": "CFR+, simultaneous, linear averaging",
            "state": ("FP64" if args.precision == "fp64" else "FP32") + " reach/values/regrets/strategy, FP64 strategy sums",
            "graph": f"{args.iters_per_graph} iteration(s) per hipGraph",
        },
        "roofline": m["roofline"],
        # whole iteration: the design bytes of all its kernels over the measured iteration time, and
        # the method's per-unit figures for reference
        "hbm_gbps_design_bytes": m["hbm_gbps_design_bytes"],
        "frac_design_bytes": m["frac_design_bytes"],
        "design_bytes_per_iteration": m["design_bytes_per_iteration"],
        "gbps_method_bytes": m["gbps_method_bytes"],
        "method_bytes_per_iteration": m["method_bytes_per_iteration"],
        "kernels": m["kernels"],
        "setup_s": {"generate": t_gen, "compile": m["compile_s"], "warmup_and_capture": m["warmup_s"]},
        "exploitability_after": m["exploitability_after"],
        "device_bytes": int(c["device_bytes"]),
    }
    if args.precision == "fp32" and not args.no_fp64:
        # the same game with FP64 state (the configuration held to the full parity bar)
        f64 = measure_game(cfr, torch, game, args, "fp64", log)
        out["fp64_state"] = {k: f64[k] for k in ("iterations_per_s", "ms_per_iteration", "hbm_gbps_design_bytes",
                                                  "frac_design_bytes", "roofline", "exploitability_after")}
    if "time_to_target" in m:
        t = dict(m["time_to_target"], rule="CFR+, simultaneous, linear averaging", state=out["config"]["state"])
        out["time_to_target_single_game"] = t
        if not args.no_rules and args.precision == "fp32":
            # the same game under the rule that reaches the target soonest on the subgame batch
            t0 = time.perf_counter()
            sv = cfr.Solver(game, rule=cfr.CFR_RULE_DCFR, order=cfr.CFR_ORDER_ALTERNATING)
            compile_s = time.perf_counter() - t0
            r = time_to_target(sv, torch, pot, log, args.ttt_max_iters, label=f"{args.workload} dcfr-alt")
            sv.close()
            del sv
            torch.cuda.empty_cache()
            out["time_to_target_single_game_rules"] = {
                "DCFR alternating": dict(r, state=out["config"]["state"], compile_s=compile_s)}
    del game
    torch.cuda.empty_cache()
    if args.workload == "large" and not args.no_sweep:
        out["size_sweep"] = run_size_sweep(cfr, torch, args, log)
    if args.workload == "large" and not args.no_mid:
        out["mid_game"] = run_mid(cfr, torch, args, log)
    if not args.no_batch:
        games, bspecs = batch_games(args.batch_games, args.seed)
        log(f"[bench] batch of {len(games)} subgames, {sum(g.n_edges for g in games)} edges")
        res, _ = run_batch(cfr, torch, games, args.batch_iters, cfr.CFR_PRECISION_FP32, log)
        out["batch"] = {"workload": f"{len(games)} subgames cut at round-B public states, 1e3-1e6 edges "
                                    f"log-uniform, Dirichlet(1) ranges", "precision": "fp32", **res}
        if not args.no_rules:
            out["batch"]["rules"] = run_rules(cfr, torch, games, log)
        out["batch"]["lifecycle"] = run_lifecycle(cfr, torch, games, bspecs, log)
        del games
    if not args.no_tiny:
        out["tiny_games"] = run_tiny(cfr, torch, log)
    if not args.no_warm:
        out["warm_start"] = run_warm(cfr, torch, args, log)
    if "batch" in out and "warm_start" in out:
        # the same 256 subgames three ways, CFR+ to exploitability <= 1e-3 pot for every game
        plain = out["batch"]["one_at_a_time"]["time_to_1e3pot_all_ms"]
        cold = out["warm_start"]["cold"]["time_ms_all"]
        warm_ = out["warm_start"]["warm"]["time_ms_all"]
        out["time_to_target"] = {
            "what": "wall time until every one of the 256 subgames reaches exploitability <= 1e-3 pot (CFR+)",
            "plain_cold_one_at_a_time_ms": plain, "batched_cold_ms": cold, "batched_warm_ms": warm_,
            "reduction_batched_warm_vs_plain_cold": 1.0 - warm_ / plain if plain else None,
            "reduction_batched_warm_vs_batched_cold": 1.0 - warm_ / cold if cold else None,
            "model": "crossing iterations (log-log interpolated between checkpoints) x measured ms per iteration, "
                     "plus the warm start's measured time",
        }
        rc_ = out["warm_start"]["cold"].get("retiring", {}).get("time_ms_all")
        rw_ = out["warm_start"]["warm"].get("retiring", {}).get("time_ms_all")
        if rc_ and rw_:
            # each game retired once it reached the target (the one-at-a-time baseline stops each game
            # at its own crossing too)
            out["time_to_target"]["retiring"] = {
                "batched_cold_ms": rc_, "batched_warm_ms": rw_,
                "reduction_batched_warm_vs_plain_cold": 1.0 - rw_ / plain if plain else None,
                "reduction_batched_warm_vs_batched_cold": 1.0 - rw_ / rc_,
            }
        sw_c = out["warm_start"]["cold"].get("stopwatch")
        sw_w = out["warm_start"]["warm"].get("stopwatch")
        if sw_c and sw_w:
            # the same two solves run straight through until every game is at the target, timed whole
            out["time_to_target"]["stopwatch"] = {
                "batched_cold": sw_c, "batched_warm": sw_w,
                "reduction_batched_warm_vs_plain_cold": 1.0 - sw_w["ms_events"] / plain if plain else None,
                "reduction_batched_warm_vs_batched_cold": 1.0 - sw_w["ms_events"] / sw_c["ms_events"],
            }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(sample_fn, n_nodes, args.cpu_seconds)
        t = out.get("time_to_target_single_game")
        if t and t.get("reached"):
            # the oracle's time to the same crossing iteration, from its measured rate (not run)
            t["oracle_s_extrapolated"] = t["iterations"] / out["cpu_baseline"]["value"]
            t["oracle_note"] = "extrapolated: crossing iterations / the oracle's measured iterations per second"
    print(json.dumps(out), flush=True)


def run_size_sweep(cfr, torch, args, log):
    """The large game's generator at K = 4, 6, 8 hands per player (K = 10 is the headline): iterations
    per second and the dominant kernel's roofline at each size."""
    import gamegen as gg
    out = []
    for K in args.sweep_K:
        if K == args.K:
            continue
        h1, h2 = gg.sample_hands(K, args.seed)
        g = gg.large(K, seed=args.seed, hands=(h1, h2))
        log(f"[bench] size sweep K={K}: {g.n_nodes} nodes")
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup, sub.traffic_workload = max(20, args.steps), args.warmup, f"large_K{K}"
        m = measure_game(cfr, torch, g, sub, "fp32", log)
        out.append(dict(K=K, nodes=int(m["counts"]["nodes"]), infosets=int(m["counts"]["infosets"]),
                        ms_per_iteration=m["ms_per_iteration"], iterations_per_s=m["iterations_per_s"],
                        frac_design_bytes=m["frac_design_bytes"], roofline=m["roofline"]))
        del g
        torch.cuda.empty_cache()
    return out


def run_mid(cfr, torch, args, log):
    """The mid game (Leduc rules, 13 ranks x 2 suits): FP32 state, ms per iteration with 1 and with 10
    iterations per hipGraph, and its time to exploitability <= 1e-3 pot (pot 2) under CFR+."""
    import gamegen as gg
    g = gg.leduc(13, 2)
    pot = float(g.pot)
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup, sub.traffic_workload = 1000, 50, "mid"
    out = {"workload": "Leduc-rule game, 13 ranks x 2 suits (1,179,777 nodes), FP32 state, CFR+ simultaneous"}
    for k in (1, 10):
        then = (lambda sv: {"time_to_target": time_to_target(sv, torch, pot, log, 20000, label="mid")}) if k == 1 \
            else None
        m = measure_game(cfr, torch, g, sub, "fp32", log, iters_per_graph=k, then=then, profile=(k == 1))
        rec = dict(iters_per_graph=k, ms_per_iteration=m["ms_per_iteration"], iterations_per_s=m["iterations_per_s"])
        if "roofline" in m:
            rec["roofline"] = m["roofline"]
        out[f"graph_{k}"] = rec
        if "time_to_target" in m:
            out["time_to_target"] = m["time_to_target"]
    return out


if __name__ == "__main__":
    main()
