"""Comparison metrics shared by the GPU parity tests (test infrastructure; imports only the oracle's
arrays and the input generator, never the library).

rel_err       normwise relative error max_k |x_k - ref_k| / max_k |ref_k|: the method's stated metric
              for regrets and strategies (applied per tensor).
set_reach     pi^s(I) = sum over the members h of I of pi^s(h), where pi^s(h) is the product of the
              chance probabilities and of both players' action probabilities on the path to h under
              the profile s (paper Sec. 3, eq. reach; the reach of an information set is the sum over
              its members): how often play under s visits I.
weighted_err  max_q w(I(q)) |x_q - ref_q|: the error of slot q weighted by the reach of its set.  A
              strategy error at a set that the average profile almost never visits moves every
              expected payoff by at most that reach times the payoff range, so this is the error that
              exploitability can see.
jitter        a game with every terminal payoff moved by up to eps (seeded): inputs that differ at a
              chosen rounding level.
"""
import dataclasses

import numpy as np


def rel_err(x, ref):
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.abs(np.asarray(x, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-30))


def canonical_order(game):
    """Input node id of every canonical node and the index into children[]/prob[] of the edge into it
    (-1 at the root): breadth-first from the root, children in action order (the canonical numbering)."""
    cb = np.asarray(game.child_begin, np.int64)
    nc = np.asarray(game.n_children, np.int64)
    ch = np.asarray(game.children, np.int64)
    order, edge = [np.array([int(getattr(game, "root", 0))])], [np.array([-1])]
    while True:
        f = order[-1]
        k = nc[f]
        tot = int(k.sum())
        if tot == 0:
            break
        idx = np.repeat(cb[f], k) + (np.arange(tot) - np.repeat(np.cumsum(k) - k, k))
        order.append(ch[idx])
        edge.append(idx)
    return np.concatenate(order), np.concatenate(edge)


def set_reach(game, layout, profile):
    """pi^profile(I) for every information set I (canonical numbering of `layout`, the oracle's arrays),
    profile in canonical slot order."""
    gid, eidx = canonical_order(game)
    nt = layout["node_type"]
    assert np.array_equal(np.asarray(game.type)[gid], nt), "breadth-first order differs from the canonical arrays"
    prob = np.asarray(game.prob, np.float64)
    par, ins, do = layout["parent"], layout["in_slot"], layout["depth_off"]
    pi = np.ones(len(gid))
    for d in range(1, len(do) - 1):
        k = np.arange(do[d], do[d + 1])
        p = par[k]
        m = np.where(nt[p] == 0, prob[np.maximum(eidx[k], 0)], 1.0)
        s = ins[k]
        m = np.where(s >= 0, np.asarray(profile, np.float64)[np.maximum(s, 0)], m)
        pi[k] = pi[p] * m
    mo, mn = layout["mem_off"], layout["mem_node"]
    if len(mn) == 0:
        return np.zeros(len(mo) - 1)
    return np.add.reduceat(pi[mn], mo[:-1])   # every set has at least one member


def slot_weights(layout, w_set):
    so = layout["slot_off"]
    return np.repeat(np.asarray(w_set, np.float64), np.diff(so))


def weighted_err(x, ref, w_slot, scale=1.0):
    if len(w_slot) == 0:
        return 0.0
    return float((w_slot * np.abs(np.asarray(x, np.float64) - np.asarray(ref, np.float64))).max() / scale)


def jitter(game, seed, eps=1e-3):
    rng = np.random.default_rng(seed)
    pay = np.array(game.payoff, np.float64)
    term = np.asarray(game.type) == 3
    pay[term] += eps * rng.uniform(-1, 1, int(term.sum()))
    return dataclasses.replace(game, payoff=pay)


TOL = 1e-5          # the method's bar (normwise and reach-weighted)
EXPL_TOL = 1e-6     # exploitability, times the pot
CAP = 1e-3          # a normwise tolerance at or above this pins nothing
EXPL_CAP = 1e-5     # an exploitability tolerance at or above this (times the pot) pins nothing
MULT = 4            # tolerance over the spread of the oracle's own runs


def free_run_compare(game, s, o, T, precision, control, perturb_inputs, current=True, note=print):
    """Compare solver s with oracle o (FP64) after T free-running iterations.

    Six state metrics -- normwise (rel_err) and reach-weighted (weighted_err, weights from the oracle's
    average profile) errors of the regrets (over max |R|), the average and the current strategy -- and
    exploitability.  The tolerance of each comes from how far runs of the same method in the same
    precision spread around the FP64 run on this game, measured on the oracle: control(game, f32_state,
    reverse) returns a finished run.  Samples: FP32 state in the default and the reverse summation order
    (FP64: reverse order only); with perturb_inputs also on payoffs moved by up to one unit of rounding
    of the precision (1e-7 FP32, 1e-15 FP64; three seeds, both orders), which models the library rounding the
    chance-folded template once per terminal (games with exact payoff ties are left out: such a move
    breaks ties the library keeps).  tol = max(bar, MULT x spread): the bar (TOL, EXPL_TOL pot) wherever
    the method's own runs agree to better than a quarter of it.

    Exploitability and the average profile's value are checked first; if their tolerance reaches
    EXPL_CAP pot nothing is pinnable and the cell is an expected failure.  Then each state metric whose
    tolerance is below CAP is asserted -- except that the reach-weighted regret and current-strategy
    errors are held only where their normwise counterparts are (where those are not, regret matching has
    switched sets between pure and mixed strategies along the run, and a few samples cannot bound where);
    anything not asserted makes the cell an expected failure naming the measured spread (the one-step
    test pins every such cell at every iteration)."""
    import pytest
    R, _ = s.state()
    avg, cur = s.strategy(average=True), s.strategy(average=False)
    Ro, _, sco, sao = o.state()
    e, _, _, v = s.exploitability()
    eo, _, _, vo = o.exploitability()
    lay = o.layout()
    w = slot_weights(lay, set_reach(game, lay, sao))
    scale_R = max(float(np.abs(Ro).max()), 1e-30)

    def metrics(Rx, ax, cx):
        return dict(regrets=rel_err(Rx, Ro), average=rel_err(ax, sao), current=rel_err(cx, sco),
                    w_regrets=weighted_err(Rx, Ro, w, scale_R), w_average=weighted_err(ax, sao, w),
                    w_current=weighted_err(cx, sco, w))

    got = metrics(R, avg, cur)
    f32 = precision == "fp32"
    samples = [control(game, True, False), control(game, True, True)] if f32 else [control(game, False, True)]
    if perturb_inputs:
        scale = max(1.0, float(np.abs(game.payoff).max()))
        eps = 1e-7 if f32 else 1e-15
        samples += [control(jitter(game, sd, eps * scale), f32, rev) for sd in (5, 6, 7) for rev in (False, True)]
    spread = {k: 0.0 for k in got}
    sp_e = 0.0
    for c in samples:
        Rc, _, scc, sac = c.state()
        for k, x in metrics(Rc, sac, scc).items():
            spread[k] = max(spread[k], x)
        sp_e = max(sp_e, abs(c.exploitability()[0] - eo))
    te = max(EXPL_TOL * game.pot, MULT * sp_e)
    note(f"  {len(samples)} oracle runs spread: " + " ".join(f"{k} {x:.1e}" for k, x in spread.items()) +
         f" expl {sp_e:.1e}")
    note(f"  gpu: " + " ".join(f"{k} {x:.2e}" for k, x in got.items()) + f" expl {e:.9e} vs {eo:.9e}")
    if te >= EXPL_CAP * game.pot:
        pytest.xfail(f"{precision} free run: the oracle's own runs differ in exploitability by {sp_e:.1e} after {T} "
                     f"iterations (regrets {spread['regrets']:.1e}, average {spread['average']:.1e}): nothing to "
                     f"pin; the one-step test pins this cell (gpu: expl {e:.4e} vs {eo:.4e}, regrets "
                     f"{got['regrets']:.1e}, average {got['average']:.1e})")
    assert abs(e - eo) <= te and abs(v - vo) <= te
    tol = {k: max(TOL, MULT * x) for k, x in spread.items()}
    unpinned = []
    # the average strategy is the solver's output: its reach-weighted error is held wherever its own
    # tolerance allows; regrets and the current strategy are internal state whose free-run divergence is
    # regret matching switching sets, so their reach-weighted error is held where the normwise one is
    groups = [("average", ["average"], ["w_average"]), ("regrets", ["regrets"], ["w_regrets"])]
    if current:
        groups.append(("current", ["current"], ["w_current"]))
    for name, norm, wtd in groups:
        keys = wtd + (norm if tol[norm[0]] < CAP else [])
        if tol[norm[0]] >= CAP and name != "average":
            keys = []
        for k in norm + wtd:
            if k in keys and tol[k] < CAP:
                assert got[k] <= tol[k], (k, got[k], tol[k])
            else:
                unpinned.append(f"{k} {got[k]:.1e} (own runs {spread[k]:.1e})")
    if unpinned:
        pytest.xfail(f"{precision} free run: the oracle's own runs spread too far to pin " + ", ".join(unpinned) +
                     "; exploitability and the other metrics are pinned, the one-step test pins the rest")
