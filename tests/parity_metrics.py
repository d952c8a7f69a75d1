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

    The tolerance of each quantity comes from how far runs of the same method in the same precision
    spread around the FP64 run on this game, measured on the oracle: control(game, f32_state, reverse)
    returns a finished run of it.  Samples: FP32 state in the default and the reverse summation order
    (FP64: reverse order only); with perturb_inputs also on payoffs moved by up to one unit of
    rounding of the precision (1e-7 FP32, 1e-15 FP64, two seeds), which models the library rounding
    the chance-folded template once per terminal (games with exact payoff ties are left out: such a
    move breaks ties the library keeps).  tol = max(bar, MULT x spread).

    Hard checks: exploitability and the average profile's value within their tolerance (< EXPL_CAP
    pot), the reach-weighted average strategy <= TOL, and every normwise quantity whose tolerance is
    below CAP.  A cell where exploitability itself spreads beyond EXPL_CAP, or any normwise tolerance
    reaches CAP, cannot be pinned by a free run: it is recorded as an expected failure with the
    measured spread (the one-step test pins such cells at every iteration); the reach-weighted regret
    and current-strategy errors are asserted only when every normwise quantity is pinned."""
    import pytest
    R, _ = s.state()
    avg, cur = s.strategy(average=True), s.strategy(average=False)
    Ro, _, sco, sao = o.state()
    e, _, _, v = s.exploitability()
    eo, _, _, vo = o.exploitability()
    eR, eavg, ecur = rel_err(R, Ro), rel_err(avg, sao), rel_err(cur, sco)
    f32 = precision == "fp32"
    samples = [control(game, True, False), control(game, True, True)] if f32 else [control(game, False, True)]
    if perturb_inputs:
        scale = max(1.0, float(np.abs(game.payoff).max()))
        eps = 1e-7 if f32 else 1e-15
        samples += [control(jitter(game, sd, eps * scale), f32, False) for sd in (5, 6)]
    sp = [0.0, 0.0, 0.0, 0.0]
    for c in samples:
        Rc, _, scc, sac = c.state()
        sp = [max(sp[0], rel_err(Rc, Ro)), max(sp[1], rel_err(sac, sao)), max(sp[2], rel_err(scc, sco)),
              max(sp[3], abs(c.exploitability()[0] - eo))]
    tR, tavg, tcur = (max(TOL, MULT * x) for x in sp[:3])
    te = max(EXPL_TOL * game.pot, MULT * sp[3])
    note(f"  spread over {len(samples)} oracle runs: R {sp[0]:.1e} avg {sp[1]:.1e} cur {sp[2]:.1e} expl {sp[3]:.1e}; "
         f"gpu R {eR:.2e} avg {eavg:.2e} cur {ecur:.2e} expl {e:.9e} vs {eo:.9e}")
    if te >= EXPL_CAP * game.pot:
        pytest.xfail(f"{precision} free run: the oracle's own runs differ in exploitability by {sp[3]:.1e} after {T} "
                     f"iterations (R {sp[0]:.1e}, average {sp[1]:.1e}): nothing to pin; the one-step test pins "
                     f"this cell (gpu: expl {e:.4e} vs {eo:.4e}, R {eR:.1e}, average {eavg:.1e})")
    assert abs(e - eo) <= te and abs(v - vo) <= te
    lay = o.layout()
    w = slot_weights(lay, set_reach(game, lay, sao))
    wavg, wcur = weighted_err(avg, sao, w), weighted_err(cur, sco, w)
    wR = weighted_err(R, Ro, w, max(float(np.abs(Ro).max()), 1e-30))
    note(f"  reach-weighted R {wR:.2e} avg {wavg:.2e} cur {wcur:.2e}; tol R {tR:.1e} avg {tavg:.1e} cur {tcur:.1e} "
         f"expl {te:.1e}")
    assert wavg <= TOL
    checks = [("regrets", eR, tR, sp[0]), ("average", eavg, tavg, sp[1])] + \
             ([("current", ecur, tcur, sp[2])] if current else [])
    unpinned = []
    for name, err, tol, spread in checks:
        if tol < CAP:
            assert err <= tol, name
        else:
            unpinned.append(f"{name} {err:.1e} (own runs {spread:.1e})")
    if unpinned:
        pytest.xfail(f"{precision} free run: the oracle's own runs spread too far to pin " + ", ".join(unpinned) +
                     "; exploitability and the reach-weighted average are pinned, the one-step test pins the rest")
    assert wR <= TOL and wcur <= TOL
