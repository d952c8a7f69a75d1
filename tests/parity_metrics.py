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
