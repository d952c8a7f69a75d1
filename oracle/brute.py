"""Brute-force checks on tiny games (TEST INFRASTRUCTURE ONLY; pure Python loops).

These compute the quantities of the paper's Section 3 a second, unrelated way:
by enumerating terminal paths instead of recursing over the tree.

* ``paths(game)``: for every terminal z its chance product pi_c(z), payoff
  u(z) and the list of (player, information set, slot, action) decisions on
  its path.
* ``root_value``: sum_z pi_c(z) pi_1(z) pi_2(z) u(z) (Proposition 1's right
  hand side at the root).
* ``best_response``: the maximum over ALL pure strategies of one player of
  that player's expected payoff against a fixed opponent profile.
* ``cfr``: CFR / CFR+ whose counterfactual values are terminal sums,
  v_i(I,a) = sum over terminals z below (h, a), h in I, of
  pi_c(z) pi_{-i}(z) pi_i(h.a -> z) u_i(z)   (eq. cfv),
  with regret, regret matching and the reach-weighted average of eqs.
  (regret) and (rm).
"""
from __future__ import annotations

import itertools

import numpy as np


def paths(game):
    """Terminal paths keyed by the game's own node ids.  Information sets are
    identified by key; slots are numbered by first occurrence in breadth-first
    order (the same rule the canonical arrays use) so results line up."""
    order = [int(game.root)]
    head = 0
    while head < len(order):
        h = order[head]; head += 1
        b, n = int(game.child_begin[h]), int(game.n_children[h])
        order.extend(int(c) for c in game.children[b:b + n])
    iset_of_key, isets = {}, []   # isets: (player, nA, first_slot)
    nslots = 0
    for h in order:
        ty = int(game.type[h])
        if ty in (1, 2):
            k = int(game.key[h])
            if k not in iset_of_key:
                iset_of_key[k] = len(isets)
                isets.append((ty, int(game.n_children[h]), nslots))
                nslots += int(game.n_children[h])
    out = []

    def rec(h, pic, decs):
        ty = int(game.type[h])
        b, n = int(game.child_begin[h]), int(game.n_children[h])
        if ty == 3:
            out.append((pic, float(game.payoff[h]), list(decs)))
            return
        for a in range(n):
            c = int(game.children[b + a])
            if ty == 0:
                rec(c, pic * float(game.prob[b + a]), decs)
            else:
                i = iset_of_key[int(game.key[h])]
                decs.append((ty, i, isets[i][2] + a, a))
                rec(c, pic, decs)
                decs.pop()

    rec(int(game.root), 1.0, [])
    return out, isets, nslots


def root_value(P, prof):
    tot = 0.0
    for pic, u, decs in P:
        p = pic
        for _, _, q, _ in decs:
            p *= prof[q]
        tot += p * u
    return tot


def best_response(P, isets, player, prof):
    """max over pure strategies of `player` of its expected payoff (u_2 = -u)."""
    own = [i for i, (pl, _, _) in enumerate(isets) if pl == player]
    sign = 1.0 if player == 1 else -1.0
    best = -np.inf
    for choice in itertools.product(*[range(isets[i][1]) for i in own]):
        pick = dict(zip(own, choice))
        tot = 0.0
        for pic, u, decs in P:
            p = pic
            for pl, i, q, a in decs:
                if pl == player:
                    if pick[i] != a:
                        p = 0.0
                        break
                else:
                    p *= prof[q]
            tot += p * sign * u
        best = max(best, tot)
    return best


def regret_match(R, isets):
    sig = np.zeros_like(R)
    for pl, nA, s in isets:
        pos = np.maximum(R[s:s + nA], 0.0)
        t = pos.sum()
        sig[s:s + nA] = pos / t if t > 0 else 1.0 / nA
    return sig


def cfr(P, isets, nslots, T, plus=True, linear=True, rule=None):
    """Simultaneous CFR / CFR+ / DCFR / PCFR+ by terminal sums; returns (R, sbar).  rule (None:
    CFR+ if plus else CFR) follows the published definitions: DCFR discounts positive regrets
    by t^1.5/(t^1.5+1), negative ones by 1/2 and the strategy sums by (t/(t+1))^2 after adding;
    PCFR+ plays regret matching of R + (last instantaneous regret) and averages with weight t^2."""
    rule = rule or ("cfr+" if plus else "cfr")
    R = np.zeros(nslots)
    S = np.zeros(nslots)
    pred = np.zeros(nslots)
    for t in range(1, T + 1):
        sig = regret_match(R + pred if rule == "pcfr+" else R, isets)
        cfv = np.zeros(nslots)
        own_reach = {}
        for pic, u, decs in P:
            for k, (pl, i, q, a) in enumerate(decs):
                sign = 1.0 if pl == 1 else -1.0
                opp = pic
                mine_before = 1.0
                mine_after = 1.0
                for kk, (pl2, _, q2, _) in enumerate(decs):
                    if pl2 != pl:
                        opp *= sig[q2]
                    elif kk < k:
                        mine_before *= sig[q2]
                    elif kk > k:
                        mine_after *= sig[q2]
                cfv[q] += opp * mine_after * sign * u
                own_reach[i] = mine_before
        for i, (pl, nA, s) in enumerate(isets):
            v = float(np.dot(sig[s:s + nA], cfv[s:s + nA]))
            r = cfv[s:s + nA] - v
            R[s:s + nA] += r
            if rule in ("cfr+", "pcfr+"):
                R[s:s + nA] = np.maximum(R[s:s + nA], 0.0)
            if rule == "dcfr":
                R[s:s + nA] *= np.where(R[s:s + nA] > 0, t ** 1.5 / (t ** 1.5 + 1), 0.5)
            if rule == "pcfr+":
                pred[s:s + nA] = r
            w = {"dcfr": 1.0, "pcfr+": float(t) * t}.get(rule, float(t) if linear else 1.0)
            # an information set every terminal path avoids has no recorded reach; its
            # average contribution is then zero (its own reach is zero under sigma)
            S[s:s + nA] += w * own_reach.get(i, 0.0) * sig[s:s + nA]
            if rule == "dcfr":
                S[s:s + nA] *= (t / (t + 1.0)) ** 2
    return R, S
