"""Sequence-form LP equilibrium of a two-player zero-sum game (TEST INFRASTRUCTURE ONLY).

Independent of the CFR recursion: it solves the game exactly with the
sequence-form linear program (Koller, Megiddo and von Stengel) using scipy's
HiGHS solver.  Player 1 maximises over realization plans x with E x = e,
x >= 0, the dual of player 2's best response:

    max_{x, q}  q_root   s.t.  F^T q - A^T x <= 0,   E x = e,   x >= 0,

where A[s1, s2] = sum over terminals z with sequences (s1, s2) of
pi_c(z) u(z).  Player 2's program is the mirror image.  The optimum is the
game value for player 1; the optimal plans give behavioural strategies
sigma(I, a) = x(I, a) / x(parent sequence of I).
"""
from __future__ import annotations

import numpy as np
import scipy.optimize
import scipy.sparse as sp


def sequences(lay: dict):
    """Per canonical node, the index of each player's last own sequence on its path
    (0 = empty sequence, 1 + k = k-th slot of that player in slot order)."""
    N = lay["node_type"].shape[0]
    parent, in_slot, ntype = lay["parent"], lay["in_slot"], lay["node_type"]
    slot_off, iset_player = lay["slot_off"], lay["iset_player"]
    I = iset_player.shape[0]
    A = int(slot_off[-1]) if I else 0
    slot_player = np.zeros(A, np.int8)
    for i in range(I):
        slot_player[slot_off[i]:slot_off[i + 1]] = iset_player[i]
    seq_index = {1: {}, 2: {}}
    for q in range(A):
        p = int(slot_player[q])
        seq_index[p][q] = len(seq_index[p]) + 1
    seq = np.zeros((N, 2), np.int64)
    for h in range(1, N):
        p = parent[h]
        seq[h] = seq[p]
        q = in_slot[h]
        if q >= 0:
            pl = int(ntype[p])
            seq[h, pl - 1] = seq_index[pl][int(q)]
    return seq, seq_index, slot_player


def solve(lay: dict, payoff_folded: np.ndarray):
    """payoff_folded: per canonical node, pi_c(z) u(z) at terminals (float64).
    Returns (value, sigma) with sigma a behavioural profile in canonical slot order."""
    seq, seq_index, slot_player = sequences(lay)
    ntype = lay["node_type"]
    slot_off, iset_player = lay["slot_off"], lay["iset_player"]
    mem_off, mem_node = lay["mem_off"], lay["mem_node"]
    I = iset_player.shape[0]
    n1, n2 = len(seq_index[1]) + 1, len(seq_index[2]) + 1
    term = np.nonzero(ntype == 3)[0]
    Am = sp.coo_matrix((payoff_folded[term], (seq[term, 0], seq[term, 1])), shape=(n1, n2)).tocsr()

    def constraints(player):
        rows, cols, vals = [0], [0], [1.0]
        par = []
        r = 1
        for i in range(I):
            if iset_player[i] != player:
                continue
            h = int(mem_node[mem_off[i]])
            ps = int(seq[h, player - 1])
            par.append((i, ps))
            for q in range(slot_off[i], slot_off[i + 1]):
                rows.append(r); cols.append(seq_index[player][q]); vals.append(1.0)
            rows.append(r); cols.append(ps); vals.append(-1.0)
            r += 1
        n = n1 if player == 1 else n2
        M = sp.coo_matrix((vals, (rows, cols)), shape=(r, n)).tocsr()
        rhs = np.zeros(r)
        rhs[0] = 1.0
        return M, rhs, par

    E, e, par1 = constraints(1)
    F, f, par2 = constraints(2)
    m1, m2 = E.shape[0], F.shape[0]
    # player 1: variables [x (n1), q (m2)], minimise -f.q
    c = np.concatenate([np.zeros(n1), -f])
    A_ub = sp.hstack([-Am.T, F.T]).tocsr()
    A_eq = sp.hstack([E, sp.csr_matrix((m1, m2))]).tocsr()
    bounds = [(0, None)] * n1 + [(None, None)] * m2
    r1 = scipy.optimize.linprog(c, A_ub=A_ub, b_ub=np.zeros(n2), A_eq=A_eq, b_eq=e, bounds=bounds, method="highs")
    assert r1.status == 0, r1.message
    x = r1.x[:n1]
    v1 = -r1.fun
    # player 2: variables [y (n2), p (m1)], minimise e.p  s.t.  A y - E^T p <= 0
    c2 = np.concatenate([np.zeros(n2), e])
    A_ub2 = sp.hstack([Am, -E.T]).tocsr()
    A_eq2 = sp.hstack([F, sp.csr_matrix((m2, m1))]).tocsr()
    bounds2 = [(0, None)] * n2 + [(None, None)] * m1
    r2 = scipy.optimize.linprog(c2, A_ub=A_ub2, b_ub=np.zeros(n1), A_eq=A_eq2, b_eq=f, bounds=bounds2,
                                method="highs")
    assert r2.status == 0, r2.message
    y = r2.x[:n2]
    v2 = r2.fun
    A = int(slot_off[-1]) if I else 0
    sigma = np.zeros(A)
    for player, plan, par in ((1, x, par1), (2, y, par2)):
        for i, ps in par:
            mass = plan[ps]
            lo, hi = slot_off[i], slot_off[i + 1]
            if mass > 1e-12:
                for q in range(lo, hi):
                    sigma[q] = max(plan[seq_index[player][q]], 0.0) / mass
                s = sigma[lo:hi].sum()
                sigma[lo:hi] /= s
            else:
                sigma[lo:hi] = 1.0 / (hi - lo)
    return 0.5 * (v1 + v2), sigma, (v1, v2)


def folded_payoffs(lay: dict, game) -> np.ndarray:
    """pi_c(z) u(z) per canonical node in float64, from the game's own chance probabilities."""
    # canonical order is breadth-first from the root with children in action order
    order = [int(game.root)]
    head = 0
    while head < len(order):
        h = order[head]; head += 1
        b, n = int(game.child_begin[h]), int(game.n_children[h])
        order.extend(int(c) for c in game.children[b:b + n])
    pic = {order[0]: 1.0}
    out = np.zeros(len(order))
    for k, h in enumerate(order):
        b, n = int(game.child_begin[h]), int(game.n_children[h])
        for a in range(n):
            c = int(game.children[b + a])
            pic[c] = pic[h] * (float(game.prob[b + a]) if game.type[h] == 0 else 1.0)
        if game.type[h] == 3:
            out[k] = pic[h] * float(game.payoff[h])
    return out
