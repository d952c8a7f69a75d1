"""Seeded synthetic game builders: the inputs of every test and benchmark.

This package produces explicit game trees (node table, children, chance
probabilities, information-set keys, payoffs) and nothing else.  It holds none
of the CFR arithmetic.  Both the CFR library and the CPU oracle consume its
output; neither is imported here.

Families (all are "private deal x public tree"; an information set is
(player, own hand, public history), which gives perfect recall):

* ``kuhn()``        3-card deck, one chance node deals both cards, pass/bet,
                    ante 1, bet 1, chip payoffs.
* ``leduc(r, s)``   r ranks x s suits, P1 card then P2 card, two limit rounds
                    (raise 2 then 4, at most 2 raises per round) with one public
                    card between them; a pair with the board wins, else rank.
* ``large(K)``      36-card deck, K sampled two-card hands per player, a joint
                    deal of compatible pairs, then public card / betting round A /
                    public card / betting round B; fold, check/call, half-pot,
                    pot, at most 3 raises per round; hashed payoffs in [-1, 1].
* ``subgame(...)``  a round-B subtree of ``large`` with explicit hand lists and
                    root ranges (joint deal weighted by r1(h1) r2(h2)).
* ``random_game``   random public trees with random chance probabilities and
                    private types, used to exercise the compiler and solver on
                    arbitrary shapes.
* ``example11()``   the 11-node example game (chance root, two decisions per
                    player, six terminals) used to illustrate compilation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import weakref
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgamegen.so")

GG_CHANCE, GG_P1, GG_P2, GG_TERMINAL = 0, 1, 2, 3
LARGE_ROOT_HASH = 0xC2C2_5EED_0000_0001
DECK36 = (9, 4)


def build_lib(force: bool = False) -> str:
    """Compile libgamegen.so in place (plain C, host only)."""
    src = os.path.join(_HERE, "gamegen.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Hand(ctypes.Structure):
    _fields_ = [("card", ctypes.c_int8 * 2), ("gid", ctypes.c_int32), ("weight", ctypes.c_double)]


class _CardParams(ctypes.Structure):
    _fields_ = [
        ("n_ranks", ctypes.c_int), ("n_suits", ctypes.c_int),
        ("n_hands1", ctypes.c_int), ("n_hands2", ctypes.c_int),
        ("hands1", ctypes.POINTER(_Hand)), ("hands2", ctypes.POINTER(_Hand)),
        ("sequential_deal", ctypes.c_int), ("n_rounds", ctypes.c_int),
        ("board_before", ctypes.c_int * 4), ("n_fixed_board", ctypes.c_int),
        ("fixed_board", ctypes.c_int8 * 4), ("betting", ctypes.c_int), ("raise_cap", ctypes.c_int),
        ("raise_size", ctypes.c_double * 4), ("contrib1", ctypes.c_double), ("contrib2", ctypes.c_double),
        ("payoff_mode", ctypes.c_int), ("seed", ctypes.c_uint64), ("root_hash", ctypes.c_uint64),
        ("first_round", ctypes.c_int),
    ]


class _RandomParams(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64), ("n_types1", ctypes.c_int), ("n_types2", ctypes.c_int),
        ("max_depth", ctypes.c_int), ("p_terminal", ctypes.c_double), ("p_chance", ctypes.c_double),
        ("max_actions", ctypes.c_int), ("max_chance", ctypes.c_int),
    ]


class _GGGame(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64), ("n_edges", ctypes.c_int64),
        ("type", ctypes.POINTER(ctypes.c_int8)), ("child_begin", ctypes.POINTER(ctypes.c_int64)),
        ("n_children", ctypes.POINTER(ctypes.c_int32)), ("children", ctypes.POINTER(ctypes.c_int64)),
        ("prob", ctypes.POINTER(ctypes.c_double)), ("key", ctypes.POINTER(ctypes.c_int64)),
        ("payoff", ctypes.POINTER(ctypes.c_double)), ("pub", ctypes.POINTER(ctypes.c_int64)),
        ("n_pub", ctypes.c_int64), ("pot_at_root", ctypes.c_double),
        ("pub_type", ctypes.POINTER(ctypes.c_int8)), ("pub_c1", ctypes.POINTER(ctypes.c_double)),
        ("pub_c2", ctypes.POINTER(ctypes.c_double)), ("pub_round", ctypes.POINTER(ctypes.c_int8)),
        ("pub_depth", ctypes.POINTER(ctypes.c_int8)), ("pub_parent", ctypes.POINTER(ctypes.c_int32)),
        ("pub_sym", ctypes.POINTER(ctypes.c_int8)),
        ("pair", ctypes.POINTER(ctypes.c_int32)), ("pair_h1", ctypes.POINTER(ctypes.c_int32)),
        ("pair_h2", ctypes.POINTER(ctypes.c_int32)), ("n_pairs", ctypes.c_int64),
        ("error", ctypes.c_int), ("msg", ctypes.c_char * 160),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_lib())
        lib.gg_build_card.argtypes = [ctypes.POINTER(_CardParams), ctypes.POINTER(_GGGame)]
        lib.gg_build_random.argtypes = [ctypes.POINTER(_RandomParams), ctypes.POINTER(_GGGame)]
        lib.gg_free.argtypes = [ctypes.POINTER(_GGGame)]
        lib.gg_hash_step.argtypes = [ctypes.c_uint64, ctypes.c_int]
        lib.gg_hash_step.restype = ctypes.c_uint64
        lib.gg_splitmix64.argtypes = [ctypes.c_uint64]
        lib.gg_splitmix64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def hash_step(h: int, sym: int) -> int:
    return int(_load().gg_hash_step(ctypes.c_uint64(h), sym))


@dataclass
class Game:
    """Explicit game tree.  Arrays may be views of C-owned memory kept alive by ``_owner``."""
    type: np.ndarray          # int8 [N]: 0 chance, 1 P1, 2 P2, 3 terminal
    child_begin: np.ndarray   # int64 [N]
    n_children: np.ndarray    # int32 [N]
    children: np.ndarray      # int64 [E]
    prob: np.ndarray          # float64 [E] (chance edges)
    key: np.ndarray           # int64 [N] information-set key (-1 if not a decision node)
    payoff: np.ndarray        # float64 [N] payoff to player 1 at terminals
    pub: np.ndarray           # int64 [N] public-state id (-1 on deal nodes)
    root: int = 0
    pot: float = 1.0          # exploitability unit
    name: str = ""
    meta: dict = field(default_factory=dict)
    _owner: object = None

    @property
    def n_nodes(self) -> int:
        return int(self.type.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.children.shape[0])


def _view(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).view(dtype)


class _Owner:
    def __init__(self, gg):
        self.gg = gg
        lib = _load()
        self._fin = weakref.finalize(self, lib.gg_free, ctypes.byref(gg))


def _wrap(gg: _GGGame, name: str, pot: float, meta: dict) -> Game:
    if gg.error:
        raise ValueError(f"gamegen: {gg.msg.decode()}")
    owner = _Owner(gg)
    N, E = gg.n_nodes, gg.n_edges
    g = Game(
        type=_view(gg.type, N, np.int8), child_begin=_view(gg.child_begin, N, np.int64),
        n_children=_view(gg.n_children, N, np.int32), children=_view(gg.children, E, np.int64),
        prob=_view(gg.prob, E, np.float64), key=_view(gg.key, N, np.int64),
        payoff=_view(gg.payoff, N, np.float64), pub=_view(gg.pub, N, np.int64),
        root=0, pot=pot, name=name, meta=dict(meta), _owner=owner,
    )
    P = gg.n_pub
    g.meta.update(
        n_pub=int(P), n_pairs=int(gg.n_pairs),
        pub_type=_view(gg.pub_type, P, np.int8).copy(), pub_c1=_view(gg.pub_c1, P, np.float64).copy(),
        pub_c2=_view(gg.pub_c2, P, np.float64).copy(), pub_round=_view(gg.pub_round, P, np.int8).copy(),
        pub_depth=_view(gg.pub_depth, P, np.int8).copy(), pub_parent=_view(gg.pub_parent, P, np.int32).copy(),
        pub_sym=_view(gg.pub_sym, P, np.int8).copy(),
        pair_h1=_view(gg.pair_h1, gg.n_pairs, np.int32).copy(), pair_h2=_view(gg.pair_h2, gg.n_pairs, np.int32).copy(),
        pot_at_root=float(gg.pot_at_root),
    )
    g.meta["node_pair"] = _view(gg.pair, N, np.int32)
    return g


def _hands(cards, gids, weights):
    arr = (_Hand * len(cards))()
    for k, (c, gid, w) in enumerate(zip(cards, gids, weights)):
        arr[k].card[0] = c[0]
        arr[k].card[1] = c[1] if len(c) > 1 else -1
        arr[k].gid = int(gid)
        arr[k].weight = float(w)
    return arr


def _card_game(*, n_ranks, n_suits, hands1, hands2, sequential, n_rounds, board_before, betting, raise_cap,
               raise_size=(0, 0, 0, 0), contrib=(1.0, 1.0), payoff_mode=0, seed=0, root_hash=0,
               fixed_board=(), first_round=0, name="", pot=2.0, meta=None) -> Game:
    lib = _load()
    p = _CardParams()
    p.n_ranks, p.n_suits = n_ranks, n_suits
    h1 = _hands(*hands1)
    h2 = _hands(*hands2)
    p.n_hands1, p.n_hands2 = len(h1), len(h2)
    p.hands1 = ctypes.cast(h1, ctypes.POINTER(_Hand))
    p.hands2 = ctypes.cast(h2, ctypes.POINTER(_Hand))
    p.sequential_deal = int(sequential)
    p.n_rounds = n_rounds
    for k in range(4):
        p.board_before[k] = board_before[k] if k < len(board_before) else 0
        p.raise_size[k] = raise_size[k] if k < len(raise_size) else 0.0
        p.fixed_board[k] = fixed_board[k] if k < len(fixed_board) else -1
    p.n_fixed_board = len(fixed_board)
    p.betting, p.raise_cap = betting, raise_cap
    p.contrib1, p.contrib2 = contrib
    p.payoff_mode = payoff_mode
    p.seed = seed
    p.root_hash = root_hash
    p.first_round = first_round
    gg = _GGGame()
    lib.gg_build_card(ctypes.byref(p), ctypes.byref(gg))
    return _wrap(gg, name, pot, meta or {})


def kuhn() -> Game:
    """Kuhn poker: one deal node over the 6 ordered card pairs; pass/bet; ante 1, bet 1."""
    cards = [(c, -1) for c in range(3)]
    hands = (cards, list(range(3)), [1.0] * 3)
    return _card_game(n_ranks=3, n_suits=1, hands1=hands, hands2=hands, sequential=False, n_rounds=1,
                      board_before=(0,), betting=0, raise_cap=1, raise_size=(1.0,), contrib=(1.0, 1.0),
                      name="kuhn", pot=2.0)


def leduc(n_ranks: int = 13, n_suits: int = 2) -> Game:
    """Leduc-rule game: P1 card, then P2 card, round 1 (raise 2), public card, round 2 (raise 4)."""
    n = n_ranks * n_suits
    cards = [(c, -1) for c in range(n)]
    hands = (cards, list(range(n)), [1.0] * n)
    return _card_game(n_ranks=n_ranks, n_suits=n_suits, hands1=hands, hands2=hands, sequential=True, n_rounds=2,
                      board_before=(0, 1), betting=0, raise_cap=2, raise_size=(2.0, 4.0), contrib=(1.0, 1.0),
                      name=f"leduc{n_ranks}x{n_suits}", pot=2.0)


def all_two_card_hands(n_cards: int = 36):
    hands = []
    for a in range(n_cards):
        for b in range(a + 1, n_cards):
            hands.append((a, b))
    return hands


def two_card_gid(a: int, b: int, n_cards: int = 36) -> int:
    a, b = min(a, b), max(a, b)
    return a * (2 * n_cards - a - 1) // 2 + (b - a - 1)


def sample_hands(K: int, seed: int, n_cards: int = 36, exclude=()):
    """K distinct two-card hands per player (numpy PCG64, seeded), excluding given cards."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = [h for h in all_two_card_hands(n_cards) if h[0] not in exclude and h[1] not in exclude]
    i1 = np.sort(rng.choice(len(pool), size=K, replace=False))
    i2 = np.sort(rng.choice(len(pool), size=K, replace=False))
    return [pool[i] for i in i1], [pool[i] for i in i2]


def large(K: int = 10, seed: int = 0, hands=None) -> Game:
    """Large synthetic game: K two-card hands per player from a 36-card deck, two public rounds."""
    h1, h2 = hands if hands is not None else sample_hands(K, seed)
    g1 = [two_card_gid(*h) for h in h1]
    g2 = [two_card_gid(*h) for h in h2]
    return _card_game(n_ranks=DECK36[0], n_suits=DECK36[1], hands1=(h1, g1, [1.0] * len(h1)),
                      hands2=(h2, g2, [1.0] * len(h2)), sequential=False, n_rounds=2, board_before=(1, 1),
                      betting=1, raise_cap=3, contrib=(0.5, 0.5), payoff_mode=1, seed=seed,
                      root_hash=LARGE_ROOT_HASH, name=f"large_K{K}_s{seed}", pot=1.0,
                      meta=dict(hands1=h1, hands2=h2))


# --- round-A sequences of the pot-betting round (for cutting subgames) -------------------------

def round_sequences(contrib=(0.5, 0.5), cap=3):
    """All betting sequences of one pot-betting round that end by check-check or a call,
    with the contributions at the end: list of (symbols, (c1, c2))."""
    out = []

    def rec(seq, to_act, raises, to_call, nact, c):
        acts = ([0] if to_call > 0 else []) + [1] + ([2, 3] if raises < cap else [])
        for a in acts:
            cc = list(c)
            me = to_act - 1
            if a == 0:
                continue
            if a == 1:
                ends = to_call > 0 or nact >= 1
                cc[me] += to_call
                if ends:
                    out.append((seq + [a], (cc[0], cc[1])))
                else:
                    rec(seq + [a], 3 - to_act, raises, 0.0, nact + 1, cc)
                continue
            pot_after_call = c[0] + c[1] + to_call
            put = to_call + (0.5 * pot_after_call if a == 2 else pot_after_call)
            cc[me] += put
            rec(seq + [a], 3 - to_act, raises + 1, put - to_call, nact + 1, cc)

    rec([], 1, 0, 0.0, 0, list(contrib))
    return out


def subgame(card1: int, seqA, card2: int, hands1, hands2, r1, r2, seed: int = 0, name: str = "") -> Game:
    """Round-B subgame of ``large(seed=seed)`` at public state (card1, round-A sequence, card2).

    hands1/hands2: lists of two-card hands avoiding the board; r1/r2: range weights.  The
    root deals compatible pairs with probability proportional to r1(h1) r2(h2).  Payoffs are
    keyed by content, so they equal the corresponding terminals of the large game."""
    seqs = {tuple(s): c for s, c in round_sequences()}
    c = seqs[tuple(seqA)]
    h = hash_step(LARGE_ROOT_HASH, 16 + card1)
    for a in seqA:
        h = hash_step(h, a)
    h = hash_step(h, 16 + card2)
    g1 = [two_card_gid(*x) for x in hands1]
    g2 = [two_card_gid(*x) for x in hands2]
    return _card_game(n_ranks=DECK36[0], n_suits=DECK36[1], hands1=(hands1, g1, list(r1)),
                      hands2=(hands2, g2, list(r2)), sequential=False, n_rounds=2, board_before=(1, 0),
                      betting=1, raise_cap=3, contrib=c, payoff_mode=1, seed=seed, root_hash=h,
                      fixed_board=(card1, card2), first_round=1, name=name or f"sub_{card1}_{card2}", pot=1.0,
                      meta=dict(card1=card1, card2=card2, seqA=list(seqA), hands1=list(hands1),
                                hands2=list(hands2), r1=np.asarray(r1, float), r2=np.asarray(r2, float),
                                contrib=c))


def random_subgames(n: int, seed: int, lo: float = 1e3, hi: float = 1e6, game_seed: int = 0):
    """n subgame specs cut at round-B public states; target sizes log-uniform in [lo, hi] edges,
    ranges Dirichlet(1).  Returns a list of dicts accepted by ``subgame(**spec)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    seqs = [s for s, _ in round_sequences()]
    specs = []
    for _ in range(n):
        c1, c2 = [int(x) for x in rng.choice(36, size=2, replace=False)]
        seqA = seqs[int(rng.integers(len(seqs)))]
        target = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        pool = [x for x in all_two_card_hands() if c1 not in x and c2 not in x]
        # edges ~= 87 per compatible pair; about 89 % of pairs are compatible
        k = int(np.clip(round(np.sqrt(target / 87.0 / 0.89)), 1, len(pool)))
        i1 = np.sort(rng.choice(len(pool), size=k, replace=False))
        i2 = np.sort(rng.choice(len(pool), size=k, replace=False))
        r1 = rng.dirichlet(np.ones(k))
        r2 = rng.dirichlet(np.ones(k))
        specs.append(dict(card1=c1, seqA=list(seqA), card2=c2, hands1=[pool[i] for i in i1],
                          hands2=[pool[i] for i in i2], r1=r1, r2=r2, seed=game_seed, target=target))
    return specs


def random_game(seed: int, n_types1: int = 2, n_types2: int = 2, max_depth: int = 5, p_terminal: float = 0.3,
                p_chance: float = 0.2, max_actions: int = 3, max_chance: int = 3) -> Game:
    lib = _load()
    p = _RandomParams()
    p.seed, p.n_types1, p.n_types2, p.max_depth = seed, n_types1, n_types2, max_depth
    p.p_terminal, p.p_chance, p.max_actions, p.max_chance = p_terminal, p_chance, max_actions, max_chance
    gg = _GGGame()
    lib.gg_build_random(ctypes.byref(p), ctypes.byref(gg))
    return _wrap(gg, f"random_s{seed}", 1.0, {})


def from_arrays(type_, children_lists, probs, key, payoff, pub=None, root=0, pot=1.0, name="explicit") -> Game:
    """Build a Game from per-node python lists (small hand-written trees)."""
    n = len(type_)
    cb = np.zeros(n, np.int64)
    nc = np.zeros(n, np.int32)
    ch, pr = [], []
    for i in range(n):
        cb[i] = len(ch)
        nc[i] = len(children_lists[i])
        ch.extend(children_lists[i])
        pr.extend(probs[i] if probs[i] is not None else [0.0] * len(children_lists[i]))
    return Game(type=np.asarray(type_, np.int8), child_begin=cb, n_children=nc,
                children=np.asarray(ch, np.int64), prob=np.asarray(pr, np.float64),
                key=np.asarray(key, np.int64), payoff=np.asarray(payoff, np.float64),
                pub=np.asarray(pub if pub is not None else [-1] * n, np.int64), root=root, pot=pot, name=name)


def example11() -> Game:
    """The 11-node example game: a chance root (0.4 / 0.6), two P1 decisions (continue to a P2
    decision, or stop at a terminal), two P2 decisions with two terminals each."""
    T = GG_TERMINAL
    type_ = [GG_CHANCE, GG_P1, GG_P1, GG_P2, T, GG_P2, T, T, T, T, T]
    kids = [[1, 2], [3, 4], [5, 6], [7, 8], [], [9, 10], [], [], [], [], []]
    probs = [[0.4, 0.6]] + [None] * 10
    key = [-1, 10, 11, 20, -1, 21, -1, -1, -1, -1, -1]
    payoff = [0, 0, 0, 0, -1.0, 0, 0.5, 2.0, -2.0, 1.0, -3.0]
    return from_arrays(type_, kids, probs, key, payoff, pot=1.0, name="example11")


def degenerate(kind: str) -> Game:
    """root_terminal: a single terminal node; all_chance: a chance tree with no decisions;
    single_action: decision nodes with one action."""
    T = GG_TERMINAL
    if kind == "root_terminal":
        return from_arrays([T], [[]], [None], [-1], [0.75], name=kind)
    if kind == "all_chance":
        return from_arrays([GG_CHANCE, GG_CHANCE, T, T, T], [[1, 2], [3, 4], [], [], []],
                           [[0.3, 0.7], [0.5, 0.5], None, None, None], [-1] * 5, [0, 0, 1.0, 2.0, -1.0],
                           name=kind)
    if kind == "single_action":
        return from_arrays([GG_P1, GG_P2, T], [[1], [2], []], [None, None, None], [5, 6, -1], [0, 0, 1.5],
                           name=kind)
    raise ValueError(kind)


# --- inputs of the learned warm start ----------------------------------------------------------

def mlp_init(sizes, seed: int) -> np.ndarray:
    """Seeded initial parameters of a ReLU network, flat float32 in layer order (W_l row-major
    [fan_in, fan_out], then b_l): He-uniform hidden weights, a smaller uniform output layer, zero
    biases.  sizes: [(fan_in, fan_out), ...]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for k, (fi, fo) in enumerate(sizes):
        lim = np.sqrt(6.0 / fi) if k + 1 < len(sizes) else np.sqrt(1.0 / fi)
        parts.append(rng.uniform(-lim, lim, size=fi * fo))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def _norm_entropy(r):
    r = np.asarray(r, np.float64)
    r = r / r.sum()
    k = len(r)
    if k <= 1:
        return 1.0
    nz = r[r > 0]
    return float(-(nz * np.log(nz)).sum() / np.log(k))


def first_members(game: Game):
    """(first member node, acting player) of every information set, sets in order of first
    occurrence among decision nodes in node-id order.  Generator node ids are breadth-first with
    children in action order, so this is the canonical set order of the compiled game."""
    import pandas as pd
    ty = np.asarray(game.type)
    dec = np.flatnonzero((ty == GG_P1) | (ty == GG_P2))
    keys = np.asarray(game.key)[dec]
    # sets are keyed by (player, key); a hashed first-occurrence pass keeps node-id order
    dup = pd.DataFrame({"p": ty[dec], "k": keys}).duplicated().to_numpy()
    first = dec[~dup]
    return first, ty[first].astype(np.int8)


def warm_descriptors(game: Game, mem_off=None, mem_node=None, iset_player=None, first=None):
    """Per-information-set inputs of the feature rows for a card game from this module, in
    canonical set order (from the compiled member lists when given, else first_members):
      bucket   int16  canonical two-card hand index of the acting player's hand, mod 64
      history  int16  rank of the set's public betting state among the decision states of the
                      public tree (same tree shape for every subgame of a round), -1 if >= 32
      scalars  float32 [I, 8]: 0 pot odds to_call / (pot + to_call); 1 own hand's range weight
                      times the own hand count (1 = uniform); 2 opponent range entropy / log K;
                      3-5 the opponent's three largest range masses; 6 log K_opp / log 630;
                      7 own range entropy / log K.
    first (optional): the sets' first members as returned by first_members."""
    m = game.meta
    if first is not None:
        first = np.asarray(first, np.int64)
        player = np.asarray(game.type)[first].astype(np.int8)
    elif mem_off is None:
        first, player = first_members(game)
    else:
        first = np.asarray(mem_node, np.int64)[np.asarray(mem_off, np.int64)[:-1]]
        player = np.asarray(iset_player)
    I = len(first)
    pt = np.asarray(m["pub_type"])
    dec = np.flatnonzero((pt == GG_P1) | (pt == GG_P2))
    code = np.full(len(pt), -1, np.int64)
    code[dec] = np.arange(len(dec))
    pub = np.asarray(game.pub, np.int64)[first]
    history = np.where(pub >= 0, code[np.maximum(pub, 0)], -1)
    history = np.where(history < 32, history, -1).astype(np.int16)
    pair = np.asarray(m["node_pair"], np.int64)[first]
    p1 = player == 1
    hidx = np.where(p1, np.asarray(m["pair_h1"])[pair], np.asarray(m["pair_h2"])[pair])
    hands = (m["hands1"], m["hands2"])
    gids = [np.array([two_card_gid(*h) for h in hs], np.int64) for hs in hands]
    bucket = (np.where(p1, gids[0][np.minimum(hidx, len(gids[0]) - 1)],
                       gids[1][np.minimum(hidx, len(gids[1]) - 1)]) % 64).astype(np.int16)
    ranges = []
    for k, hs in enumerate(hands):
        r = np.asarray(m.get(f"r{k + 1}", np.ones(len(hs))), np.float64)
        ranges.append(r / r.sum())
    K = [len(r) for r in ranges]
    ent = [_norm_entropy(r) for r in ranges]
    top = []
    for r in ranges:
        t = np.sort(r)[::-1][:3]
        top.append(np.concatenate([t, np.zeros(3 - len(t))]))
    c1 = np.asarray(m["pub_c1"])[np.maximum(pub, 0)]
    c2 = np.asarray(m["pub_c2"])[np.maximum(pub, 0)]
    to_call = np.abs(c1 - c2)
    sc = np.zeros((I, 8), np.float64)
    sc[:, 0] = to_call / (c1 + c2 + to_call)
    own = np.where(p1, 0, 1)
    opp = 1 - own
    sc[:, 1] = np.where(p1, ranges[0][np.minimum(hidx, K[0] - 1)] * K[0],
                        ranges[1][np.minimum(hidx, K[1] - 1)] * K[1])
    sc[:, 2] = np.array(ent)[opp]
    sc[:, 3:6] = np.stack(top)[opp]
    sc[:, 6] = np.log(np.array(K, np.float64))[opp] / np.log(630.0)
    sc[:, 7] = np.array(ent)[own]
    return bucket, history, sc.astype(np.float32)
