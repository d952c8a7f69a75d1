"""CPU tests of the persistent schedule's work plan (cfr_persistent_plan_host) and of the claim protocol
the kernel runs on it: workgroups claim (game, rank) tickets in order from per-XCD queues, a game's
ranks meet at barriers, and a rank blocks its workgroup until the game's other ranks have been claimed.
A discrete model of that protocol shows that every game finishes as soon as 8 (max_w - 1) + 1
workgroups can be resident -- the plan's guarantee -- and the model's bound is tight."""
import numpy as np
import pytest

import paper_2609_11923_amd as cfr

QUEUES = 8


def sizes(n, seed):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(1e3), np.log(1e6), n)).astype(np.int64)


@pytest.mark.parametrize("n,wg,max_w", [(256, 16384, 40), (256, 1024, 40), (32, 4096, 8), (1, 0, 1), (9, 512, 160)])
def test_plan_arithmetic(n, wg, max_w):
    nodes = sizes(n, n)
    p = cfr.cfr_persistent_plan_host(nodes, wg, max_w)
    used = p["wg_nodes"]
    base = wg if wg > 0 else 16384
    assert used >= base and used % base == 0 and (used // base) & (used // base - 1) == 0   # base times 2^k
    W = p["W"]
    assert np.array_equal(W, np.maximum(1, -(-nodes // used)))
    assert W.max() <= max_w
    if used > base:   # the smallest doubling that fits
        assert np.maximum(1, -(-nodes // (used // 2))).max() > max_w
    q_off = p["q_off"]
    assert q_off[0] == 0 and np.all(np.diff(q_off) >= 0) and q_off[-1] == W.sum()
    for q in range(QUEUES):
        assert W[p["queue"] == q].sum() == q_off[q + 1] - q_off[q]
    # largest first on the least loaded queue: no queue exceeds the mean by more than the largest game
    load = np.array([nodes[p["queue"] == q].sum() for q in range(QUEUES)])
    assert load.max() <= load.mean() + nodes.max()


def claim_model(W, queue, slots):
    """Tickets of each queue in plan order (a game's ranks consecutive, games in placement order);
    `slots` workgroups are resident, the i-th with home queue i % 8.  A free workgroup claims the next
    ticket of its home queue, else of the next queues in turn; a game whose ranks are all claimed runs
    to its end and frees its workgroups.  Returns the number of games finished."""
    order = {q: [g for g in np.argsort(-W, kind="stable") if queue[g] == q] for q in range(QUEUES)}
    tickets = {q: [(g, r) for g in order[q] for r in range(W[g])] for q in range(QUEUES)}
    nxt = {q: 0 for q in range(QUEUES)}
    claimed = np.zeros(len(W), np.int64)
    free = list(range(slots))
    busy = {}   # game -> workgroups holding its ranks
    finished = 0
    progress = True
    while progress:
        progress = False
        still = []
        for wg in free:
            home = wg % QUEUES
            for k in range(QUEUES):
                q = (home + k) % QUEUES
                if nxt[q] < len(tickets[q]):
                    g, _ = tickets[q][nxt[q]]
                    nxt[q] += 1
                    claimed[g] += 1
                    busy.setdefault(g, []).append(wg)
                    progress = True
                    break
            else:
                continue
        free = []
        for g in list(busy):
            if claimed[g] == W[g]:   # every rank is running: the game finishes and frees them
                free += busy.pop(g)
                finished += 1
                progress = True
        free += still
    return finished


def test_claim_protocol_finishes_every_game_with_a_quarter_of_the_device():
    nodes = sizes(256, 7)
    capacity = 1280                        # 256 compute units x 5 resident workgroups
    max_w = capacity // QUEUES // 4        # what the library uses
    p = cfr.cfr_persistent_plan_host(nodes, 4096, max_w)
    W, queue = p["W"], p["queue"]
    need = QUEUES * (W.max() - 1) + 1
    assert need <= capacity // 4 + QUEUES
    assert claim_model(W, queue, need) == len(W)
    assert claim_model(W, queue, capacity) == len(W)


def test_claim_model_bound_is_tight():
    """Eight queues whose first games need 5 ranks each: 8 x 4 resident workgroups can all end up
    waiting on partly claimed games, one more always finishes them."""
    W = np.array([5] * 8 + [1] * 8)
    queue = np.array(list(range(8)) * 2)
    assert claim_model(W, queue, 8 * 4) < len(W)
    assert claim_model(W, queue, 8 * 4 + 1) == len(W)


def test_plan_rejects_bad_arguments():
    with pytest.raises(cfr.CfrError) as e:
        cfr.cfr_persistent_plan_host(np.array([10, -1]), 1024, 4)
    assert e.value.status == cfr.CFR_EINVAL
    with pytest.raises(cfr.CfrError) as e:
        cfr.cfr_persistent_plan_host(np.array([10]), 1024, 0)
    assert e.value.status == cfr.CFR_EINVAL
