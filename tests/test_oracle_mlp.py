"""Pins of the FP64 warm-start network reference (oracle.mlp) against things other than itself:
central finite differences, an independent autograd implementation (torch on the CPU, FP64), a
library bfloat16 conversion, and closed forms of the loss, Adam and the feature rows."""
import numpy as np
import pytest
import torch

import gamegen as gg
from oracle import mlp as om


def tiny(seed=0, n_in=6, hidden=5, n_hidden=2, rows=7):
    sizes = om.layer_sizes(n_in, hidden, n_hidden, om.OUT)
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.7, om.n_params(sizes))
    X = rng.normal(0, 1, (rows, n_in))
    nact = rng.integers(1, 5, rows)
    T = np.zeros((rows, 4))
    for r in range(rows):
        T[r, :nact[r]] = rng.dirichlet(np.ones(nact[r]))
    w = rng.uniform(0.2, 2.0, rows)
    return sizes, theta, X, T, w, nact


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.normal(0, 1e-3, 5000),
                        # exact ties between two bf16 neighbours, both parities
                        1.0 + np.arange(1, 64) * 2.0 ** -8, -(3.0 + np.arange(1, 64) * 2.0 ** -7),
                        [0.0, -0.0, 1.0, 65504.0, 1e-30, 3.4e38]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(om.bf16(x), ref)
    assert om.bf16(1.0 + 2.0 ** -8) == 1.0           # tie to even
    assert om.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_gradient_matches_central_differences():
    sizes, theta, X, T, w, nact = tiny()
    L, g = om.loss_and_grad(theta, sizes, X, T, w, nact)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (om.loss_and_grad(theta + e, sizes, X, T, w, nact)[0] -
                 om.loss_and_grad(theta - e, sizes, X, T, w, nact)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max()


def test_loss_and_gradient_match_torch_autograd():
    sizes, theta, X, T, w, nact = tiny(seed=3, n_in=8, hidden=6, n_hidden=3, rows=11)
    L, g = om.loss_and_grad(theta, sizes, X, T, w, nact)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    h = torch.tensor(X, dtype=torch.float64)
    o = 0
    for k, (fi, fo) in enumerate(sizes):
        W = th[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = th[o:o + fo]
        o += fo
        h = h @ W + b
        if k + 1 < len(sizes):
            h = torch.relu(h)
    legal = torch.arange(4)[None, :] < torch.tensor(nact)[:, None]
    p = torch.nn.functional.softplus(h) * legal
    q = p / p.sum(dim=1, keepdim=True)
    Tt = torch.tensor(T)
    ce = -(Tt * torch.where(legal, torch.log(torch.where(legal, q, torch.ones_like(q))), torch.zeros_like(q))).sum(1)
    wt = torch.tensor(w)
    Lt = (wt * ce).sum() / wt.sum()
    Lt.backward()
    assert L == pytest.approx(Lt.item(), rel=1e-12)
    assert np.abs(g - th.grad.numpy()).max() <= 1e-12 * np.abs(g).max()


def test_loss_closed_forms():
    # equal logits and a one-hot target over n legal actions: CE = log n
    for n in (1, 2, 3, 4):
        z = np.full((1, 4), 0.37)
        T = np.zeros((1, 4))
        T[0, 0] = 1.0
        ce, dz = om.row_loss(z, T, np.array([n]))
        assert ce[0] == pytest.approx(np.log(n), abs=1e-15)
        assert np.all(dz[0, n:] == 0.0)
    # a single legal action: nothing to learn
    ce, dz = om.row_loss(np.array([[-3.0, 5.0, 1.0, 2.0]]), np.array([[1.0, 0, 0, 0]]), np.array([1]))
    assert ce[0] == pytest.approx(0.0, abs=1e-15) and np.abs(dz).max() < 1e-15
    # very negative logits stay finite and keep the ratio of softplus values
    ce, dz = om.row_loss(np.array([[-200.0, -201.0, 0, 0]]), np.array([[0.5, 0.5, 0, 0]]), np.array([2]))
    q0 = 1.0 / (1.0 + np.exp(-1.0))
    assert ce[0] == pytest.approx(-0.5 * np.log(q0) - 0.5 * np.log(1 - q0), rel=1e-9)
    assert np.all(np.isfinite(dz))


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(4)
    th = rng.normal(size=50)
    g1, g2 = rng.normal(size=50), rng.normal(size=50)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    t1, m, v = om.adam(th, g1, np.zeros(50), np.zeros(50), 1, lr, b1, b2, eps)
    # step 1: the bias-corrected moments are g and g^2
    assert np.allclose(t1, th - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    t2, m2, v2 = om.adam(t1, g2, m, v, 2, lr, b1, b2, eps)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    assert np.allclose(t2, t1 - lr * mh / (np.sqrt(vh) + eps), rtol=1e-13, atol=1e-15)


def test_quantised_forward_is_exact_on_representable_values():
    # small integers and halves are exact in bfloat16 and their sums stay exact: rounding points
    # then change nothing, and the quantised forward equals the plain one
    sizes = om.layer_sizes(8, 6, 2, om.OUT)
    rng = np.random.default_rng(5)
    theta = rng.integers(-4, 5, om.n_params(sizes)) * 0.5
    X = rng.integers(-3, 4, (9, 8)).astype(np.float64)
    _, z0 = om.forward(theta, sizes, X, quant=False)
    _, z1 = om.forward(theta, sizes, X, quant=True)
    assert np.array_equal(z0, z1)


def test_warm_regrets_and_fallback():
    slot_off = np.array([0, 2, 7, 10])      # 2 actions, 5 actions (fallback), 3 actions
    z = np.array([[0.0, 1.0, 9, 9], [1, 1, 1, 1], [-1.0, 0.0, 2.0, 9]])
    R1 = np.array([1.0, -2.0, 1, 1, 1, 1, 1, 0.5, 0.25, -0.25])
    unit = om.regret_unit(slot_off, R1)
    assert np.array_equal(unit, [3.0, 0.0, 1.0])
    R0 = om.warm_regrets(z, slot_off, 2.0, unit)
    assert R0[0] == pytest.approx(6 * np.log(2.0))
    assert R0[1] == pytest.approx(6 * np.log1p(np.e))
    assert np.all(R0[2:7] == 0.0)
    assert R0[9] == pytest.approx(2 * np.log1p(np.exp(2.0)))


def test_feature_rows_by_hand():
    slot_off = np.array([0, 3, 5, 10])
    player = np.array([1, 2, 1])
    R1 = np.array([2.0, -1.0, -1.0, 0.0, 0.0, 1, 2, 3, 4, 5])
    bucket = np.array([5, 63, 70], np.int16)
    history = np.array([0, 31, -1], np.int16)
    sc = np.arange(24, dtype=np.float32).reshape(3, 8) / 10
    X = om.features(slot_off, player, R1, bucket, history, sc)
    assert X.shape == (3, 128)
    assert X[0, 5] == 1 and X[0, :64].sum() == 1 and X[0, 64] == 1
    assert X[1, 63] == 1 and X[1, 95] == 1 and X[2, :96].sum() == 0
    assert np.array_equal(X[0, 104:108], [1, 1, 1, 0])
    assert np.array_equal(X[0, 108:112], [0.5, -0.25, -0.25, 0])
    assert np.array_equal(X[0, 112:116], [1, 0, 0, 0])
    # all-zero regrets: uniform regret matching, zero normalised regrets
    assert np.array_equal(X[1, 108:112], [0, 0, 0, 0]) and np.array_equal(X[1, 112:116], [0.5, 0.5, 0, 0])
    # a five-action set: mask of four, no regret block
    assert np.array_equal(X[2, 104:108], [1, 1, 1, 1]) and np.all(X[2, 108:116] == 0)
    assert list(X[:, 116]) == [0, 1, 0]
    assert np.array_equal(X[:, 96:104], om.bf16(sc))
    assert np.all(X[:, 117:120] == 0)
    # no probe: uniform strategies; none for the five-action set
    assert np.array_equal(X[0, 120:128], om.bf16([1 / 3, 1 / 3, 1 / 3, 0, 1 / 3, 1 / 3, 1 / 3, 0]))
    assert np.array_equal(X[1, 120:128], [0.5, 0.5, 0, 0, 0.5, 0.5, 0, 0]) and np.all(X[2, 120:] == 0)
    cur = np.array([0.25, 0.75, 0, 1, 0, 0.2, 0.2, 0.2, 0.2, 0.2])
    avg = np.array([0.5, 0.5, 0, 0.125, 0.875, 0.2, 0.2, 0.2, 0.2, 0.2])
    X = om.features(slot_off, player, R1, bucket, history, sc, cur, avg)
    assert np.array_equal(X[0, 120:128], [0.25, 0.75, 0, 0, 0.5, 0.5, 0, 0])
    assert np.array_equal(X[1, 120:128], [1, 0, 0, 0, 0.125, 0.875, 0, 0]) and np.all(X[2, 120:] == 0)


def test_instantaneous_regret_feature_source_is_brute_force_regret():
    """The regret block is built from one plain CFR iteration from zero regrets: on a subgame that
    must equal the counterfactual regret of the uniform strategy summed over terminal paths."""
    import oracle
    from oracle import brute
    spec = gg.random_subgames(1, 2, lo=300, hi=600)[0]
    spec.pop("target")
    g = gg.subgame(**spec)
    o = oracle.Oracle(g, plus=False, linear=False)
    o.iterate(1)
    R1 = o.state()[0]
    P, isets, ns = brute.paths(g)
    ref = brute.cfr(P, isets, ns, 1, plus=False, linear=False)[0]
    assert np.abs(R1 - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-30)


def test_descriptors_of_a_subgame():
    import oracle
    spec = gg.random_subgames(1, 0, lo=1e3, hi=3e3)[0]
    spec.pop("target")
    g = gg.subgame(**spec)
    L = oracle.Oracle(g).layout()
    b, h, sc = gg.warm_descriptors(g, L["mem_off"], L["mem_node"], L["iset_player"])
    I = len(L["mem_off"]) - 1
    assert b.shape == (I,) and h.shape == (I,) and sc.shape == (I, 8)
    assert b.min() >= 0 and b.max() < 64
    # round B's pot-betting tree has 30 decision states
    assert sorted(set(h.tolist())) == list(range(30))
    # every set's members share the descriptor (they differ only in the opponent's hand)
    first = L["mem_node"][L["mem_off"][:-1]]
    assert np.all(np.asarray(g.type)[first] == L["iset_player"])
    assert np.all((sc[:, 0] >= 0) & (sc[:, 0] < 0.5))


@pytest.mark.parametrize("which", ["kuhn", "leduc", "subgame", "random"])
def test_first_members_follow_the_canonical_set_order(which):
    import oracle
    if which == "kuhn":
        g = gg.kuhn()
    elif which == "leduc":
        g = gg.leduc(3, 2)
    elif which == "subgame":
        spec = gg.random_subgames(1, 5, lo=2e3, hi=5e3)[0]
        spec.pop("target")
        g = gg.subgame(**spec)
    else:
        g = gg.random_game(11, 5, 5, 7, max_actions=5)
    L = oracle.Oracle(g).layout()
    first, player = gg.first_members(g)
    assert np.array_equal(first, L["mem_node"][L["mem_off"][:-1]])
    assert np.array_equal(player, L["iset_player"])
