"""GPU tests of the learned warm start: the BF16 MFMA network kernels against the FP64 reference
(oracle.mlp, with the kernels' bfloat16 rounding points), the feature kernel against the
reference feature rows built from the oracle's own CFR, and the warm-start injection against the
oracle's CFR from the same initial regrets.

Tolerances: loss and gradients <= 1e-3 normwise relative (the bar for BF16 kernels against FP64;
the rounding points are emulated, so what remains is FP32 accumulation order and the rare
bfloat16 rounding flip of an activation sitting on a rounding boundary); logits <= 1e-4 in the
Frobenius norm and <= 4e-3 in the max norm, which a few isolated flips can reach; Adam from the
same gradients to FP32 rounding; feature rows bit-exact except the regret blocks, which may
differ by one bfloat16 step where the FP64 and FP32 normalisations round apart."""
import sys

import numpy as np
import pytest
import torch

import gamegen as gg
import oracle
import paper_2609_11923_amd as cfr
from oracle import mlp as om

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-30))


def bf16_dev(a):
    return torch.tensor(np.asarray(om.bf16(a), np.float32)).to(torch.bfloat16).to(DEV).contiguous()


def dataset(rows, n_in, seed):
    rng = np.random.default_rng(seed)
    X = om.bf16(rng.normal(0, 1, (rows, n_in)))
    nact = rng.integers(1, 5, rows)
    T = np.zeros((rows, 4))
    for r in range(rows):
        T[r, :nact[r]] = rng.dirichlet(np.ones(nact[r]))
    w = rng.uniform(0.1, 3.0, rows)
    return X, T, w, nact


def to_dev(X, T, w, nact):
    return (bf16_dev(X), torch.tensor(T, dtype=torch.float32, device=DEV),
            torch.tensor(w, dtype=torch.float32, device=DEV), torch.tensor(nact, dtype=torch.uint8, device=DEV))


def net(n_in=128, hidden=256, n_hidden=3, max_rows=4096, seed=0):
    sizes = om.layer_sizes(n_in, hidden, n_hidden, om.OUT)
    theta = gg.mlp_init(sizes, seed)
    m = cfr.Mlp(in_dim=n_in, hidden=hidden, n_hidden=n_hidden, max_rows=max_rows)
    m.set_params(theta)
    assert m.P == theta.size
    return m, sizes, theta.astype(np.float64)


def layer_slices(sizes):
    out, o = [], 0
    for fi, fo in sizes:
        out.append(slice(o, o + fi * fo))
        o += fi * fo
        out.append(slice(o, o + fo))
        o += fo
    return out


@pytest.mark.parametrize("shape", [(128, 256, 3), (64, 64, 1), (256, 128, 2)])
@pytest.mark.parametrize("rows", [1, 300, 5000])
def test_forward_matches_oracle(shape, rows):
    n_in, hidden, nh = shape
    note(f"[mlp fwd] shape={shape} rows={rows}")
    m, sizes, theta = net(n_in, hidden, nh, max_rows=2048, seed=1)
    X, _, _, _ = dataset(rows, n_in, seed=2)
    z = torch.zeros(rows, 4, dtype=torch.float32, device=DEV)
    m.forward(bf16_dev(X), rows, z)
    torch.cuda.synchronize()
    _, zq = om.forward(theta, sizes, X, quant=True)
    _, z64 = om.forward(theta, sizes, X, quant=False)
    zg = z.cpu().numpy().astype(np.float64)
    e = rel(zg, zq)
    fro = float(np.linalg.norm(zg - zq) / max(np.linalg.norm(zq), 1e-30))
    note(f"  rel vs emulated: max {e:.2e}, frobenius {fro:.2e}; vs unrounded FP64 {rel(zg, z64):.2e}")
    # typical rows agree to FP32 accumulation order; an activation whose FP32 and FP64 values round
    # to neighbouring bfloat16 numbers moves its row by about one bfloat16 step (2^-8) of that
    # contribution, so the max-norm bound allows a few such flips
    assert fro <= 1e-4
    assert e <= 4e-3


@pytest.mark.parametrize("shape", [(128, 256, 3), (64, 64, 1), (256, 128, 2), (128, 64, 4), (64, 256, 2),
                                   (256, 256, 1)])
@pytest.mark.parametrize("rows", [1, 127, 129, 5000])
def test_fused_inference_equals_the_layered_kernels(shape, rows):
    """cfr_mlp_forward runs every layer in one kernel (activations kept in LDS); its logits equal bitwise
    those of the layer-by-layer kernels (cfr_mlp_forward_noalloc), for every hidden width and input
    width, ragged row tiles and more rows than max_rows, and again after an Adam step has moved the
    weights (the transposed weight copy is refreshed by every call)."""
    n_in, hidden, nh = shape
    note(f"[mlp fused] shape={shape} rows={rows}")
    m, sizes, theta = net(n_in, hidden, nh, max_rows=2048, seed=4)
    X, T, w, nact = dataset(rows, n_in, seed=5)
    x = bf16_dev(X)
    for step in range(2):
        za = torch.full((rows, 4), float("nan"), dtype=torch.float32, device=DEV)
        zb = torch.full((rows, 4), float("nan"), dtype=torch.float32, device=DEV)
        m.forward(x, rows, za)
        m.forward_noalloc(x, rows, zb)
        torch.cuda.synchronize()
        a, b = za.cpu().numpy(), zb.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), (step, np.abs(a - b).max())
        k = min(rows, 2048)
        d = to_dev(X[:k], T[:k], w[:k], nact[:k])
        m.backward(*d, k)
        m.adam(1e-2)


@pytest.mark.parametrize("shape", [(128, 256, 3), (64, 64, 1)])
@pytest.mark.parametrize("rows", [37, 1000, 4096])
def test_gradients_match_oracle(shape, rows):
    n_in, hidden, nh = shape
    note(f"[mlp grad] shape={shape} rows={rows}")
    m, sizes, theta = net(n_in, hidden, nh, max_rows=4096, seed=3)
    X, T, w, nact = dataset(rows, n_in, seed=4)
    Xd, Td, wd, nd = to_dev(X, T, w, nact)
    loss = m.backward(Xd, Td, wd, nd, rows)
    g = m.get(cfr.CFR_MLP_GRADS)
    L, gref = om.loss_and_grad(theta, sizes, X, T, w, nact, quant=True)
    assert loss == pytest.approx(L, rel=1e-5)
    for k, sl in enumerate(layer_slices(sizes)):
        e = rel(g[sl], gref[sl])
        note(f"  {'Wb'[k % 2]}{k // 2 + 1}: rel {e:.2e}")
        assert e <= 1e-3, k
    # the plain FP64 gradient (no rounding points) stays close as well
    _, g64 = om.loss_and_grad(theta, sizes, X, T, w, nact, quant=False)
    assert rel(g, g64) <= 3e-2


def test_gradients_with_index_list_and_no_weights():
    m, sizes, theta = net(seed=5)
    X, T, w, nact = dataset(3000, 128, seed=6)
    Xd, Td, wd, nd = to_dev(X, T, w, nact)
    rng = np.random.default_rng(7)
    idx = rng.choice(3000, size=777, replace=False)
    loss = m.backward(Xd, Td, None, nd, 777, idx=torch.tensor(idx, dtype=torch.int32, device=DEV), n_data=3000)
    g = m.get(cfr.CFR_MLP_GRADS)
    L, gref = om.loss_and_grad(theta, sizes, X[idx], T[idx], None, nact[idx], quant=True)
    assert loss == pytest.approx(L, rel=1e-5)
    assert rel(g, gref) <= 1e-3


def test_backward_is_deterministic():
    m, sizes, theta = net(seed=8)
    X, T, w, nact = dataset(2500, 128, seed=9)
    d = to_dev(X, T, w, nact)
    m.backward(*d, 2500)
    g1 = m.get(cfr.CFR_MLP_GRADS)
    m.backward(*d, 2500)
    assert np.array_equal(g1, m.get(cfr.CFR_MLP_GRADS))


def test_adam_step_matches_oracle():
    m, sizes, theta = net(seed=10)
    X, T, w, nact = dataset(512, 128, seed=11)
    d = to_dev(X, T, w, nact)
    th = m.get(cfr.CFR_MLP_PARAMS).astype(np.float64)
    mo, vo = np.zeros_like(th), np.zeros_like(th)
    for t in (1, 2, 3):
        m.backward(*d, 512)
        g = m.get(cfr.CFR_MLP_GRADS).astype(np.float64)
        m.adam(1e-3)
        th, mo, vo = om.adam(th, g, mo, vo, t, 1e-3)
        got = m.get(cfr.CFR_MLP_PARAMS)
        # FP32 update of an FP32 master copy: the reference's FP64 step, to FP32 rounding
        assert np.abs(got - th).max() <= 1e-6 * 1e-3 + 2e-7 * np.abs(th).max(), t
        th = got.astype(np.float64)
        mo = m.get(cfr.CFR_MLP_ADAM_M).astype(np.float64)
        vo = m.get(cfr.CFR_MLP_ADAM_V).astype(np.float64)


def test_training_follows_the_oracle_and_learns():
    """A few Adam steps on one fixed batch: the GPU's losses track the FP64 reference's
    (rounding points emulated) step by step, and the loss falls."""
    m, sizes, theta = net(seed=12)
    X, T, w, nact = dataset(1024, 128, seed=13)
    d = to_dev(X, T, w, nact)
    mo, vo = np.zeros_like(theta), np.zeros_like(theta)
    th = theta.copy()
    lg, lr_ = [], 3e-3
    lo = []
    for t in range(1, 21):
        lg.append(m.train_step(*d, 1024, lr_, want_loss=True))
        L, g = om.loss_and_grad(th, sizes, X, T, w, nact, quant=True)
        lo.append(L)
        th, mo, vo = om.adam(th, g, mo, vo, t, lr_)
    note(f"[train] gpu {lg[0]:.5f} -> {lg[-1]:.5f}; oracle {lo[0]:.5f} -> {lo[-1]:.5f}")
    assert lg[0] == pytest.approx(lo[0], rel=1e-5)
    assert np.allclose(lg, lo, rtol=1e-2)
    assert lg[-1] < 0.9 * lg[0]


def test_mlp_rejects_bad_arguments():
    with pytest.raises(cfr.CfrError) as e:
        cfr.Mlp(hidden=100)
    assert e.value.status == cfr.CFR_EINVAL
    m, _, _ = net(max_rows=64)
    X, T, w, nact = dataset(100, 128, seed=0)
    with pytest.raises(cfr.CfrError) as e:
        m.backward(*to_dev(X, T, w, nact), 100)
    assert e.value.status == cfr.CFR_EINVAL and "max_rows" in str(e.value)
    with pytest.raises(cfr.CfrError):
        m.set_params(np.zeros(3, np.float32))


# ---- features and warm start -----------------------------------------------------------------

def warm_games():
    sub = [gg.subgame(**{k: v for k, v in s.items() if k != "target"})
           for s in gg.random_subgames(4, seed=21, lo=500, hi=5000)]
    return sub


def descriptors(games):
    bs, hs, ss = [], [], []
    for g in games:
        L = oracle.Oracle(g).layout()
        b, h, s = gg.warm_descriptors(g, L["mem_off"], L["mem_node"], L["iset_player"])
        bs.append(b); hs.append(h); ss.append(s)
    return np.concatenate(bs), np.concatenate(hs), np.concatenate(ss)


def oracle_features(games, b, h, sc):
    rows, o = [], 0
    for g in games:
        orc = oracle.Oracle(g, plus=False, linear=False)
        orc.iterate(1)
        L = orc.layout()
        I = len(L["slot_off"]) - 1
        rows.append(om.features(L["slot_off"], L["iset_player"], orc.state()[0], b[o:o + I], h[o:o + I],
                                sc[o:o + I]))
        o += I
    return np.concatenate(rows)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_features_match_oracle_and_reset(precision):
    extra = [gg.leduc(3, 2), gg.random_game(13, 6, 6, 7, max_actions=6, max_chance=4)]
    games = warm_games() + extra
    # games without subgame descriptors get synthetic ones (out-of-range codes included)
    b, h, sc = descriptors(games[:-len(extra)])
    rng = np.random.default_rng(0)
    for g in extra:
        In = len(oracle.Oracle(g).layout()["slot_off"]) - 1
        b = np.concatenate([b, rng.integers(-2, 70, In).astype(np.int16)])
        h = np.concatenate([h, rng.integers(-2, 34, In).astype(np.int16)])
        sc = np.concatenate([sc, rng.normal(0, 1, (In, 8)).astype(np.float32)])
    p = cfr.CFR_PRECISION_FP64 if precision == "fp64" else cfr.CFR_PRECISION_FP32
    s = cfr.Solver(games, precision=p)
    I = s.n_infosets
    assert I == len(b)
    note(f"[features] {precision} {len(games)} games, {I} sets")
    s.iterate(5)  # some state that features must clear
    x = torch.zeros(I, 128, dtype=torch.bfloat16, device=DEV)
    s.features(torch.tensor(b, device=DEV), torch.tensor(h, device=DEV), torch.tensor(sc, device=DEV), x)
    torch.cuda.synchronize()
    got = x.float().cpu().numpy().astype(np.float64)
    ref = oracle_features(games, b, h, sc)
    exact = np.r_[0:108, 116:128]   # 120-127: uniform without a probe, computed identically
    assert np.array_equal(got[:, exact], ref[:, exact])
    d = np.abs(got[:, 108:116] - ref[:, 108:116])
    note(f"  regret block: {(d > 0).mean():.2e} of entries differ, max {d.max():.2e}")
    if precision == "fp64":
        # one bfloat16 step at most (2^-8 relative), only where the roundings part
        assert np.all(d <= 2.0 ** -8 * np.abs(ref[:, 108:116]) + 1e-30)
        assert (d > 0).mean() < 1e-3
    else:
        # FP32 state: the regrets themselves carry FP32 rounding
        assert (d > 2.0 ** -6).mean() < 1e-3
    # the handle is back at iteration 0 and continues exactly like a fresh one
    assert s.iterations == 0
    R, S = s.state()
    assert not R.any() and not S.any()
    s.iterate(7)
    t = cfr.Solver(games, precision=p)
    t.iterate(7)
    assert np.array_equal(s.state()[0], t.state()[0])


@pytest.mark.parametrize("probe", [1, 8])
def test_probe_columns_match_oracle_and_the_solve_continues(probe):
    games = warm_games()
    b, h, sc = descriptors(games)
    s = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64)
    I = s.n_infosets
    x = torch.zeros(I, 128, dtype=torch.bfloat16, device=DEV)
    s.features(torch.tensor(b, device=DEV), torch.tensor(h, device=DEV), torch.tensor(sc, device=DEV), x,
               probe_iters=probe)
    torch.cuda.synchronize()
    assert s.iterations == probe
    got = x.float().cpu().numpy().astype(np.float64)
    rows, o = [], 0
    for g in games:
        orc = oracle.Oracle(g, plus=False, linear=False)
        orc.iterate(1)
        L = orc.layout()
        I_k = len(L["slot_off"]) - 1
        op = oracle.Oracle(g)
        op.iterate(probe)
        _, _, cur, avg = op.state()
        rows.append(om.features(L["slot_off"], L["iset_player"], orc.state()[0], b[o:o + I_k], h[o:o + I_k],
                                sc[o:o + I_k], cur, avg))
        o += I_k
    ref = np.concatenate(rows)
    assert np.array_equal(got[:, :108], ref[:, :108]) and np.array_equal(got[:, 116:120], ref[:, 116:120])
    d = np.abs(got[:, 108:] - ref[:, 108:])
    note(f"[probe {probe}] strategy columns: {(d[:, 12:] > 0).mean():.2e} differ, max {d.max():.2e}")
    assert np.all(d <= 2.0 ** -8 * np.abs(ref[:, 108:]) + 1e-12)
    # the probe iterations are the first iterations of the solve
    s.iterate(20)
    t = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64)
    t.iterate(probe + 20)
    assert np.array_equal(s.state()[0], t.state()[0]) and np.array_equal(s.state()[1], t.state()[1])


def test_warm_start_matches_oracle_cfr_from_the_same_regrets():
    games = warm_games()
    b, h, sc = descriptors(games)
    s = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64)
    I = s.n_infosets
    x = torch.zeros(I, 128, dtype=torch.bfloat16, device=DEV)
    s.features(torch.tensor(b, device=DEV), torch.tensor(h, device=DEV), torch.tensor(sc, device=DEV), x)
    m, sizes, theta = net(seed=30)
    scale = 2.0
    s.warm_start(m, x, scale)
    z = torch.zeros(I, 4, dtype=torch.float32, device=DEV)
    m.forward(x, I, z)
    torch.cuda.synchronize()
    zc = z.cpu().numpy()
    base = s.slot_base
    R, S = s.state()
    o_off = 0
    Rrefs = []
    for k, g in enumerate(games):
        orc = oracle.Oracle(g, plus=False, linear=False)
        orc.iterate(1)
        L = orc.layout()
        Ik = len(L["slot_off"]) - 1
        unit = om.regret_unit(L["slot_off"], orc.state()[0])
        R0 = om.warm_regrets(zc[o_off:o_off + Ik], L["slot_off"], scale, unit)
        o_off += Ik
        # the handle stores FP64 state: softplus in FP32 on the device, widened
        assert rel(R[base[k]:base[k + 1]], R0) <= 1e-6, k
        Rrefs.append(R[base[k]:base[k + 1]].copy())
    assert not S.any()
    # the network's logits equal the reference forward of the same rows
    _, zq = om.forward(theta, sizes, x.float().cpu().numpy().astype(np.float64), quant=True)
    assert rel(zc, zq) <= 1e-3
    s.iterate(60)
    R, S = s.state()
    avg = s.strategy(average=True)
    for k, g in enumerate(games):
        o = oracle.Oracle(g)
        o.set_state(R=Rrefs[k], sbar=np.zeros(o.A), t=0)
        o.iterate(60)
        Ro, _, _, sao = o.state()
        assert rel(R[base[k]:base[k + 1]], Ro) <= 1e-5, k
        assert rel(avg[base[k]:base[k + 1]], sao) <= 1e-5, k


def test_warm_start_scale_zero_is_the_cold_start():
    games = warm_games()[:2]
    b, h, sc = descriptors(games)
    s = cfr.Solver(games)
    I = s.n_infosets
    x = torch.zeros(I, 128, dtype=torch.bfloat16, device=DEV)
    m0, _, _ = net(seed=32)
    with pytest.raises(cfr.CfrError) as e:
        s.warm_start(m0, x, 1.0)
    assert e.value.status == cfr.CFR_ESTATE
    s.features(torch.tensor(b, device=DEV), torch.tensor(h, device=DEV), torch.tensor(sc, device=DEV), x)
    m, _, _ = net(seed=31)
    s.warm_start(m, x, 0.0)
    s.iterate(25)
    t = cfr.Solver(games)
    t.iterate(25)
    assert np.array_equal(s.state()[0], t.state()[0])
    with pytest.raises(cfr.CfrError):
        s.warm_start(m, x, -1.0)
    with pytest.raises(cfr.CfrError):
        cfr.cfr_warm_start(s.h, m.h, x, I - 1, 1.0)


def test_warm_start_add_mode_adds_to_the_probe_regrets():
    games = warm_games()
    b, h, sc = descriptors(games)
    s = cfr.Solver(games, precision=cfr.CFR_PRECISION_FP64, rule=cfr.CFR_RULE_DCFR, order=cfr.CFR_ORDER_ALTERNATING)
    I = s.n_infosets
    x = torch.zeros(I, 128, dtype=torch.bfloat16, device=DEV)
    s.features(torch.tensor(b, device=DEV), torch.tensor(h, device=DEV), torch.tensor(sc, device=DEV), x,
               probe_iters=5)
    R5, S5 = s.state()
    m, _, _ = net(seed=33)
    z = torch.zeros(I, 4, dtype=torch.float32, device=DEV)
    m.forward(x, I, z)
    unit = torch.zeros(I, dtype=torch.float32, device=DEV)
    s.regret_unit(unit)
    s.warm_start(m, x, 0.5, add=True)
    R, S = s.state()
    zc, uc = z.cpu().numpy(), unit.cpu().numpy().astype(np.float64)
    base, o = s.slot_base, 0
    for k, g in enumerate(games):
        L = oracle.Oracle(g).layout()
        Ik = len(L["slot_off"]) - 1
        add = om.warm_regrets(zc[o:o + Ik], L["slot_off"], 0.5, uc[o:o + Ik])
        o += Ik
        sl = slice(base[k], base[k + 1])
        assert rel(R[sl] - R5[sl], add) <= 1e-6, k
    assert np.array_equal(S, S5) and s.iterations == 5
