"""FP64 reference of the warm-start network and its features (TEST INFRASTRUCTURE ONLY).

Only the test suite may import this module; the product path never does.  The paper has no
learned part: the network, its loss and its features are this project's own definitions,
written out here plainly so that the GPU kernels can be checked against them.

Network (parameters in one flat FP32 vector, layer by layer: W_l row-major [fan_in, fan_out],
then b_l):
    h_0 = x,  h_l = relu(h_{l-1} W_l + b_l) for the hidden layers,  z = h_L W_out + b_out.
Loss of one row with n legal actions (the first n of the outputs), target distribution t and
row weight w:
    p_a = softplus(z_a),  q_a = p_a / sum_b p_b,  CE = -sum_a t_a log q_a,
    L = sum_r w_r CE_r / sum_r w_r.
Warm-start regrets: R0(I, a) = c * m(I) * softplus(z_a) for the legal actions of a set with at
most 4 actions, and 0 (the uniform strategy) for larger sets; m(I) is the sum of the magnitudes
of the set's instantaneous regrets under the uniform strategy (the regret unit of the set).
Adam: Kingma and Ba (2015), Algorithm 1, with the bias corrections.

quant=True rounds to bfloat16 (round to nearest, ties to even, from the FP32 value) exactly
where the GPU kernels store bfloat16: the input rows, the weight matrices, every hidden
activation, and every hidden-layer gradient of a pre-activation.  Everything else is FP64.
"""
from __future__ import annotations

import numpy as np

OUT = 4          # outputs (actions) of the network
FEAT = 128       # feature width
N_SCALARS = 8    # caller-supplied scalar features per row
LOG_CUT = -30.0  # below this, log softplus(z) = z and sigmoid(z)/softplus(z) = 1 (error < 1e-13)


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through FP32; returns FP64 values."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def layer_sizes(n_in=FEAT, hidden=256, n_hidden=3, n_out=OUT):
    dims = [n_in] + [hidden] * n_hidden + [n_out]
    return list(zip(dims[:-1], dims[1:]))


def unflatten(theta, sizes):
    """Views (W, b) per layer into the flat parameter vector."""
    out, o = [], 0
    for fi, fo in sizes:
        W = theta[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = theta[o:o + fo]
        o += fo
        out.append((W, b))
    assert o == theta.size
    return out


def n_params(sizes):
    return sum(fi * fo + fo for fi, fo in sizes)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def log_softplus(z):
    sp = softplus(np.maximum(z, LOG_CUT))
    return np.where(z < LOG_CUT, z, np.log(sp))


def forward(theta, sizes, X, quant=False):
    """Returns (hidden activations [h_0 .. h_L], logits z)."""
    layers = unflatten(np.asarray(theta, np.float64), sizes)
    h = np.asarray(X, np.float64)
    if quant:
        h = bf16(h)
    hs = [h]
    for W, b in layers[:-1]:
        Wq = bf16(W) if quant else W
        h = np.maximum(h @ Wq + b, 0.0)
        if quant:
            h = bf16(h)
        hs.append(h)
    W, b = layers[-1]
    z = hs[-1] @ (bf16(W) if quant else W) + b
    return hs, z


def row_loss(z, T, nact):
    """Per-row cross entropy and its gradient with respect to z (legal actions only)."""
    z = np.asarray(z, np.float64)
    legal = np.arange(z.shape[1])[None, :] < np.asarray(nact)[:, None]
    ls = np.where(legal, log_softplus(z), -np.inf)
    m = ls.max(axis=1, keepdims=True)
    lS = m + np.log(np.exp(ls - m).sum(axis=1, keepdims=True))
    Tm = np.where(legal, T, 0.0)
    ce = -(Tm * np.where(legal, ls - lS, 0.0)).sum(axis=1)
    ratio = np.where(z < LOG_CUT, 1.0, sigmoid(z) / softplus(np.maximum(z, LOG_CUT)))
    lsig = -softplus(-z)
    dz = np.where(legal, -Tm * ratio + Tm.sum(axis=1, keepdims=True) * np.exp(lsig - lS), 0.0)
    return ce, dz


def loss_and_grad(theta, sizes, X, T, w, nact, quant=False):
    """Weighted mean cross entropy and its gradient (flat, in the parameter layout)."""
    theta = np.asarray(theta, np.float64)
    layers = unflatten(theta, sizes)
    hs, z = forward(theta, sizes, X, quant)
    w = np.ones(z.shape[0]) if w is None else np.asarray(w, np.float64)
    ce, dce = row_loss(z, T, nact)
    W = w.sum()
    L = float((w * ce).sum() / W)
    dz = dce * (w / W)[:, None]
    grads = [None] * len(layers)
    Wout = bf16(layers[-1][0]) if quant else layers[-1][0]
    grads[-1] = (hs[-1].T @ dz, dz.sum(axis=0))
    dA = (dz @ Wout.T) * (hs[-1] > 0)
    if quant:
        dA = bf16(dA)
    for l in range(len(layers) - 2, -1, -1):
        grads[l] = (hs[l].T @ dA, dA.sum(axis=0))
        if l > 0:
            Wl = bf16(layers[l][0]) if quant else layers[l][0]
            dA = (dA @ Wl.T) * (hs[l] > 0)
            if quant:
                dA = bf16(dA)
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, g


def adam(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step number t >= 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def regret_unit(slot_off, R1):
    """m(I): the sum of |R1| over the first four actions of each set with at most four actions
    (0 for larger sets), R1 being the instantaneous regrets of the uniform strategy."""
    slot_off = np.asarray(slot_off)
    m = np.zeros(len(slot_off) - 1)
    for i in range(len(m)):
        n = slot_off[i + 1] - slot_off[i]
        if n <= OUT:
            m[i] = np.abs(np.asarray(R1[slot_off[i]:slot_off[i + 1]], np.float64)).sum()
    return m


def warm_regrets(z, slot_off, scale, unit):
    """Initial regrets in slot order from per-set logits z [I, 4]: scale * m(I) * softplus(z) on
    the legal actions of sets with at most four actions, zero (uniform) elsewhere."""
    slot_off = np.asarray(slot_off)
    R0 = np.zeros(int(slot_off[-1]))
    for i in range(len(slot_off) - 1):
        n = slot_off[i + 1] - slot_off[i]
        if n <= OUT:
            R0[slot_off[i]:slot_off[i + 1]] = scale * unit[i] * softplus(np.asarray(z[i][:n], np.float64))
    return R0


def features(slot_off, player, R1, bucket, history, scalars, cur=None, avg=None):
    """Feature rows [I, 128] (bfloat16 values held in FP64) of every information set.

    R1: the regrets after one plain CFR iteration from zero regrets (the instantaneous regrets
    of the uniform strategy), in slot order.  Columns: 0-63 one-hot hand bucket; 64-95 one-hot
    public-history code; 96-103 the caller's scalars; 104-107 legal-action mask; 108-111 the
    first four regrets over the sum of their magnitudes; 112-115 regret matching (plus) of those
    regrets; 116 the acting player (0 or 1); 117-119 zero; 120-123 the current strategy and
    124-127 the normalised average strategy after a probe run (slot order arrays cur and avg;
    uniform when not given); 120-127 are zero for sets of more than four actions."""
    slot_off = np.asarray(slot_off)
    I = len(slot_off) - 1
    X = np.zeros((I, FEAT))
    for i in range(I):
        if 0 <= bucket[i] < 64:
            X[i, bucket[i]] = 1.0
        if 0 <= history[i] < 32:
            X[i, 64 + history[i]] = 1.0
        X[i, 96:104] = scalars[i]
        n = int(slot_off[i + 1] - slot_off[i])
        k = min(n, OUT)
        X[i, 104:104 + k] = 1.0
        if n <= OUT:
            r = np.asarray(R1[slot_off[i]:slot_off[i] + k], np.float64)
            s = np.abs(r).sum()
            if s > 0:
                X[i, 108:108 + k] = r / s
            pos = np.maximum(r, 0.0)
            X[i, 112:112 + k] = pos / pos.sum() if pos.sum() > 0 else 1.0 / k
        X[i, 116] = float(player[i] == 2)
        if n <= OUT:
            sl = slice(slot_off[i], slot_off[i + 1])
            X[i, 120:120 + n] = 1.0 / n if cur is None else np.asarray(cur[sl], np.float64)
            X[i, 124:124 + n] = 1.0 / n if avg is None else np.asarray(avg[sl], np.float64)
    return bf16(X)
