"""FP64 numpy oracle of the coupling normalising flow used as a learned proposal.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names "new algorithms based on deep learning techniques" as future
work for the integrator (Sec. 1); the proposal follows Muller, McWilliams,
Rousselle, Gross, Novak, "Neural Importance Sampling" (ACM TOG 2019):

* the unit hypercube of VEGAS y-space is mapped by L coupling layers; layer l
  keeps the coordinates A_l unchanged and transforms the coordinates B_l one
  by one with a piecewise-quadratic (PQ) monotone map whose parameters come
  from an MLP of y_A: d_A -> H -> H -> d_B (2K+1), LeakyReLU(0.01);
* per transformed coordinate the MLP gives K width logits w and K+1 vertex
  logits v: W = softmax(w), V_k = exp(v_k) / sum_j (exp(v_j)+exp(v_j+1)) W_j / 2,
  so the density is linear inside each bin and integrates to 1;
* in bin b (edges S_b = sum_{k<b} W_k, alpha = (y - S_b)/W_b):
  pdf = V_b + alpha (V_b+1 - V_b),
  C(y) = sum_{k<b} W_k (V_k + V_k+1)/2 + W_b (alpha V_b + alpha^2 (V_b+1 - V_b)/2);
* log q(y) = sum over layers and transformed coordinates of log pdf;
* training minimises the forward KL divergence on weighted samples,
  L = - sum_i w_i log q(y_i) / sum_i w_i, or the variance of the weights
  under q: for points uniform in y, V = sum_i w_i^2 / q(y_i) estimates
  n int p^2/q, and the gradient of log V is the KL gradient with the
  per-point weights w_i^2 / q(y_i) (held fixed), normalised by their sum;
* as a proposal the flow can be mixed with the uniform density,
  q_mix = a + (1 - a) q, which bounds the weights by w / a.

Everything here is FP64 with the analytic reverse-mode gradient written out
step by step (pinned by central differences in the tests).
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.01


def masks(d: int, layers: int = 6):
    """Transformed-coordinate masks.  With nb = number of bits of d-1, layer l
    looks at bit l mod nb of the coordinate index and transforms the
    coordinates that have it set in the first nb layers and clear in the next
    nb, then repeats.  For 2 <= d <= 16 and six layers, every layer keeps and
    transforms at least one coordinate, every coordinate is transformed at least
    twice and every pair of coordinates is split in some layer."""
    nb = max(1, int(d - 1).bit_length())
    j = np.arange(d)
    out = []
    for l in range(layers):
        bit = (j >> (l % nb)) & 1
        out.append(bit == (1 if (l // nb) % 2 == 0 else 0))
    return out


def leaky(x):
    return np.where(x > 0, x, SLOPE * x)


def leaky_grad(x):
    return np.where(x > 0, 1.0, SLOPE)


def _pq_params(o, K):
    """Width and vertex parameters from the raw MLP outputs o[..., 2K+1]."""
    wl = o[..., :K]
    vl = o[..., K:]
    wl = wl - wl.max(axis=-1, keepdims=True)
    ew = np.exp(wl)
    W = ew / ew.sum(axis=-1, keepdims=True)
    vl = vl - vl.max(axis=-1, keepdims=True)
    ev = np.exp(vl)
    N = np.sum(0.5 * (ev[..., :-1] + ev[..., 1:]) * W, axis=-1, keepdims=True)
    V = ev / N
    return W, V, N


def _pq_forward(y, W, V):
    """C(y) and pdf(y) for y[n], W[n,K], V[n,K+1]; also the bin and alpha."""
    K = W.shape[-1]
    S = np.concatenate([np.zeros((W.shape[0], 1)), np.cumsum(W, axis=-1)], axis=-1)  # [n, K+1]
    b = np.sum(S[:, 1:K] <= y[:, None], axis=-1)  # bins 0..K-1
    r = np.arange(y.shape[0])
    Wb = W[r, b]
    alpha = np.clip((y - S[r, b]) / Wb, 0.0, 1.0)
    area = 0.5 * (V[:, :-1] + V[:, 1:]) * W
    A = np.concatenate([np.zeros((W.shape[0], 1)), np.cumsum(area, axis=-1)], axis=-1)
    Vb, Vb1 = V[r, b], V[r, b + 1]
    z = A[r, b] + Wb * (alpha * Vb + 0.5 * alpha * alpha * (Vb1 - Vb))
    pdf = Vb + alpha * (Vb1 - Vb)
    return z, pdf, b, alpha


def _pq_inverse(z, W, V):
    K = W.shape[-1]
    area = 0.5 * (V[:, :-1] + V[:, 1:]) * W
    A = np.concatenate([np.zeros((W.shape[0], 1)), np.cumsum(area, axis=-1)], axis=-1)
    b = np.sum(A[:, 1:K] <= z[:, None], axis=-1)
    r = np.arange(z.shape[0])
    Wb, Vb, Vb1 = W[r, b], V[r, b], V[r, b + 1]
    c = (z - A[r, b]) / Wb
    dV = Vb1 - Vb
    alpha = 2.0 * c / (Vb + np.sqrt(np.maximum(Vb * Vb + 2.0 * dV * c, 0.0)))
    alpha = np.clip(alpha, 0.0, 1.0)
    S = np.concatenate([np.zeros((W.shape[0], 1)), np.cumsum(W, axis=-1)], axis=-1)
    y = S[r, b] + alpha * Wb
    pdf = Vb + alpha * dV
    return y, pdf


def mlp(p, x):
    a1 = x @ p["W1"] + p["b1"]
    h1 = leaky(a1)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = leaky(a2)
    o = h2 @ p["W3"] + p["b3"]
    return o, (x, a1, h1, a2, h2)


def forward(params, mk, y, K=32):
    """y[n,d] -> (z[n,d], logq[n], caches) through all layers (training direction)."""
    caches = []
    logq = np.zeros(y.shape[0])
    cur = y.copy()
    for p, m in zip(params, mk):
        A, B = ~m, m
        o, mc = mlp(p, cur[:, A])
        dB = int(B.sum())
        o = o.reshape(cur.shape[0], dB, 2 * K + 1)
        nxt = cur.copy()
        per = []
        for i, j in enumerate(np.flatnonzero(B)):
            W, V, N = _pq_params(o[:, i, :], K)
            z, pdf, b, alpha = _pq_forward(cur[:, j], W, V)
            nxt[:, j] = z
            logq += np.log(pdf)
            per.append((W, V, N, b, alpha, pdf, cur[:, j].copy()))
        caches.append((cur.copy(), mc, per))
        cur = nxt
    return cur, logq, caches


def inverse(params, mk, z, K=32):
    """z[n,d] -> (y[n,d], logq[n]) (sampling direction)."""
    cur = z.copy()
    logq = np.zeros(z.shape[0])
    for p, m in reversed(list(zip(params, mk))):
        A, B = ~m, m
        o, _ = mlp(p, cur[:, A])
        dB = int(B.sum())
        o = o.reshape(cur.shape[0], dB, 2 * K + 1)
        for i, j in enumerate(np.flatnonzero(B)):
            W, V, N = _pq_params(o[:, i, :], K)
            yv, pdf = _pq_inverse(cur[:, j], W, V)
            cur[:, j] = yv
            logq += np.log(pdf)
    return cur, logq


def loss(logq, w):
    return -np.sum(w * logq) / np.sum(w)


def variance_weights(logq, w):
    """Per-point weights w^2 / q whose weighted log-likelihood gradient is
    the gradient of log sum_i w_i^2 / q(y_i)."""
    return w * w * np.exp(-logq)


def log_variance_loss(logq, w):
    """log sum_i w_i^2 / q(y_i)."""
    return float(np.log(np.sum(variance_weights(logq, w))))


def relative_variance(logq, w):
    """n sum_i w_i^2/q_i / (sum_i w_i)^2 - 1: the relative variance per event
    of the estimator that samples q, estimated from points uniform in y."""
    return float(w.size * np.sum(variance_weights(logq, w)) / np.sum(w) ** 2 - 1.0)


def mixture_density(logq, a):
    """a + (1 - a) q."""
    return a + (1.0 - a) * np.exp(logq)


def _pq_backward(gz, glp, W, V, N, b, alpha, pdf, y):
    """Gradients of gz*z + glp*log(pdf) with respect to y and to the 2K+1 logits."""
    n, K = W.shape
    r = np.arange(n)
    Wb, Vb, Vb1 = W[r, b], V[r, b], V[r, b + 1]
    dV = Vb1 - Vb
    # derivatives of z and pdf with respect to W_k and V_k at fixed y
    dz_dW = np.zeros((n, K))
    dp_dW = np.zeros((n, K))
    kk = np.arange(K)[None, :]
    below = kk < b[:, None]
    dz_dW = np.where(below, 0.5 * (V[:, :-1] + V[:, 1:]) - Vb[:, None] - (alpha * dV)[:, None], 0.0)
    dz_dW[r, b] = -0.5 * alpha * alpha * dV
    dp_dW = np.where(below, (-dV / Wb)[:, None], 0.0)
    dp_dW[r, b] = -alpha * dV / Wb
    dz_dV = np.zeros((n, K + 1))
    kv = np.arange(K + 1)[None, :]
    # area terms: A_b = sum_{k<b} W_k (V_k + V_k+1)/2
    left = np.where(kv < b[:, None], np.concatenate([W, np.zeros((n, 1))], axis=1), 0.0)  # W_k for k<b
    right = np.where((kv >= 1) & (kv <= b[:, None]), np.concatenate([np.zeros((n, 1)), W], axis=1), 0.0)  # W_{k-1}
    dz_dV = 0.5 * (left + right)
    dz_dV[r, b] += Wb * (alpha - 0.5 * alpha * alpha)
    dz_dV[r, b + 1] += Wb * 0.5 * alpha * alpha
    dp_dV = np.zeros((n, K + 1))
    dp_dV[r, b] = 1.0 - alpha
    dp_dV[r, b + 1] = alpha
    GW = gz[:, None] * dz_dW + (glp / pdf)[:, None] * dp_dW
    GV = gz[:, None] * dz_dV + (glp / pdf)[:, None] * dp_dV
    gy = gz * pdf + glp * (dV / Wb) / pdf
    # through V = exp(v)/N with N = sum_k W_k (e_k + e_k+1)/2
    SG = np.sum(GV * V, axis=1)
    GWt = GW - SG[:, None] * 0.5 * (V[:, :-1] + V[:, 1:])
    Wm = np.concatenate([np.zeros((n, 1)), W], axis=1)
    Wp = np.concatenate([W, np.zeros((n, 1))], axis=1)
    gv = V * (GV - SG[:, None] * 0.5 * (Wm + Wp))
    gw = W * (GWt - np.sum(W * GWt, axis=1, keepdims=True))
    return gy, np.concatenate([gw, gv], axis=1)


def backward(params, mk, caches, w, K=32):
    """Gradient of loss(logq, w) with respect to every parameter."""
    n = w.shape[0]
    glp = -w / np.sum(w)                # dL/dlogq_i
    d = caches[0][0].shape[1]
    gcur = np.zeros((n, d))             # dL/d(output of the current layer)
    grads = [None] * len(params)
    for li in reversed(range(len(params))):
        p, m = params[li], mk[li]
        cur, (x, a1, h1, a2, h2), per = caches[li]
        A, B = ~m, m
        gin = gcur.copy()               # coordinates of A pass through
        go = np.zeros((n, int(B.sum()), 2 * K + 1))
        for i, j in enumerate(np.flatnonzero(B)):
            W, V, N, b, alpha, pdf, y = per[i]
            gy, glog = _pq_backward(gcur[:, j], glp, W, V, N, b, alpha, pdf, y)
            gin[:, j] = gy
            go[:, i, :] = glog
        go = go.reshape(n, -1)
        g = {}
        g["W3"] = h2.T @ go
        g["b3"] = go.sum(axis=0)
        gh2 = go @ p["W3"].T
        ga2 = gh2 * leaky_grad(a2)
        g["W2"] = h1.T @ ga2
        g["b2"] = ga2.sum(axis=0)
        gh1 = ga2 @ p["W2"].T
        ga1 = gh1 * leaky_grad(a1)
        g["W1"] = x.T @ ga1
        g["b1"] = ga1.sum(axis=0)
        gx = ga1 @ p["W1"].T
        gin[:, A] += gx
        grads[li] = g
        gcur = gin
    return grads


def adam_step(params, grads, state, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    for p, g, s in zip(params, grads, state):
        for k in p:
            s["m" + k] = b1 * s["m" + k] + (1 - b1) * g[k]
            s["v" + k] = b2 * s["v" + k] + (1 - b2) * g[k] ** 2
            mh = s["m" + k] / (1 - b1**t)
            vh = s["v" + k] / (1 - b2**t)
            p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
