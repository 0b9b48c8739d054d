"""FP64 reference multilayer perceptron for the learned warm start (oracle).

TEST INFRASTRUCTURE ONLY.  Not a paper construct: the warm-start network is an addition
to the method (the paper starts its Lanczos iteration from a generic vector, Sec. 4.4.2).
This module is the gradient oracle for the GPU training kernels:
  forward   h_0 = x,  z_l = h_{l-1} W_l + b_l,  h_l = tanh(z_l) (hidden), output z_L
  loss      0.5 / B * sum (z_L - T)^2    (mean over the batch, summed over outputs);
            with `group` = g, each output row is split into consecutive groups of g values
            (one eigenvector each) and every group is compared with the sign of its target
            that fits best: 0.5 / B * sum_groups min_{s = +-1} ||y_g - s t_g||^2, where
            s = +1 when <y_g, t_g> >= 0 (eigenvectors are defined up to sign);
            with a subspace weight mu > 0 also mu * 0.5 / B * sum_groups ||(I - P) y_g||^2,
            P = sum_j t_j t_j^T / <t_j, t_j> over the row's target groups: the part of each
            output group outside the span of the targets, unchanged when the targets are
            rotated within their span (eigenvectors of a cluster are defined up to a
            rotation); P is the orthogonal projector onto that span when the target groups
            are mutually orthogonal, as eigenvectors are
  backward  the chain rule written out layer by layer
  adam      Kingma and Ba (2015) with bias correction.
Pinned by central differences (tests/test_oracle_mlp.py), which do not use the backward code.
Weights W_l are (fan_in, fan_out) row-major, matching the library.
"""

import numpy as np


def init_params(sizes, seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        bound = 1.0 / np.sqrt(fi)
        params.append([rng.uniform(-bound, bound, size=(fi, fo)), np.zeros(fo)])
    return params


def forward(params, x):
    """Returns the output and the list of layer activations needed by backward."""
    hs = [np.asarray(x, dtype=np.float64)]
    L = len(params)
    for l, (W, b) in enumerate(params):
        z = hs[-1] @ W + b
        hs.append(np.tanh(z) if l < L - 1 else z)
    return hs[-1], hs


def group_signs(y, T, group):
    """Per-row, per-group sign s = +1 if <y_g, t_g> >= 0 else -1 (shape B x n_groups)."""
    B, n = y.shape
    dots = np.einsum("bgi,bgi->bg", y.reshape(B, n // group, group), T.reshape(B, n // group, group))
    return np.where(dots >= 0.0, 1.0, -1.0)


def signed_target(y, T, group):
    """The target with every group's sign aligned to the output (T itself if group is None)."""
    if group is None:
        return T
    B, n = y.shape
    s = group_signs(y, T, group)
    return (T.reshape(B, n // group, group) * s[:, :, None]).reshape(B, n)


def outside_span(y, T, group):
    """(I - P) y_g for every output group g of every row, P = sum_j t_j t_j^T / <t_j, t_j>
    over that row's target groups (shape of y)."""
    B, n = y.shape
    Y = y.reshape(B, n // group, group)
    Tg = T.reshape(B, n // group, group)
    out = np.empty_like(Y)
    for b in range(B):
        P = sum(np.outer(t, t) / (t @ t) for t in Tg[b])
        out[b] = Y[b] - Y[b] @ P.T
    return out.reshape(B, n), Tg


def loss(params, x, T, group=None, sub_w=0.0):
    y, _ = forward(params, x)
    val = 0.5 * np.sum((y - signed_target(y, T, group)) ** 2) / x.shape[0]
    if sub_w > 0.0 and group is not None:
        r, _ = outside_span(y, T, group)
        val += sub_w * 0.5 * np.sum(r ** 2) / x.shape[0]
    return val


def backward(params, x, T, group=None, sub_w=0.0):
    """Gradients [(dW_l, db_l)] of `loss` by the chain rule (the group signs are
    piecewise constant, so they are held fixed in the derivative)."""
    y, hs = forward(params, x)
    B = x.shape[0]
    L = len(params)
    grads = [None] * L
    delta = (y - signed_target(y, T, group)) / B      # dloss / dz_L
    if sub_w > 0.0 and group is not None:
        # d/dy 0.5 ||(I - P) y||^2 = (I - P)^T (I - P) y per group
        r, Tg = outside_span(y, T, group)
        R = r.reshape(Tg.shape)
        for b in range(B):
            P = sum(np.outer(t, t) / (t @ t) for t in Tg[b])
            R[b] = R[b] - R[b] @ P
        delta = delta + sub_w * R.reshape(B, -1) / B
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        grads[l] = [hs[l].T @ delta, delta.sum(axis=0)]
        if l > 0:
            delta = (delta @ W.T) * (1.0 - hs[l] ** 2)   # through tanh of layer l
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; state = {"t": int, "m": [...], "v": [...]}."""
    if not state:
        state["t"] = 0
        state["m"] = [[np.zeros_like(p) for p in layer] for layer in params]
        state["v"] = [[np.zeros_like(p) for p in layer] for layer in params]
    state["t"] += 1
    t = state["t"]
    for l, layer in enumerate(params):
        for q in range(2):
            g = grads[l][q]
            m = state["m"][l][q] = beta1 * state["m"][l][q] + (1 - beta1) * g
            v = state["v"][l][q] = beta2 * state["v"][l][q] + (1 - beta2) * g * g
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            layer[q] -= lr * mh / (np.sqrt(vh) + eps)
    return params
