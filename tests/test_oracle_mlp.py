"""Pins of the FP64 MLP oracle: backpropagation against central differences (which use
only the forward pass), and Adam against its closed form on a scalar quadratic."""

import numpy as np

from oracle import mlp


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    sizes = [3, 7, 5, 4]
    params = mlp.init_params(sizes, seed=1)
    x = rng.standard_normal((6, 3))
    T = rng.standard_normal((6, 4))
    grads = mlp.backward(params, x, T)
    h = 1e-6
    for l in range(len(params)):
        for q in range(2):
            P = params[l][q]
            G = grads[l][q]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = P[idx]
                P[idx] = old + h
                fp = mlp.loss(params, x, T)
                P[idx] = old - h
                fm = mlp.loss(params, x, T)
                P[idx] = old
                assert abs((fp - fm) / (2 * h) - G[idx]) < 1e-8


def test_forward_shapes_and_tanh_range():
    params = mlp.init_params([3, 16, 16, 10], seed=2)
    y, hs = mlp.forward(params, np.ones((4, 3)))
    assert y.shape == (4, 10)
    assert all(np.all(np.abs(h) <= 1.0) for h in hs[1:-1])


def test_adam_first_step_closed_form():
    """With zero moments, the first Adam step moves each parameter by -lr * sign(g)
    (bias-corrected m/sqrt(v) = g/|g|), up to eps."""
    params = [[np.array([[2.0, -3.0]]), np.array([0.5, 0.0])]]
    grads = [[np.array([[4.0, -1.0]]), np.array([0.25, 0.0])]]
    state = {}
    mlp.adam_step(params, grads, state, lr=0.1)
    assert np.allclose(params[0][0], [[1.9, -2.9]], atol=1e-7)
    assert np.allclose(params[0][1], [0.4, 0.0], atol=1e-7)


def test_signed_loss_central_differences_and_sign_invariance():
    """Sign-invariant loss: gradients by central differences (targets far from the
    switching surface <y_g, t_g> = 0), and the value does not change when the sign of
    any target group is flipped."""
    rng = np.random.default_rng(3)
    sizes = [3, 6, 8]
    params = mlp.init_params(sizes, seed=4)
    x = rng.standard_normal((5, 3))
    y, _ = mlp.forward(params, x)
    # targets = output plus noise, with random signs per group of 4: |<y, t>| is large
    signs = rng.choice([-1.0, 1.0], size=(5, 2))
    T = (y + 0.1 * rng.standard_normal(y.shape)).reshape(5, 2, 4) * signs[:, :, None]
    T = T.reshape(5, 8)
    grads = mlp.backward(params, x, T, group=4)
    h = 1e-6
    for l in range(len(params)):
        for q in range(2):
            P, G = params[l][q], grads[l][q]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = P[idx]
                P[idx] = old + h
                fp = mlp.loss(params, x, T, group=4)
                P[idx] = old - h
                fm = mlp.loss(params, x, T, group=4)
                P[idx] = old
                assert abs((fp - fm) / (2 * h) - G[idx]) < 1e-8
    base = mlp.loss(params, x, T, group=4)
    T2 = T.copy()
    T2[2, 4:8] *= -1.0
    assert abs(mlp.loss(params, x, T2, group=4) - base) < 1e-14
    # all signs aligned with the output: the signed loss is the plain loss of the aligned targets
    Ta = (T.reshape(5, 2, 4) * signs[:, :, None]).reshape(5, 8)
    assert abs(mlp.loss(params, x, Ta) - base) < 1e-14


def _orthogonal_targets(rng, B, ng, g, scale):
    T = np.empty((B, ng * g))
    for b in range(B):
        Q, _ = np.linalg.qr(rng.standard_normal((g, ng)))
        T[b] = (Q.T * scale).reshape(-1)
    return T


def test_subspace_loss_central_differences():
    """Sign-invariant plus subspace loss: gradients by central differences (targets far
    from the sign switching surface)."""
    rng = np.random.default_rng(5)
    sizes = [3, 6, 12]
    params = mlp.init_params(sizes, seed=6)
    x = rng.standard_normal((4, 3))
    y, _ = mlp.forward(params, x)
    T = y + 0.3 * rng.standard_normal(y.shape)        # <y_g, t_g> far from zero
    grads = mlp.backward(params, x, T, group=4, sub_w=0.7)
    h = 1e-6
    for l in range(len(params)):
        for q in range(2):
            P = params[l][q]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = P[idx]
                P[idx] = old + h
                fp = mlp.loss(params, x, T, group=4, sub_w=0.7)
                P[idx] = old - h
                fm = mlp.loss(params, x, T, group=4, sub_w=0.7)
                P[idx] = old
                assert abs((fp - fm) / (2 * h) - grads[l][q][idx]) < 1e-7


def test_subspace_term_is_rotation_invariant_and_vanishes_in_the_span():
    """Rotating each row's orthogonal target groups by an orthogonal matrix (a rotation
    inside an eigenvector cluster) leaves the subspace term unchanged while the per-group
    term changes; an output inside the span of its targets has no subspace term."""
    rng = np.random.default_rng(7)
    B, ng, g = 3, 4, 9
    sizes = [2, 5, ng * g]
    params = mlp.init_params(sizes, seed=8)
    x = rng.standard_normal((B, 2))
    T = _orthogonal_targets(rng, B, ng, g, 3.0)
    Q, _ = np.linalg.qr(rng.standard_normal((ng, ng)))
    Tr = np.einsum("ij,bjk->bik", Q, T.reshape(B, ng, g)).reshape(B, -1)
    sub = lambda TT: mlp.loss(params, x, TT, group=g, sub_w=1.0) - mlp.loss(params, x, TT, group=g)   # noqa: E731
    assert abs(sub(T) - sub(Tr)) < 1e-12 * abs(sub(T))
    assert abs(mlp.loss(params, x, T, group=g) - mlp.loss(params, x, Tr, group=g)) > 1e-3
    # inside the span: y = combination of the row's targets
    y, _ = mlp.forward(params, x)
    C = rng.standard_normal((B, ng, ng))
    Ys = np.einsum("bij,bjk->bik", C, T.reshape(B, ng, g)).reshape(B, -1)
    r, _ = mlp.outside_span(Ys, T, g)
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(Ys))
