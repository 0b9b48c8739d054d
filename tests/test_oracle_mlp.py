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
