"""GPU parity of the warm-start network kernels (kl_mlp_*) against the FP64 oracle MLP.

The oracle's backpropagation is pinned by central differences (test_oracle_mlp.py).
Here the GPU forward pass, gradients and Adam step are compared with it on the same
FP32 parameters (converted exactly to FP64).  Tolerance: 1e-4 relative for FP32 GEMMs
with FP32 accumulation over at most a few thousand terms (forward outputs 1e-5).
"""

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
from oracle import mlp

pytestmark = pytest.mark.gpu


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def _unflat(flat, sizes):
    out, off = [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        W = flat[off:off + fi * fo].reshape(fi, fo)
        off += fi * fo
        b = flat[off:off + fo]
        off += fo
        out.append([W.astype(np.float64).copy(), b.astype(np.float64).copy()])
    return out


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _setup(sizes, B, seed, group):
    rng = np.random.default_rng(seed)
    flat = _flat(mlp.init_params(sizes, seed=seed)).astype(np.float32)
    # non-zero biases so that the bias paths are exercised
    params = _unflat(flat, sizes)
    for W, b in params:
        b[:] = rng.uniform(-0.2, 0.2, size=b.shape).astype(np.float32)
    flat = _flat(params).astype(np.float32)
    params = _unflat(flat, sizes)
    x = rng.standard_normal((B, sizes[0])).astype(np.float32)
    y, _ = mlp.forward(params, x.astype(np.float64))
    if group:
        # targets near +-output per group, so the sign choice is unambiguous
        ng = sizes[-1] // group
        s = rng.choice([-1.0, 1.0], size=(B, ng))
        t = (y + 0.3 * np.abs(y).mean() * rng.standard_normal(y.shape)).reshape(B, ng, group) * s[:, :, None]
        t = t.reshape(B, -1)
    else:
        t = y + rng.standard_normal(y.shape)
    return flat, params, x, t.astype(np.float32)


# Widths that are multiples of 4 (with 16-byte aligned weight blocks) take the float4 form
# of the product: "aligned_ragged" on ragged tiles and split K ranges, "aligned_odd_batch"
# with 19 rows, "aligned_tiles" on exact 64-multiples, "warmstart_b64" at the training
# minibatch of the warm-start network (every layer but the first in the float4 form).
# "direct_forms": fan-ins of at most 8 (3 inputs, 5 rows, 8 outputs) take the one-thread-
# per-output kernel in its plain, transposed-A and transposed-B forms.  "ragged_split": the
# delta back through 1030 unaligned outputs takes the scalar-load form over split K ranges.
CASES = [([3, 16, 16, 10], 7, 0), ([3, 16, 16, 10], 7, 5), ([5, 70, 33, 130], 67, 13),
         ([3, 256, 256, 41616], 8, 2601), ([4, 36, 68, 1300], 20, 13), ([4, 36, 68, 1300], 19, 13),
         ([8, 64, 128, 4160], 64, 0), ([3, 256, 256, 41616], 64, 2601), ([3, 16, 8], 5, 0),
         ([5, 70, 33, 1030], 9, 0)]
CASE_IDS = ["small_mse", "small_signed", "ragged", "warmstart_size", "aligned_ragged",
            "aligned_odd_batch", "aligned_tiles", "warmstart_b64", "direct_forms", "ragged_split"]


def _max_rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("sizes,B,group", CASES, ids=CASE_IDS)
def test_forward_and_gradients_match_oracle(sizes, B, group):
    flat, params, x, t = _setup(sizes, B, 11, group)
    net = kl.MLP(sizes)
    net.set_params(flat)
    assert np.array_equal(net.get_params(), flat)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    y = net.forward(xd).cpu().numpy()
    y_ref, _ = mlp.forward(params, x.astype(np.float64))
    assert _rel(y, y_ref) <= 1e-5
    assert _max_rel(y, y_ref) <= 1e-5     # every element, so that one wrong tile shows
    loss, g = net.gradients(xd, td, group=group)
    loss_ref = mlp.loss(params, x.astype(np.float64), t.astype(np.float64), group=group or None)
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    g_ref = mlp.backward(params, x.astype(np.float64), t.astype(np.float64), group=group or None)
    gl = _unflat(g.cpu().numpy(), sizes)
    for l, ((dW, db), (rW, rb)) in enumerate(zip(gl, g_ref)):
        assert _rel(dW, rW) <= 1e-4, (l, "W", _rel(dW, rW))
        assert _rel(db, rb) <= 1e-4, (l, "b", _rel(db, rb))
        assert _max_rel(dW, rW) <= 1e-4, (l, "W", _max_rel(dW, rW))


def _epoch_perm(n, state):
    """Minibatch order of one epoch of kl_mlp_train: a Fisher-Yates shuffle whose draws are
    splitmix64 of the running state (the published generator: add 0x9E3779B97F4A7C15, then
    two xor-shift-multiply rounds and a final xor-shift)."""
    mask = (1 << 64) - 1
    perm = list(range(n))
    for i in range(n - 1, 0, -1):
        state = (state + 0x9E3779B97F4A7C15) & mask
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        z ^= z >> 31
        j = z % (i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    return perm, state


# warm-start network (W2, W3 updated in their gradient products' epilogues, W1 and the
# biases in the ranged step; the first layer's forward product, fan-in 3, in the
# one-thread-per-output kernel), the same with 72 samples (minibatches of 64 and 8 rows),
# all weights fused, none fused (split K ranges: batch 512), none in the float4 form, and 11
# layers none of which is fused (11 merged parameter ranges in the ranged Adam launch)
TRAIN_CASES = [([3, 256, 256, 41616], 64, 64, 2601, 3.0), ([3, 256, 256, 41616], 72, 64, 2601, 3.0),
               ([8, 64, 128, 4160], 64, 64, 0, 0.0), ([4, 36, 68, 1300], 512, 512, 65, 0.5),
               ([5, 70, 33, 130], 67, 67, 13, 0.0), ([5] + [9] * 10 + [7], 20, 20, 0, 0.0)]


@pytest.mark.parametrize("sizes,n,B,group,sub", TRAIN_CASES,
                         ids=["warmstart", "warmstart_ragged_batch", "all_fused", "split_k", "scalar_form",
                              "deep_unfused"])
def test_training_step_matches_gradients_and_adam(sizes, n, B, group, sub):
    """Two epochs of kl_mlp_train give the same bits as the same steps taken through
    kl_mlp_gradients and kl_mlp_adam on the minibatches in the training order: the Adam
    step that runs in a weight product's epilogue (no stored gradient) equals the separate
    one."""
    flat, _, x, t = _setup(sizes, n, 21, group)
    fused, ref = kl.MLP(sizes), kl.MLP(sizes)
    fused.set_params(flat)
    ref.set_params(flat)
    if sub:
        fused.set_subspace(sub)
        ref.set_subspace(sub)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    seed, lr = 5, 1e-3
    fused.train(xd, td, group=group, epochs=2, batch=B, lr0=lr, lr1=lr, seed=seed)
    state = seed
    for _ in range(2):
        perm, state = _epoch_perm(n, state)
        for b0 in range(0, n, B):
            idx = torch.tensor(perm[b0:b0 + B], device="cuda")
            ref.gradients(xd[idx].contiguous(), td[idx].contiguous(), group=group)
            ref.adam(lr)
    a, b = fused.get_params(), ref.get_params()
    assert not np.array_equal(a, flat)
    diff = np.flatnonzero(a != b)
    assert diff.size == 0, (diff.size, diff[:4], np.max(np.abs(a - b)))


def test_adam_step_matches_oracle():
    """Three Adam steps on the GPU gradients, against the oracle's Adam fed the same
    gradients (the update rule alone, FP32 against FP64)."""
    sizes = [3, 20, 9]
    flat, params, x, t = _setup(sizes, 6, 5, 0)
    net = kl.MLP(sizes)
    net.set_params(flat)
    state = {}
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    for _ in range(3):
        _, g = net.gradients(xd, td)
        net.adam(1e-2)
        mlp.adam_step(params, _unflat(g.cpu().numpy(), sizes), state, lr=1e-2)
    got = net.get_params()
    ref = _flat(params)
    assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


def test_training_reduces_loss():
    """kl_mlp_train on a smooth synthetic regression: the epoch loss falls by 20x."""
    rng = np.random.default_rng(2)
    n = 512
    x = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32)
    freq = rng.standard_normal((3, 24))
    t = np.sin(x @ freq).astype(np.float32)
    net = kl.MLP([3, 64, 64, 24], seed=3)
    losses = net.train(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), epochs=150, batch=64,
                       lr0=3e-3, lr1=3e-4, seed=4)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < losses[0] / 20, (losses[0], losses[-1])


def test_mlp_errors():
    with pytest.raises(kl.KLError):
        kl.MLP([3])
    net = kl.MLP([3, 4, 6])
    x = torch.zeros((2, 3), dtype=torch.float32, device="cuda")
    t = torch.zeros((2, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(kl.KLError):
        net.gradients(x, t, group=4)           # 4 does not divide 6
    with pytest.raises(ValueError):
        net.forward(torch.zeros((2, 5), dtype=torch.float32, device="cuda"))


def _orthogonal_targets_near(y, B, ng, group, rng):
    """Per row, the output groups plus noise, orthogonalised (QR) and scaled to the output
    groups' norms, with random signs: orthogonal targets whose sign choice is unambiguous."""
    t = np.empty_like(y)
    for b in range(B):
        Yg = y[b].reshape(ng, group)
        Q, _ = np.linalg.qr((Yg + 0.2 * np.abs(Yg).mean() * rng.standard_normal(Yg.shape)).T)
        Tg = Q.T * np.linalg.norm(Yg, axis=1)[:, None]
        Tg *= np.sign(np.sum(Tg * Yg, axis=1))[:, None] * rng.choice([-1.0, 1.0], size=(ng, 1))
        t[b] = Tg.reshape(-1)
    return t


# 7 groups of 300 (several LDS chunks per slice, ragged tail); 32 groups of 150; 32 groups
# of 48 (residual slices of 2 elements: slices 24 to 31 are empty)
SUB_CASES = CASES[1:4] + [CASES[7]] + [([3, 16, 16, 2100], 5, 300), ([3, 16, 16, 4800], 3, 150),
                            ([3, 8, 8, 1536], 4, 48)]


@pytest.mark.parametrize("sizes,B,group", SUB_CASES,
                         ids=["small_signed", "ragged", "warmstart_size", "warmstart_b64", "g7", "g32",
                              "g32_short"])
def test_subspace_loss_gradients_match_oracle(sizes, B, group):
    """The grouped loss with its subspace term (weight 0.8) against the oracle, on
    mutually orthogonal target groups per row (2 to 32 groups: every register bucket of
    the residual pass)."""
    flat, params, x, _ = _setup(sizes, B, 12, group)
    y, _ = mlp.forward(params, x.astype(np.float64))
    ng = sizes[-1] // group
    t = _orthogonal_targets_near(y, B, ng, group, np.random.default_rng(13)).astype(np.float32)
    net = kl.MLP(sizes)
    net.set_params(flat)
    net.set_subspace(0.8)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss, g = net.gradients(xd, td, group=group)
    t64 = t.astype(np.float64)
    loss_ref = mlp.loss(params, x.astype(np.float64), t64, group=group, sub_w=0.8)
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref, (loss, loss_ref)
    assert loss_ref > mlp.loss(params, x.astype(np.float64), t64, group=group) * 1.01   # the term is present
    g_ref = mlp.backward(params, x.astype(np.float64), t64, group=group, sub_w=0.8)
    gl = _unflat(g.cpu().numpy(), sizes)
    for l, ((dW, db), (rW, rb)) in enumerate(zip(gl, g_ref)):
        assert _rel(dW, rW) <= 1e-4, (l, "W", _rel(dW, rW))
        assert _rel(db, rb) <= 1e-4, (l, "b", _rel(db, rb))
    # weight 0 is the plain grouped loss again
    net.set_subspace(0.0)
    loss0, _ = net.gradients(xd, td, group=group)
    assert abs(loss0 - mlp.loss(params, x.astype(np.float64), t64, group=group)) <= 1e-4 * loss0


def test_subspace_weight_errors():
    net = kl.MLP([3, 4, 66])
    with pytest.raises(kl.KLError):
        net.set_subspace(-1.0)
    with pytest.raises(kl.KLError):
        net.set_subspace(float("nan"))
    net.set_subspace(1.0)
    x = torch.zeros((2, 3), dtype=torch.float32, device="cuda")
    t = torch.ones((2, 66), dtype=torch.float32, device="cuda")
    with pytest.raises(kl.KLError):
        net.gradients(x, t, group=2)           # 33 groups per row: more than 32
    net.gradients(x, t, group=3)                # 22 groups
