"""The stage-5 autotuner: it picks a setting among the candidates it timed, records it in
its JSON cache under the (architecture, dimension, kind, precision, size) key, the cached
setting is applied to a fresh handle, and results stay correct under the tuned setting."""

import json

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
import workloads
from paper_2011_13861_amd import autotune
from oracle import cstage5, operator

pytestmark = pytest.mark.gpu


def test_tune_problem_records_and_reapplies(tmp_path):
    path = str(tmp_path / "tune.json")
    desc = workloads.quarter_annulus(20, 3, "sqexp", (0.5, 0.5))
    G = kl.Problem(desc)
    best = autotune.tune_problem(G, "sqexp", precisions=("f32", "f64"), reps=5, max_split=16, path=path)
    data = json.load(open(path))
    for prec in ("f32", "f64"):
        rb, ns, us = best[prec]
        key = autotune.problem_key(G, "sqexp", prec)
        assert data[key]["rb"] == rb and data[key]["nsplit"] == ns and us > 0
        assert G.stage5_config(prec) == (rb if prec != "f64" else 4, ns)
        F = kl.Problem(desc)
        assert autotune.apply_cached(F, "sqexp", prec, path=path) is not None
        assert F.stage5_config(prec)[1] == ns
    # correctness under the tuned setting
    P = operator.Problem(desc)
    V = workloads.random_block(P.N, 9, seed=2)
    x = kl.to_device_block(V)
    y = kl.new_block(G.N, 9)
    G.apply(x, y, "f32")
    torch.cuda.synchronize()
    ref = P.apply(V)
    assert np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref) <= 2e-6


def test_tune_problem_apply_objective(tmp_path):
    """Tuning on the whole apply records its own cache entry (apart from the
    kernel-alone one) and the setting it picks keeps the apply correct."""
    path = str(tmp_path / "tune.json")
    desc = workloads.quarter_annulus(24, 3, "sqexp", (0.5, 0.5))
    G = kl.Problem(desc)
    rb, ns, us = autotune.tune_problem(G, "sqexp", precisions=("f32",), reps=5, max_split=12, path=path,
                                       objective="apply")["f32"]
    data = json.load(open(path))
    assert autotune.problem_key(G, "sqexp", "f32") not in data
    e = data[autotune.problem_key(G, "sqexp", "f32", "apply")]
    assert (e["rb"], e["nsplit"]) == (rb, ns) and us > 0
    assert isinstance(e["fuse"], bool)            # fused or per-direction Kronecker launches
    F = kl.Problem(desc)
    assert autotune.apply_cached(F, "sqexp", "f32", path=path) is None
    assert autotune.apply_cached(F, "sqexp", "f32", path=path, objective="apply") is not None
    assert F.stage5_config("f32") == (rb, ns)
    P = operator.Problem(desc)
    V = workloads.random_block(P.N, 32, seed=3)
    x = kl.to_device_block(V)
    y = kl.new_block(F.N, 32)
    F.apply(x, y, "f32")
    torch.cuda.synchronize()
    ref = P.apply(V)
    assert np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref) <= 2e-6
    with pytest.raises(ValueError):
        autotune.tune_problem(G, "sqexp", objective="wall")


def test_tune_batch_records_and_stays_correct(tmp_path):
    path = str(tmp_path / "tune.json")
    descs = workloads.batch_problems(7, count=6)
    kinds = [d["cov"]["kind"] for d in descs]
    B = kl.Batch(descs)
    rb, lc, us = autotune.tune_batch(B, kinds, "f32", reps=3, path=path)
    data = json.load(open(path))
    assert data[autotune.batch_key(B, kinds, "f32")]["lchunk"] == lc and us > 0
    x = B.arena(4)
    host = []
    for i in range(B.n):
        V = workloads.random_block(B.N[i], 4, seed=i)
        B.block(x, i, 4).copy_(torch.from_numpy(V))
        host.append(V)
    y = B.arena(4)
    B.apply(x, y, 4, "f32")
    torch.cuda.synchronize()
    for i in (0, 3):
        P = operator.Problem(descs[i])
        ref = P.apply(host[i], stage5=lambda Y: cstage5.stage5(P, Y))
        out = B.block(y, i, 4).cpu().numpy()
        assert np.linalg.norm(out - ref) / np.linalg.norm(ref) <= 2e-6
