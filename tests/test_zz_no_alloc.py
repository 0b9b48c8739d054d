"""kl_apply_noalloc (the apply with every intermediate in the library's static device
scratch) against kl_apply, through the C ABI: two calls in a row on one device, the second
on a smaller problem (the scratch keeps the first call's contents, which must not leak into
the second), in every precision, with ragged column counts; and the size limit."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
import workloads

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6, "bf16x3": 5e-5, "bf16": 5e-3}


def _noalloc(G, x, y, precision):
    L = kl.lib()
    nvec = x.shape[1]
    return L.kl_apply_noalloc(G.handle, kl.PRECISIONS[precision], nvec, ctypes.c_void_p(x.data_ptr()),
                              x.stride(1), ctypes.c_void_p(y.data_ptr()), y.stride(1),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x3", "bf16"])
def test_noalloc_matches_apply_on_two_calls(precision):
    cases = [(workloads.config("cube24")[0], 35), (workloads.config("square16")[0], 7)]
    for desc, nvec in cases:
        G = kl.Problem(desc)
        x = kl.to_device_block(workloads.random_block(G.N, nvec, seed=nvec))
        ref = kl.new_block(G.N, nvec)
        G.apply(x, ref, precision)
        out = kl.new_block(G.N, nvec)
        st = _noalloc(G, x, out, precision)
        assert st == 0, kl.lib().kl_last_error()
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        err = np.max(np.abs(a - b)) / np.max(np.abs(b)) if precision == "f64" else np.linalg.norm(a - b) / np.linalg.norm(b)
        print("noalloc", precision, G.N, nvec, err)
        assert err <= TOL[precision], (precision, G.N, err)


def test_noalloc_rejects_problems_beyond_the_scratch():
    G = kl.Problem(workloads.sine_cube(40, 2, "exp", 0.5))
    x = kl.new_block(G.N, 1)
    y = kl.new_block(G.N, 1)
    assert _noalloc(G, x, y, "f64") == -1
    assert b"MiB of scratch" in kl.lib().kl_last_error()
