"""Matrix-free isogeometric Galerkin Karhunen-Loeve eigensolver for one AMD MI355X.

The computation lives in the HIP/C++ library lib/libklmf.so (C ABI: include/kl.h);
this package is its thin Python binding.  Build the library with
`python -m paper_2011_13861_amd.build` (or __graft_entry__.build()).
"""

from ._binding import (Batch, KLError, MLP, Problem, PRECISIONS, EXPORTS, LIB_PATH, lib,  # noqa: F401
                       make_desc)


def new_block(n, nvec, device="cuda"):
    """Zero FP64 device block of shape (n, nvec) in column-major storage."""
    import torch
    return torch.zeros((nvec, n), dtype=torch.float64, device=device).T


def to_device_block(a, device="cuda"):
    """Copies a host (n, nvec) array into a column-major FP64 device block."""
    import numpy as np
    import torch
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(device).T
