"""Shared helpers of the GPU tests (device inputs, oracle comparisons)."""
import sys

import numpy as np
import scipy.sparse as sp


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def scipy_csr(H):
    """scipy matrix of a lradi.HostCsr (library generator output)."""
    return sp.csr_matrix((H.val, H.colind, H.rowptr), shape=(H.n, H.n))
