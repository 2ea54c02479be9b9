"""Shared helpers of the GPU parity tests."""
import numpy as np
import pytest


def gpu_ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2409_05572_amd import api

    return api.Context(0)


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def cluster_angles(lam, V, W, rtol=1e-6):
    """Largest sin of principal angles between V and W over complete clusters.

    Clusters are runs of eigenvalues closer than rtol (relative); a trailing
    cluster that may continue past the last index is skipped.
    """
    n_ev = len(lam)
    worst = 0.0
    i = 0
    while i < n_ev:
        j = i + 1
        while j < n_ev and abs(lam[j] - lam[j - 1]) <= rtol * max(abs(lam[j]), 1e-300):
            j += 1
        if j < n_ev:  # complete cluster [i, j)
            s = np.linalg.svd(V[:, i:j].T @ W[:, i:j], compute_uv=False)
            worst = max(worst, float(np.sqrt(max(0.0, 1.0 - min(1.0, s.min()) ** 2))))
        i = j
    return worst
