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
            s = np.linalg.svd(V[:, i:j].conj().T @ W[:, i:j], compute_uv=False)
            worst = max(worst, float(np.sqrt(max(0.0, 1.0 - min(1.0, s.min()) ** 2))))
        i = j
    return worst


def matrix_with_empty_runs():
    """Rows of 1-12 nonzeros with empty rows at the start and end of 32-row
    runs, a fully empty run, an empty last row, n not a multiple of 32."""
    import numpy as np
    import scipy.sparse as sp

    import workloads as W

    n = 3001
    rng = np.random.default_rng(17)
    deg = rng.integers(1, 13, n)
    empty = [0, 31, 32, 63, 2999, 3000] + list(range(64, 130))
    deg[empty] = 0
    rows = np.repeat(np.arange(n), deg)
    cols = rng.integers(0, n, deg.sum())
    a = sp.csr_matrix((rng.standard_normal(deg.sum()), (rows, cols)), shape=(n, n))
    a.sum_duplicates()
    a.sort_indices()
    return W.CSRMatrix(n, a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data, 1.0)
