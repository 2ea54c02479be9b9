"""Vectors appended at an expansion (Section 6): random blocks and the powered
X_drop on the GPU against the oracle fed by the same seeded generator (GPU).

The random blocks are drawn on the device; the oracle draws them with
workloads.seeded_expansion_block. A different block would change the residual
history from the first expansion on, so the histories are compared step by
step as well as the final eigenpairs.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import _pins as pins
from tests.gpu_util import cluster_angles, gpu_ctx

pytestmark = pytest.mark.gpu

SEED = 11


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _run(ctx, solver, kind, strategy="fix", m=20, n_ev=6, n_extra=6, n_es=8, x0_seed=5):
    from paper_2409_05572_amd import api

    A = W.laplacian_2d(m)
    nb = n_ev + n_extra
    X0 = W.gaussian_block(A.n, nb, x0_seed)
    M = api.Matrix.from_csr(ctx, A)
    max_iter = 20000 if solver == "si" else 3000
    lam, V, info = api.solve(ctx, M, X0, n_ev, n_extra, history_cap=max_iter, solver=solver,
                             strategy=strategy, n_es=n_es, max_iter=max_iter, expand_vectors=kind,
                             seed=SEED)
    f = {"si": O.subspace_iteration, "lobpcg": O.lobpcg, "sd": O.steepest_descent}[solver]
    draw = lambda e, d: W.seeded_expansion_block(A.n, d, nb, e, SEED)  # noqa: E731
    ref = f(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_es, se=O.SEParams(strategy),
            max_iter=max_iter, expand_vectors=kind, random_block=draw)
    return A, lam, V, info, ref


def _assert_same_run(A, m, lam, V, info, ref, n_ev, rtol=1e-4, window=None, it_frac=20):
    assert info.converged and ref.converged
    assert info.n_expands >= 1 and ref.n_expands >= 1
    exact = pins.laplacian_spectrum(m, 2, n_ev)
    assert np.max(np.abs(lam - ref.lam) / ref.lam) <= 1e-10
    assert np.max(np.abs(lam - exact) / exact) <= 1e-10
    R = O.solvers._apply(A.to_scipy(), V) - V * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))) <= 1e-8 * 1.0001
    assert np.abs(V.T @ V - np.eye(n_ev)).max() <= 1e-12
    assert cluster_angles(lam, V, ref.V) <= 1e-6
    # the same trajectory: r(j) step by step while it is well above rounding
    r_gpu = info.history[:, 1]
    r_ref = np.array([h["r"] for h in ref.history])
    L = min(len(r_gpu), len(r_ref))
    if window is not None:
        first = next(h["j"] for h in ref.history if h["expand"])
        L = min(L, first + window)
    big = r_ref[:L] > 1e-6
    assert big.sum() >= 10
    np.testing.assert_allclose(r_gpu[:L][big], r_ref[:L][big], rtol=rtol)
    assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // it_frac)


@pytest.mark.parametrize("solver,kind", [("si", "random"), ("si", "powered"), ("lobpcg", "random"),
                                         ("sd", "random")])
def test_expansion_vectors_match_oracle(ctx, solver, kind):
    A, lam, V, info, ref = _run(ctx, solver, kind)
    if solver == "sd":
        # Steepest descent amplifies rounding: two oracle runs whose start
        # blocks differ by 1e-13 drift apart by up to 3e-4 in r(j) within
        # twenty iterations of the first expansion, while a different random
        # block moves r(j) by 0.15 - 0.3 there. Compare through that window.
        # Its final iteration count is rounding-decided on the GPU: start
        # blocks perturbed by 1e-14 (relative) end after 220 to 232
        # iterations (measured), so the count is held to 10% of the oracle's.
        _assert_same_run(A, 20, lam, V, info, ref, 6, rtol=3e-2, window=20, it_frac=10)
    else:
        _assert_same_run(A, 20, lam, V, info, ref, 6)


def test_powered_xdrop_under_slopek_matches_oracle(ctx):
    A, lam, V, info, ref = _run(ctx, "si", "powered", strategy="slopek")
    _assert_same_run(A, 20, lam, V, info, ref, 6)


def test_expansion_vector_options_are_validated(ctx):
    from paper_2409_05572_amd import api
    from paper_2409_05572_amd._lib import SeError

    A = W.laplacian_2d(8)
    M = api.Matrix.from_csr(ctx, A)
    X0 = W.gaussian_block(A.n, 8, 1)
    with pytest.raises(SeError, match="invalid"):
        api.solve(ctx, M, X0, 4, 4, strategy="fix", expand_vectors="powered")  # LOBPCG
    with pytest.raises(SeError, match="unsupported"):
        api.solve(ctx, M, X0, 4, 4, strategy="fix", expand_vectors="random", precision="fp32")
