"""TraceMIN (Algorithm 4) on the GPU against the oracle's TraceMIN (GPU).

The inner projected CG runs per column on the device (column dot products,
a fused step that updates D and R and sums the new residual norms, and the
direction update); the oracle runs the same CG in numpy. TraceMIN is not
sensitive to rounding here (two oracle runs whose start blocks differ by
1e-14 agree in r(j) to 1e-8 while r(j) > 1e-6), so the residual histories are
compared step by step.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from tests import _pins as pins
from tests.gpu_util import cluster_angles, gpu_ctx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _run(ctx, A, n_ev, n_extra, strategy="none", n_es=0, cg_steps=0, kind="xdrop", x0_seed=5):
    from paper_2409_05572_amd import api

    nb = n_ev + n_extra
    X0 = W.gaussian_block(A.n, nb, x0_seed)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve(ctx, M, X0, n_ev, n_extra, history_cap=4000, solver="tracemin",
                             strategy=strategy, n_es=n_es, max_iter=3000, cg_steps=cg_steps,
                             expand_vectors=kind, seed=11, r_warm=1e-2)
    draw = lambda e, d: W.seeded_expansion_block(A.n, d, nb, e, 11)  # noqa: E731
    ref = O.tracemin(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8,
                     n_es=n_es if n_es else n_ev + min(5, n_extra - 1),
                     se=O.SEParams(strategy, r_warm=1e-2), max_iter=3000,
                     cg_steps=cg_steps if cg_steps else 5, expand_vectors=kind, random_block=draw)
    return lam, V, info, ref


def _assert_same(A, lam, V, info, ref, exact, n_ev):
    assert info.converged and ref.converged
    assert np.max(np.abs(lam - ref.lam) / np.abs(ref.lam)) <= 1e-10
    assert np.max(np.abs(lam - exact) / np.abs(exact)) <= 1e-10
    R = O.solvers._apply(A.to_scipy(), V) - V * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))) <= 1e-8 * 1.0001
    assert np.abs(V.T @ V - np.eye(n_ev)).max() <= 1e-12
    assert cluster_angles(lam, V, ref.V) <= 1e-6
    r_gpu = info.history[:, 1]
    r_ref = np.array([h["r"] for h in ref.history])
    L = min(len(r_gpu), len(r_ref))
    big = r_ref[:L] > 1e-6
    assert big.sum() >= 5
    np.testing.assert_allclose(r_gpu[:L][big], r_ref[:L][big], rtol=1e-6)
    assert abs(info.iterations - ref.iterations) <= 1
    assert info.n_shrinks == ref.n_shrinks and info.n_expands == ref.n_expands


@pytest.mark.parametrize("strategy", ["none", "fix", "slopek"])
def test_tracemin_matches_oracle(ctx, strategy):
    A = W.laplacian_2d(20)
    lam, V, info, ref = _run(ctx, A, 6, 6, strategy=strategy, n_es=8)
    if strategy != "none":
        assert info.n_shrinks >= 1
    _assert_same(A, lam, V, info, ref, pins.laplacian_spectrum(20, 2, 6), 6)


@pytest.mark.parametrize("cg_steps", [2, 10])
def test_tracemin_inner_steps(ctx, cg_steps):
    A = W.laplacian_2d(20)
    lam, V, info, ref = _run(ctx, A, 6, 6, strategy="fix", n_es=8, cg_steps=cg_steps)
    _assert_same(A, lam, V, info, ref, pins.laplacian_spectrum(20, 2, 6), 6)


def test_tracemin_odd_width_and_random_expansion(ctx):
    A = W.laplacian_2d(20)
    lam, V, info, ref = _run(ctx, A, 5, 4, strategy="fix", n_es=7, kind="random")
    assert info.n_expands >= 1
    _assert_same(A, lam, V, info, ref, pins.laplacian_spectrum(20, 2, 5), 5)


def test_tracemin_block_64_on_3d_laplacian(ctx):
    A = W.laplacian_3d(16)
    lam, V, info, ref = _run(ctx, A, 40, 24, strategy="fix", n_es=45)
    _assert_same(A, lam, V, info, ref, pins.laplacian_spectrum(16, 3, 40), 40)


def test_tracemin_block_wider_than_a_workgroup(ctx):
    """Block 300 (> 256 threads: one column per thread in the CG kernels) on a
    sparse SPD matrix whose spectrum has a gap after the 260th eigenvalue."""
    n = 1200
    rng = np.random.default_rng(7)
    d = np.concatenate([np.linspace(1.0, 2.0, 260), np.linspace(10.0, 20.0, n - 260)])
    B = sp.random(n, n, density=4.0 / n, random_state=rng, format="csr")
    S = (sp.diags(d) + 0.05 * (B + B.T)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    anorm = float(abs(S).sum(axis=1).max())
    A = W.CSRMatrix(n, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64),
                    anorm, "gapped_spd_1200")
    exact = np.linalg.eigvalsh(S.toarray())[:260]
    lam, V, info, ref = _run(ctx, A, 260, 40)
    _assert_same(A, lam, V, info, ref, exact, 260)


def test_tracemin_options_are_validated(ctx):
    from paper_2409_05572_amd import api
    from paper_2409_05572_amd._lib import SeError

    A = W.laplacian_2d(8)
    M = api.Matrix.from_csr(ctx, A)
    X0 = W.gaussian_block(A.n, 8, 1)
    with pytest.raises(SeError, match="unsupported"):
        api.solve(ctx, M, X0, 4, 4, solver="tracemin", precision="fp32")
    with pytest.raises(SeError, match="invalid"):
        api.solve(ctx, M, X0, 4, 4, solver="tracemin", cg_steps=101)
    with pytest.raises(SeError, match="invalid"):
        api.solve(ctx, M, X0, 4, 4, solver="tracemin", filter_degree=3)


def test_tracemin_on_the_64_cubed_laplacian(ctx):
    """A larger solve (n = 262,144, block 48, fix): every eigenvalue against
    the closed form and the stopping test recomputed on the host for sampled
    eigenvectors."""
    from paper_2409_05572_amd import api

    A = W.laplacian_3d(64)
    X0 = W.gaussian_block(A.n, 48, 7)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve(ctx, M, X0, 32, 16, solver="tracemin", strategy="fix", max_iter=3000)
    assert info.converged
    exact = pins.laplacian_spectrum(64, 3, 32)
    assert np.max(np.abs(lam - exact) / exact) <= 1e-10
    cols = np.array([0, 5, 19, 31])
    R = O.solvers._apply(A.to_scipy(), V[:, cols]) - V[:, cols] * lam[cols][None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V[:, cols], axis=0))) <= 1e-8 * 1.0001
    assert np.abs(V.T @ V - np.eye(32)).max() <= 1e-12
