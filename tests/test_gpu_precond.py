"""Preconditioned LOBPCG and steepest descent (W <- T R with the Jacobi
preconditioner T = diag(1/|a_ii|)) on the GPU against the oracle (GPU).

The oracle's preconditioned runs are insensitive to rounding on these
matrices (start blocks differing by 1e-14 move r(j) by at most 6e-7 while
r(j) > 1e-6), so the residual histories are compared step by step; the GPU's
implicit orthonormalization of W and the oracle's explicit projections agree
to that level.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from tests.gpu_util import cluster_angles, gpu_ctx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _csr(S, name):
    S = S.tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return W.CSRMatrix(S.shape[0], S.indptr.astype(np.int64), S.indices.astype(np.int32),
                       S.data.astype(np.float64), float(abs(S).sum(axis=1).max()), name)


def _scaled_laplacian(m=24, seed=3):
    L = W.laplacian_2d(m).to_scipy()
    d = np.exp(np.random.default_rng(seed).uniform(-2.0, 2.0, L.shape[0]))
    return _csr(sp.diags(np.sqrt(d)) @ L @ sp.diags(np.sqrt(d)), f"scaled_laplace2d_{m}")


def _run(ctx, A, solver, precond, n_ev=6, n_extra=6, n_es=8, rtol=1e-5):
    from paper_2409_05572_amd import api

    nb = n_ev + n_extra
    X0 = W.gaussian_block(A.n, nb, 5)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve(ctx, M, X0, n_ev, n_extra, history_cap=4000, solver=solver, strategy="fix",
                             n_es=n_es, max_iter=3000, precond=precond)
    f = O.lobpcg if solver == "lobpcg" else O.steepest_descent
    S = A.to_scipy()
    ref = f(S, X0, n_ev, A.anorm, tol=1e-8, n_es=n_es, se=O.SEParams("fix"), max_iter=3000,
            precond=O.jacobi_preconditioner(S) if precond == "jacobi" else None)
    exact = np.sort(np.linalg.eigvalsh(S.toarray()))[:n_ev]
    assert info.converged and ref.converged
    assert np.max(np.abs(lam - exact) / np.abs(exact)) <= 1e-10
    assert np.max(np.abs(lam - ref.lam) / np.abs(ref.lam)) <= 1e-10
    R = S @ V - V * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))) <= 1e-8 * 1.0001
    assert np.abs(V.T @ V - np.eye(n_ev)).max() <= 1e-12
    assert cluster_angles(lam, V, ref.V) <= 1e-6
    r_gpu = info.history[:, 1]
    r_ref = np.array([h["r"] for h in ref.history])
    L = min(len(r_gpu), len(r_ref))
    big = r_ref[:L] > 1e-6
    assert big.sum() >= 10
    np.testing.assert_allclose(r_gpu[:L][big], r_ref[:L][big], rtol=rtol)
    return info, ref


@pytest.mark.parametrize("solver", ["lobpcg", "sd"])
def test_jacobi_on_a_badly_scaled_laplacian_matches_oracle(ctx, solver):
    A = _scaled_laplacian()
    info, ref = _run(ctx, A, solver, "jacobi")
    assert abs(info.iterations - ref.iterations) <= 1
    # the preconditioner pays: far fewer iterations than T = I (oracle count)
    plain = (O.lobpcg if solver == "lobpcg" else O.steepest_descent)(
        A.to_scipy(), W.gaussian_block(A.n, 12, 5), 6, A.anorm, tol=1e-8, n_es=8, se=O.SEParams("fix"),
        max_iter=3000)
    assert 2 * info.iterations < plain.iterations


@pytest.mark.parametrize("solver", ["lobpcg", "sd"])
def test_jacobi_on_anderson_matches_oracle(ctx, solver):
    """Indefinite Anderson matrix (diagonal 6 + U[-4, 4]); brute-force spectrum."""
    A = W.anderson_3d(14, 4.0, 103)
    info, ref = _run(ctx, A, solver, "jacobi", rtol=1e-4)
    assert abs(info.iterations - ref.iterations) <= 2


def test_precond_options_are_validated(ctx):
    from paper_2409_05572_amd import api
    from paper_2409_05572_amd._lib import SeError

    A = W.laplacian_2d(8)
    M = api.Matrix.from_csr(ctx, A)
    X0 = W.gaussian_block(A.n, 8, 1)
    with pytest.raises(SeError, match="invalid"):
        api.solve(ctx, M, X0, 4, 4, solver="si", precond="jacobi")
    with pytest.raises(SeError, match="invalid"):
        api.solve(ctx, M, X0, 4, 4, solver="tracemin", precond="jacobi")
    with pytest.raises(SeError, match="unsupported"):
        api.solve(ctx, M, X0, 4, 4, precond="jacobi", precision="fp32")


def test_jacobi_on_a_larger_anderson_matrix(ctx):
    """Anderson 50^3 + U[-4, 4] (n = 125,000), n_ev 40, block 56, fix: the
    preconditioned and plain GPU solves reach the same eigenvalues, each
    sampled pair passes the stopping test on the host, and the preconditioner
    takes fewer iterations."""
    from paper_2409_05572_amd import api

    A = W.anderson_3d(50, 4.0, 103)
    X0 = W.gaussian_block(A.n, 56, 9)
    M = api.Matrix.from_csr(ctx, A)
    lam0, V0, i0 = api.solve(ctx, M, X0, 40, 16, strategy="fix")
    lam1, V1, i1 = api.solve(ctx, M, X0, 40, 16, strategy="fix", precond="jacobi")
    assert i0.converged and i1.converged
    assert np.max(np.abs(lam1 - lam0)) <= 1e-9 * A.anorm
    assert i1.iterations < i0.iterations
    cols = np.array([0, 13, 39])
    R = A.to_scipy() @ V1[:, cols] - V1[:, cols] * lam1[cols][None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V1[:, cols], axis=0))) <= 1e-8 * 1.0001
