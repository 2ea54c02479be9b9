"""Whole solves on the GPU against the FP64 oracle and closed forms (GPU).

Eigenvalues are compared one to one; eigenvectors through principal angles of
complete clusters (repeated eigenvalues make single vectors non-unique) and
through the stopping test recomputed on the host with the oracle's product.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import _pins as pins
from tests.gpu_util import cluster_angles, gpu_ctx, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _residual_ratio(A, lam, V):
    R = O.solvers._apply(A.to_scipy(), V) - V * lam[None, :]
    return np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))


def _gpu_solve(ctx, A, X0, n_ev, n_extra, **kw):
    from paper_2409_05572_amd import api

    M = api.Matrix.from_csr(ctx, A)
    return api.solve(ctx, M, X0, n_ev, n_extra, history_cap=4000, **kw)


def _assert_parity(A, lam, V, ref, exact=None, tol=1e-8, lam_rtol=1e-10):
    assert np.max(np.abs(lam - ref.lam) / np.abs(ref.lam)) <= lam_rtol
    if exact is not None:
        assert np.max(np.abs(lam - exact) / np.abs(exact)) <= lam_rtol
    assert np.max(_residual_ratio(A, lam, V)) <= tol * 1.0001
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() <= 1e-12
    assert cluster_angles(lam, V, ref.V) <= 1e-6


def test_config1_lobpcg_matches_oracle(ctx):
    A = W.laplacian_2d(32)
    X0 = W.gaussian_block(A.n, 16, 201)
    lam, V, info = _gpu_solve(ctx, A, X0, 8, 8)
    ref = O.lobpcg(A.to_scipy(), X0, 8, A.anorm, tol=1e-8)
    assert info.converged and info.status == 0
    assert info.max_stop_ratio <= 1e-8
    _assert_parity(A, lam, V, ref, pins.laplacian_spectrum(32, 2, 8))
    assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // 10)


def test_config1_subspace_iteration_matches_oracle(ctx):
    A = W.laplacian_2d(32)
    X0 = W.gaussian_block(A.n, 16, 201)
    lam, V, info = _gpu_solve(ctx, A, X0, 8, 8, solver="si")
    ref = O.subspace_iteration(A.to_scipy(), X0, 8, A.anorm, tol=1e-8)
    assert info.converged
    _assert_parity(A, lam, V, ref, pins.laplacian_spectrum(32, 2, 8), lam_rtol=1e-10)
    assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // 20)


@pytest.mark.parametrize("strategy", ["none", "fix", "slope", "slopek"])
def test_lobpcg_shrink_expand_3d_matches_oracle(ctx, strategy):
    m, n_ev, n_extra = 16, 32, 16
    A = W.laplacian_3d(m)
    X0 = W.gaussian_block(A.n, n_ev + n_extra, 7)
    lam, V, info = _gpu_solve(ctx, A, X0, n_ev, n_extra, strategy=strategy)
    ref = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 5,
                   se=O.SEParams(strategy))
    assert info.converged
    _assert_parity(A, lam, V, ref, pins.laplacian_spectrum(m, 3, n_ev), lam_rtol=1e-10)
    if strategy != "none":
        assert info.n_shrinks >= 1
        hist = info.history
        assert np.any(hist[:, 7].astype(int) & 2)
        assert hist[:, 3].min() == n_ev + 5


@pytest.mark.parametrize("strategy", ["fix", "slopek"])
def test_si_shrink_expand_matches_oracle(ctx, strategy):
    m, n_ev, n_extra = 20, 6, 6
    A = W.laplacian_2d(m)
    X0 = W.gaussian_block(A.n, n_ev + n_extra, 5)
    lam, V, info = _gpu_solve(ctx, A, X0, n_ev, n_extra, solver="si", strategy=strategy,
                              n_es=n_ev + 2)
    ref = O.subspace_iteration(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                               se=O.SEParams(strategy))
    assert info.converged and info.n_shrinks >= 1
    _assert_parity(A, lam, V, ref, pins.laplacian_spectrum(m, 2, n_ev), lam_rtol=1e-10)


def test_anderson_small_matches_oracle(ctx):
    """Indefinite Anderson matrix (parity unpinned by closed form): oracle agreement."""
    A = W.anderson_3d(14, 4.0, 103)
    X0 = W.gaussian_block(A.n, 30, 8)
    lam, V, info = _gpu_solve(ctx, A, X0, 20, 10, strategy="fix")
    ref = O.lobpcg(A.to_scipy(), X0, 20, A.anorm, tol=1e-8, n_es=25, se=O.SEParams("fix"))
    assert info.converged and ref.converged
    assert np.max(np.abs(lam - ref.lam) / np.maximum(np.abs(ref.lam), 1e-3 * A.anorm)) <= 1e-10
    assert np.max(_residual_ratio(A, lam, V)) <= 1e-8 * 1.0001


@pytest.mark.parametrize("strategy", ["none", "fix", "slopek"])
def test_steepest_descent_matches_oracle(ctx, strategy):
    """Algorithm 2 on the GPU (the LOBPCG engine without P) against the
    oracle's steepest descent and the closed form."""
    m, n_ev, nb = 16, 6, 12
    A = W.laplacian_2d(m)
    X0 = W.gaussian_block(A.n, nb, 7)
    lam, V, info = _gpu_solve(ctx, A, X0, n_ev, nb - n_ev, solver="sd", strategy=strategy, n_es=n_ev + 2,
                              max_iter=3000)
    ref = O.steepest_descent(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                             se=O.SEParams(strategy), max_iter=3000)
    assert info.converged and ref.converged
    _assert_parity(A, lam, V, ref, pins.laplacian_spectrum(m, 2, n_ev))
    assert abs(info.iterations - ref.iterations) <= max(5, ref.iterations // 7)
    assert np.all(info.history[:, 4] == 0)  # no P block
    if strategy != "none":
        assert info.n_shrinks >= 1


def test_steepest_descent_mixed_precision(ctx):
    A = W.laplacian_2d(16)
    X0 = W.gaussian_block(A.n, 12, 7)
    lam, V, info = _gpu_solve(ctx, A, X0, 6, 6, solver="sd", precision="fp32", strategy="fix",
                              max_iter=3000)
    assert info.converged and info.lp_iterations >= 1
    assert np.max(np.abs(lam - pins.laplacian_spectrum(16, 2, 6)) / lam) <= 1e-10
    assert np.max(_residual_ratio(A, lam, V)) <= 1e-8 * 1.0001
    assert np.abs(V.T @ V - np.eye(6)).max() <= 1e-12


def test_device_pointers_give_identical_result(ctx):
    import torch

    A = W.laplacian_2d(24)
    X0 = W.gaussian_block(A.n, 12, 3)
    lam_h, V_h, _ = _gpu_solve(ctx, A, X0, 6, 6, strategy="fix")
    X0d = to_dev(X0.T.copy())
    lam_d, V_d, info = _gpu_solve(ctx, A, X0d, 6, 6, strategy="fix")
    torch.cuda.synchronize()
    assert np.array_equal(lam_h, lam_d.cpu().numpy())
    assert np.array_equal(V_h, V_d.cpu().numpy().T)


def test_solves_are_bitwise_deterministic(ctx):
    A = W.laplacian_3d(12)
    X0 = W.gaussian_block(A.n, 24, 4)
    a = _gpu_solve(ctx, A, X0, 16, 8, strategy="slopek")
    b = _gpu_solve(ctx, A, X0, 16, 8, strategy="slopek")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2].iterations == b[2].iterations


def test_not_converged_returns_best_iterate(ctx):
    A = W.laplacian_2d(16)
    X0 = W.gaussian_block(A.n, 8, 1)
    lam, V, info = _gpu_solve(ctx, A, X0, 4, 4, max_iter=2)
    assert info.status == 1 and not info.converged and info.iterations == 2
    assert np.all(np.isfinite(lam)) and np.abs(V.T @ V - np.eye(4)).max() < 1e-10


def test_invalid_arguments_are_rejected(ctx):
    from paper_2409_05572_amd import api
    from paper_2409_05572_amd._lib import SeError

    A = W.laplacian_2d(8)
    with pytest.raises(SeError, match="invalid"):
        _gpu_solve(ctx, A, W.gaussian_block(A.n, 70, 1), 60, 10)  # nb > n
    bad = W.laplacian_2d(8)
    bad.colind = bad.colind.copy()
    bad.colind[3] = 10**6
    with pytest.raises(SeError, match="invalid"):
        api.Matrix.from_csr(ctx, bad)
    nanm = W.laplacian_2d(8)
    nanm.val = nanm.val.copy()
    nanm.val[0] = np.nan
    with pytest.raises(SeError, match="invalid"):
        api.Matrix.from_csr(ctx, nanm)


def test_residual_block_orthonormalized_implicitly_except_at_expansions(ctx):
    """Most iterations whiten the Gram matrix of [X, P, W] in coefficient
    space (history bit 3); expansion iterations (bit 0) project and
    orthonormalize W explicitly. The pairs still meet the closed form, the
    stopping test and orthonormality to 1e-12."""
    m = 16
    A = W.laplacian_3d(m)
    X0 = W.gaussian_block(A.n, 48, 203)
    lam, V, info = _gpu_solve(ctx, A, X0, 32, 16, strategy="fix")
    fl = info.history[:, 7].astype(int)
    assert info.converged and info.n_expands >= 1
    assert ((fl & 8) != 0).sum() >= 0.6 * len(fl)
    assert not np.any(((fl & 1) != 0) & ((fl & 8) != 0))
    exact = pins.laplacian_spectrum(m, 3, 32)
    assert np.max(np.abs(lam - exact) / exact) <= 1e-10
    assert np.max(_residual_ratio(A, lam, V)) <= 1e-8 * 1.0001
    assert np.abs(V.T @ V - np.eye(32)).max() <= 1e-12


def test_explicit_and_implicit_orthonormalization_agree(ctx):
    """implicit_pivot > 1 forces the explicit projection and Cholesky-QR of W
    in every iteration (the path taken when the Schur pivots are small); a tiny
    threshold takes the implicit path in every iteration without an
    expansion. Both meet the same bars and find the same pairs."""
    from tests.gpu_util import cluster_angles

    m = 14
    A = W.laplacian_3d(m)
    X0 = W.gaussian_block(A.n, 40, 207)
    exact = pins.laplacian_spectrum(m, 3, 28)
    runs = {}
    for piv in (2.0, 1e-12):
        lam, V, info = _gpu_solve(ctx, A, X0, 28, 12, strategy="fix", implicit_pivot=piv)
        fl = info.history[:, 7].astype(int)
        assert info.converged and info.n_expands >= 1
        if piv > 1:
            assert not np.any(fl & 8)
        else:
            body = fl[:-1]  # the last row is the converged check, before any W is formed
            assert np.all(((body & 8) != 0) | ((body & 1) != 0))
        assert np.max(np.abs(lam - exact) / exact) <= 1e-10
        assert np.max(_residual_ratio(A, lam, V)) <= 1e-8 * 1.0001
        assert np.abs(V.T @ V - np.eye(28)).max() <= 1e-12
        runs[piv] = (lam, V)
    assert cluster_angles(runs[2.0][0], runs[2.0][1], runs[1e-12][1]) <= 1e-6


@pytest.mark.parametrize("solver,precision", [("lobpcg", "fp64"), ("si", "fp64"), ("lobpcg", "fp32")])
def test_seeded_start_block_matches_the_host_generator(ctx, solver, precision):
    """X0 = NULL: the library's start block is the SplitMix64 block of
    workloads.seeded_uniform_block (exact in FP64), so the solve is bitwise the
    one started from the host copy of that block."""
    A = W.laplacian_2d(24)
    seed = 12345
    lam_n, V_n, info_n = _gpu_solve(ctx, A, None, 6, 6, solver=solver, precision=precision, seed=seed,
                                    strategy="fix")
    X0 = W.seeded_uniform_block(A.n, 12, seed)
    lam_h, V_h, info_h = _gpu_solve(ctx, A, X0, 6, 6, solver=solver, precision=precision, strategy="fix")
    assert info_n.converged and info_n.iterations == info_h.iterations
    assert np.array_equal(lam_n, lam_h) and np.array_equal(V_n, V_h)
    assert np.max(np.abs(lam_n - pins.laplacian_spectrum(24, 2, 6)) / lam_n) <= 1e-10


def test_zero_anorm_takes_the_gershgorin_bound(ctx):
    """anorm = 0 at matrix creation: the library uses max_i sum_j |a_ij|, the
    bound the Anderson workload passes explicitly, and the solve is the same."""
    from paper_2409_05572_amd import api

    A = W.anderson_3d(10, 4.0, 9)
    S = A.to_scipy()
    gersh = float(abs(S).sum(axis=1).max())
    M0 = api.Matrix(ctx, A.n, A.rowptr, A.colind, A.val, 0.0)
    assert abs(M0.anorm - gersh) <= 1e-14 * gersh
    X0 = W.gaussian_block(A.n, 16, 5)
    r0 = api.solve(ctx, M0, X0, 10, 6, strategy="fix")
    r1 = api.solve(ctx, api.Matrix(ctx, A.n, A.rowptr, A.colind, A.val, M0.anorm), X0, 10, 6, strategy="fix")
    assert r0[2].converged and np.array_equal(r0[0], r1[0]) and np.array_equal(r0[1], r1[1])
    with pytest.raises(Exception):
        api.Matrix(ctx, A.n, A.rowptr, A.colind, A.val, -1.0)


def test_invalid_implicit_pivot_is_rejected(ctx):
    from paper_2409_05572_amd._lib import SeError

    A = W.laplacian_2d(8)
    X0 = W.gaussian_block(A.n, 6, 1)
    for bad in (-1.0, float("nan")):
        with pytest.raises(SeError):
            _gpu_solve(ctx, A, X0, 3, 3, implicit_pivot=bad)


def test_full_config2_lobpcg_shrink_expand(ctx):
    """3-D 128^3 Laplacian, 64 wanted + 32 extra, fix strategy, at full size
    and in the launch configuration the benchmark times: every eigenvalue
    against the closed form, within 1e-10 and within the per-pair bound
    |theta - lambda| <= ||r||^2 / gap (gap to the nearest eigenvalue outside
    the pair's cluster, from the closed form); the stopping test recomputed
    on the host with the oracle's product for all 64 eigenvectors (in row
    chunks); orthonormality of the returned block."""
    A = W.laplacian_3d(128)
    X0 = W.gaussian_block(A.n, 96, 202)
    lam, V, info = _gpu_solve(ctx, A, X0, 64, 32, strategy="fix")
    assert info.converged and info.n_shrinks >= 1
    exact_all = pins.laplacian_spectrum(128, 3, 100)
    exact = exact_all[:64]
    assert np.max(np.abs(lam - exact) / exact) <= 1e-10
    S = A.to_scipy()
    rn = np.zeros(64)
    for c0 in range(0, 64, 16):  # column chunks keep the host copy of A V small
        R = S @ V[:, c0:c0 + 16] - V[:, c0:c0 + 16] * lam[None, c0:c0 + 16]
        rn[c0:c0 + 16] = np.linalg.norm(R, axis=0)
    xn = np.linalg.norm(V, axis=0)
    assert np.max(rn / (A.anorm * xn)) <= 1e-8 * 1.0001
    for i in range(64):
        others = exact_all[np.abs(exact_all - exact[i]) > 1e-9 * exact[i]]
        gap = np.min(np.abs(others - lam[i]))
        assert abs(lam[i] - exact[i]) <= max(1e-13 * exact[i], (rn[i] / xn[i]) ** 2 / gap)
    assert np.abs(V.T @ V - np.eye(64)).max() <= 1e-12


def test_matrix_released_after_its_context(ctx):
    """Finalizers can run in any order (a garbage cycle holding both): a
    matrix destroyed after its context must release cleanly and leave no HIP
    error behind for the next solve on another context."""
    from paper_2409_05572_amd import api

    other = api.Context(0)
    A = W.laplacian_2d(8)
    M = api.Matrix.from_csr(other, A)
    other.close()
    M.close()
    lam, V, info = _gpu_solve(ctx, A, W.gaussian_block(A.n, 8, 1), 4, 4)
    assert info.converged and info.status == 0


@pytest.mark.parametrize("strategy", ["none", "fix"])
def test_iteration_counts_on_the_benchmark_shape_match_the_oracle(ctx, strategy):
    """The benchmark's block shape (64 wanted + 32 extra, start seed 202) on a
    32^3 Laplacian: the fixed-block and the shrink-and-expand iteration counts
    agree with the oracle's (98 and 103 there: at this size shrink-and-expand
    takes a few more iterations, as the paper reports about 10% more), so the
    GPU's fixed-vs-S&E comparison runs the same iteration as the oracle."""
    m = 32
    A = W.laplacian_3d(m)
    X0 = W.gaussian_block(A.n, 96, 202)
    lam, V, info = _gpu_solve(ctx, A, X0, 64, 32, strategy=strategy)
    ref = O.lobpcg(A.to_scipy(), X0, 64, A.anorm, tol=1e-8, n_es=69, se=O.SEParams(strategy))
    assert info.converged and ref.converged
    assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // 20)
    assert abs(info.n_shrinks - ref.n_shrinks) <= 1
    exact = pins.laplacian_spectrum(m, 3, 64)
    assert np.max(np.abs(lam - exact) / exact) <= 1e-10
    assert np.max(_residual_ratio(A, lam, V)) <= 1e-8 * 1.0001
