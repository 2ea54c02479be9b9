"""HIP building blocks of the Rayleigh-Ritz step against their definitions (GPU)."""
import numpy as np
import pytest

import oracle.solvers as OS
import workloads as W
from tests.gpu_util import gpu_ctx, matrix_with_empty_runs, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _row_major(n, w, ld, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, ld))
    X[:, :w] = rng.standard_normal((n, w))
    return X


def _matrix_with_empty_and_dense_rows():
    import scipy.sparse as sp

    n = 3000
    rng = np.random.default_rng(7)
    a = sp.random(n, n, density=0.002, random_state=rng, format="lil")
    a[5, :] = rng.standard_normal(n)  # one dense (hub) row
    a[:, 5] = a[5, :].T
    for r in (0, 17, 2999):  # empty rows and columns
        a[r, :] = 0
        a[:, r] = 0
    a = sp.csr_matrix(a + a.T)
    a.sort_indices()
    return W.CSRMatrix(n, a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data, 1.0)


@pytest.mark.parametrize("w", [1, 2, 7, 16, 17, 48, 69, 96, 129, 250])
def test_spmm_matches_oracle_product(ctx, w):
    from paper_2409_05572_amd import api

    A = W.laplacian_3d(20)
    M = api.Matrix.from_csr(ctx, A)
    ld = w + (w % 2)
    X = _row_major(A.n, w, ld, w)
    Xd = to_dev(X)
    Yd = to_dev(np.full((A.n, ld), np.nan))
    api.spmm(ctx, M, Xd, Yd, w)
    Y = Yd.cpu().numpy()
    ref = OS._apply(A.to_scipy(), X[:, :w])
    bound = 1e-15 * 16 * (abs(A.to_scipy()) @ np.abs(X[:, :w]))
    assert np.all(np.abs(Y[:, :w] - ref) <= bound + 1e-300)


def test_spmm_empty_rows_and_hub_row(ctx):
    from paper_2409_05572_amd import api

    A = _matrix_with_empty_and_dense_rows()
    M = api.Matrix.from_csr(ctx, A)
    X = _row_major(A.n, 33, 34, 3)
    Yd = to_dev(np.full((A.n, 34), np.nan))
    api.spmm(ctx, M, to_dev(X), Yd, 33)
    Y = Yd.cpu().numpy()[:, :33]
    ref = OS._apply(A.to_scipy(), X[:, :33])
    assert np.all(Y[[0, 17, 2999]] == 0.0)
    assert np.allclose(Y, ref, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("w", [1, 2, 3, 64, 96, 127, 128, 129, 250])
def test_spmm_empty_rows_without_heavy_rows(ctx, w):
    from paper_2409_05572_amd import api

    A = matrix_with_empty_runs()
    assert np.diff(A.rowptr).max() <= 64  # no heavy rows: the streaming kernel alone
    M = api.Matrix.from_csr(ctx, A)
    ld = w + (w % 2)
    X = _row_major(A.n, w, ld, w + 3)
    Yd = to_dev(np.full((A.n, ld), np.nan))
    api.spmm(ctx, M, to_dev(X), Yd, w)
    Y = Yd.cpu().numpy()
    ref = OS._apply(A.to_scipy(), X[:, :w])
    assert np.all(Y[np.diff(A.rowptr) == 0, :w] == 0.0)
    bound = 1e-15 * 16 * (abs(A.to_scipy()) @ np.abs(X[:, :w]))
    assert np.all(np.abs(Y[:, :w] - ref) <= bound + 1e-300)
    if ld > w:
        assert np.all(np.isnan(Y[:, w:]))  # padding column untouched


@pytest.mark.parametrize("w", [1, 5, 48, 69, 130])
def test_spmm_power_law_rows(ctx, w):
    """Normalized Laplacian of a Chung-Lu graph: rows from a few to hundreds of
    nonzeros, the long ones computed one workgroup per row."""
    from paper_2409_05572_amd import api

    A = W.chung_lu_laplacian(20000, 16.0, 2.5, 11)
    deg = np.diff(A.rowptr)
    assert deg.max() > 64 and (deg > 64).sum() >= 50  # both row kernels take part
    M = api.Matrix.from_csr(ctx, A)
    ld = w + (w % 2)
    X = _row_major(A.n, w, ld, w + 1)
    Yd = to_dev(np.full((A.n, ld), np.nan))
    api.spmm(ctx, M, to_dev(X), Yd, w)
    Y = Yd.cpu().numpy()
    ref = OS._apply(A.to_scipy(), X[:, :w])
    bound = 1e-15 * (deg.max() + 2) * (abs(A.to_scipy()) @ np.abs(X[:, :w]))
    assert np.all(np.abs(Y[:, :w] - ref) <= bound + 1e-300)


def test_spmm_full_config2_sampled_rows(ctx):
    """3-D 128^3 Laplacian, 96 columns: the launch the solver uses, checked on
    2000 sampled rows against the oracle's sparse product."""
    import torch
    from paper_2409_05572_amd import api

    A = W.laplacian_3d(128)
    M = api.Matrix.from_csr(ctx, A)
    g = torch.Generator(device="cuda").manual_seed(5)
    Xd = torch.randn((A.n, 96), generator=g, device="cuda", dtype=torch.float64)
    Yd = torch.empty_like(Xd)
    api.spmm(ctx, M, Xd, Yd, 96)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.integers(0, A.n, 1995), [0, 1, A.n - 1, 16383, 16384]]))
    S = A.to_scipy()[rows]
    cols = np.unique(S.indices)
    Xs = Xd[torch.from_numpy(cols).cuda()].cpu().numpy()
    ref = OS._apply(S[:, cols], Xs)
    got = Yd[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * 12 * np.abs(Xs).max())


@pytest.mark.parametrize("n,mu,mv", [(1, 1, 1), (1000, 1, 1), (4097, 17, 33), (20000, 96, 96),
                                     (50001, 288, 96), (3001, 250, 250), (777, 300, 7)])
def test_gram_matches_definition(ctx, n, mu, mv):
    from paper_2409_05572_amd import api

    U = _row_major(n, mu, mu + mu % 2, 1)
    V = _row_major(n, mv, mv + mv % 2 + 2, 2)
    Cd = to_dev(np.full((mu, mv), np.nan))
    api.gram(ctx, to_dev(U), mu, to_dev(V), mv, Cd)
    C = Cd.cpu().numpy()
    ref = U[:, :mu].T @ V[:, :mv]
    bound = 4 * n * 1.2e-16 * (np.abs(U[:, :mu]).T @ np.abs(V[:, :mv]))
    assert np.all(np.abs(C - ref) <= bound + 1e-300)


@pytest.mark.parametrize("n,m", [(1, 1), (1000, 17), (4097, 69), (20000, 96), (20001, 97), (7777, 150),
                                 (50001, 288), (3001, 300)])
def test_symmetric_gram_matches_definition(ctx, n, m):
    """U^T U through the symmetric path (triangular diagonal tiles, mirrored
    blocks): within the summation bound and exactly symmetric."""
    from paper_2409_05572_amd import api

    U = _row_major(n, m, m + m % 2, 3)
    Ud = to_dev(U)
    Cd = to_dev(np.full((m, m), np.nan))
    api.gram(ctx, Ud, m, Ud, m, Cd)
    C = Cd.cpu().numpy()
    ref = U[:, :m].T @ U[:, :m]
    bound = 4 * n * 1.2e-16 * (np.abs(U[:, :m]).T @ np.abs(U[:, :m]))
    assert np.all(np.abs(C - ref) <= bound + 1e-300)
    assert np.array_equal(C, C.T)


def test_gram_is_deterministic(ctx):
    from paper_2409_05572_amd import api

    U = to_dev(_row_major(100003, 96, 96, 4))
    outs = []
    for _ in range(2):
        Cd = to_dev(np.zeros((96, 96)))
        api.gram(ctx, U, 96, U, 96, Cd)
        outs.append(Cd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("n,K,N,beta", [(1, 1, 1, 0.0), (1000, 1, 1, 1.0), (4097, 37, 69, 0.0),
                                        (20000, 288, 192, 0.0), (5003, 250, 250, 1.0),
                                        (64, 96, 97, 1.0), (70001, 96, 96, 1.0), (65601, 250, 69, 0.0),
                                        (66000, 5, 3, 1.0), (65536, 288, 128, 0.0),
                                        # tall panels, ragged last row block
                                        (600001, 96, 96, 1.0), (300001, 250, 69, 0.0),
                                        (600001, 5, 3, 1.0), (300007, 288, 192, 0.0)])
def test_update_matches_definition(ctx, n, K, N, beta):
    from paper_2409_05572_amd import api

    rng = np.random.default_rng(K + N)
    U = _row_major(n, K, K + K % 2, 5)
    Cm = rng.standard_normal((K, N))
    O0 = _row_major(n, N, N + N % 2, 6)
    Od = to_dev(O0)
    api.update(ctx, to_dev(U), K, to_dev(Cm), N, Od, beta)
    got = Od.cpu().numpy()[:, :N]
    ref = beta * O0[:, :N] + U[:, :K] @ Cm
    bound = 4 * (K + 1) * 1.2e-16 * (beta * np.abs(O0[:, :N]) + np.abs(U[:, :K]) @ np.abs(Cm))
    assert np.all(np.abs(got - ref) <= bound + 1e-300)


@pytest.mark.parametrize("K,N,beta", [(96, 96, 1.0), (288, 192, 0.0), (37, 5, 1.0), (250, 69, 1.0)])
def test_update_rows_do_not_depend_on_the_row_range(ctx, K, N, beta):
    """A tall update and the same rows updated on their own (other row-block
    boundaries, other grid) agree bitwise: every output has one fixed
    summation order."""
    import torch

    from paper_2409_05572_amd import api

    n, h = 600001, 5000
    g = torch.Generator(device="cuda").manual_seed(K * 7 + N)
    ldu, ldo = K + 3 + (K + 3) % 2, N + 1 + (N + 1) % 2  # even leading dimensions, padded
    U = torch.randn((n, ldu), dtype=torch.float64, device="cuda", generator=g)
    Cm = torch.randn((K, N), dtype=torch.float64, device="cuda", generator=g)
    O0 = torch.randn((n, ldo), dtype=torch.float64, device="cuda", generator=g)
    full = O0.clone()
    api.update(ctx, U, K, Cm, N, full, beta)
    for sl in (slice(0, h), slice(n - h, n), slice(123456, 123456 + 77)):
        part = O0[sl].clone()
        api.update(ctx, U[sl], K, Cm, N, part, beta)
        assert torch.equal(part[:, :N], full[sl][:, :N])
    assert torch.equal(full[:, N:], O0[:, N:])  # padding columns untouched


def _sym_with_spectrum(m, seed, clustered):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    if clustered:
        lam = np.sort(np.concatenate([np.full(m // 3, 0.01), np.full(m // 4, 0.0100000001),
                                      rng.uniform(-3, 12, m - m // 3 - m // 4)]))
    else:
        lam = np.sort(rng.uniform(-5, 12, m))
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("m", [1, 2, 3, 16, 48, 63, 64, 65, 97, 113, 130, 192, 207, 224, 225, 288, 750])
@pytest.mark.parametrize("clustered", [False, True])
def test_syev_matches_definition(ctx, m, clustered):
    from paper_2409_05572_amd import api

    A = _sym_with_spectrum(m, m, clustered)
    Ad = to_dev(A.copy())
    wd = to_dev(np.zeros(m))
    Zd = to_dev(np.zeros((m, m)))
    api.syev(ctx, Ad, wd, Zd)
    w = wd.cpu().numpy()
    Z = Zd.cpu().numpy()
    nrm = np.linalg.norm(A, 2)
    ref = np.linalg.eigvalsh(A)
    assert np.all(np.diff(w) >= 0)
    assert np.max(np.abs(w - ref)) <= 1e-13 * max(nrm, 1.0) * 8
    R = A @ Z - Z * w
    # Eigenvectors of a cluster of width delta (here 1e-10: 0.01 and
    # 0.0100000001) are fixed only up to mixing inside it, which costs up to
    # delta in the residual; every other column must be accurate to rounding.
    inc = (w > 0.0099) & (w < 0.0101) if clustered else np.zeros(m, dtype=bool)
    assert np.linalg.norm(R[:, ~inc], 2) <= 8e-12 * max(nrm, 1.0)
    if inc.any():
        assert np.linalg.norm(R[:, inc], 2) <= 2e-10 + 8e-12 * max(nrm, 1.0)
    assert np.abs(Z.T @ Z - np.eye(m)).max() <= 1e-12


def _degenerate(g, seed, extra=0):
    """Q diag(lam) Q^T with lam the spectrum of the g^3 Dirichlet Laplacian
    (eigenvalue multiplicities 1, 3 and 6, exactly) plus `extra` random ones."""
    rng = np.random.default_rng(seed)
    one = 2.0 - 2.0 * np.cos(np.arange(1, g + 1) * np.pi / (g + 1))
    lam = (one[:, None, None] + one[None, :, None] + one[None, None, :]).ravel()
    lam = np.sort(np.concatenate([lam, rng.uniform(0, 12, extra)]))
    m = lam.size
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), lam


@pytest.mark.parametrize("g,extra,k", [(4, 19, 69), (4, 0, 64), (5, 0, 125), (5, 100, 96),
                                       (6, 0, 69), (6, 72, 192)])
def test_syev_lowest_degenerate_clusters(ctx, g, extra, k):
    """Exactly repeated eigenvalues (the projected matrix of a converged
    Laplacian block has them): the k lowest pairs must still come out with
    orthonormal vectors."""
    from paper_2409_05572_amd import api

    A, lam = _degenerate(g, 100 * g + extra, extra)
    m = A.shape[0]
    Ad = to_dev(A.copy())
    wd = to_dev(np.zeros(k))
    Zd = to_dev(np.zeros((m, k)))
    api.syev_lowest(ctx, Ad, k, wd, Zd)
    w = wd.cpu().numpy()
    Z = Zd.cpu().numpy()
    nrm = np.abs(lam).max()
    assert np.max(np.abs(w - lam[:k])) <= 8e-13 * nrm
    assert np.linalg.norm(A @ Z - Z * w, 2) <= 8e-12 * nrm
    assert np.abs(Z.T @ Z - np.eye(k)).max() <= 1e-12


@pytest.mark.parametrize("w", [24, 130, 250, 500, 896])
def test_cholqr_orthonormalizes_and_drops_dependent_columns(ctx, w):
    """Widths up to 112 take the in-LDS blocked transform, wider ones (up to
    896) the blocked transform in global memory; both drop the dependent
    columns."""
    from paper_2409_05572_amd import api

    rng = np.random.default_rng(11)
    n = 20001
    U, _ = np.linalg.qr(rng.standard_normal((n, w)))
    Vt, _ = np.linalg.qr(rng.standard_normal((w, w)))
    Wm = U @ np.diag(np.logspace(0, -5, w)) @ Vt
    Wm[:, 10] = 2 * Wm[:, 3] - Wm[:, 4]  # exactly dependent columns
    dep = 1
    if w > 112:
        Wm[:, w - 3] = Wm[:, 0] + 0.5 * Wm[:, w - 10]
        dep = 2
    Wd = to_dev(Wm)
    r = api.cholqr(ctx, Wd, w)
    Q = Wd.cpu().numpy()[:, :r]
    assert r == w - dep
    assert np.abs(Q.T @ Q - np.eye(r)).max() <= 1e-13
    assert np.linalg.norm(Wm - Q @ (Q.T @ Wm)) <= 1e-9 * np.linalg.norm(Wm)
