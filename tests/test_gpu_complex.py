"""Complex Hermitian A on the GPU (the paper's problem statement allows A in
C^{n x n}, Section 1): the complex CSR product, the complex Gram and update
(matrix-core kernels on the interleaved real views), the Hermitian small
eigensolve, and whole LOBPCG / SI solves with shrink-and-expand against the
closed-form spectrum of the magnetic torus Laplacian and the FP64 oracle.

Error bounds of the building blocks follow from FP64 arithmetic: a product
summing K terms is within about K u sum |a||b| of the exact one.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cluster_angles, gpu_ctx

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
PH2 = (0.3, 0.7)
PH3 = (0.3, 0.7, 1.1)


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _cdev(a, ld=None):
    """complex128 device block with leading dimension ld (padding garbage)."""
    import torch

    n, w = a.shape
    ld = ld or (w + 1) // 2 * 2
    full = np.full((n, ld), 5.0e3 - 7.0e3j)
    full[:, :w] = a
    return torch.from_numpy(full).cuda()


def _crand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("w", [1, 3, 16, 48, 64, 65, 130])
@pytest.mark.parametrize("kind", ["magnetic", "random"])
def test_spmm_z_matches_the_product(ctx, w, kind):
    from paper_2409_05572_amd import api

    A = W.magnetic_laplacian(12, PH3) if kind == "magnetic" else W.random_sparse_hermitian(3001, 0.003, 5)
    S = A.to_scipy()
    M = api.Matrix.from_csr(ctx, A)
    X = _crand((A.n, w), w)
    Xd = _cdev(X)
    Yd = _cdev(np.zeros((A.n, w)))
    api.spmm_z(ctx, M, Xd, Yd, w)
    got = Yd.cpu().numpy()[:, :w]
    ref = S @ X
    nz = int(np.diff(A.rowptr).max())
    bound = 4 * (nz + 2) * U * (abs(S) @ abs(X)) + 1e-300
    assert np.all(np.abs(got - ref) <= bound)
    pad = Yd.cpu().numpy()[:, w:]
    assert np.all(pad == 5.0e3 - 7.0e3j)  # padding columns untouched


@pytest.mark.parametrize("n,mu,mv", [(1, 1, 1), (1000, 5, 7), (50001, 96, 48), (20000, 144, 144), (3000, 300, 20)])
def test_gram_z_is_the_conjugate_product(ctx, n, mu, mv):
    import torch

    from paper_2409_05572_amd import api

    Uh = _crand((n, mu), 1)
    Vh = _crand((n, mv), 2)
    Ud, Vd = _cdev(Uh), _cdev(Vh)
    out = torch.zeros((mu, mv), dtype=torch.complex128, device="cuda")
    api.gram_z(ctx, Ud, mu, Vd, mv, out)
    got = out.cpu().numpy()
    ref = Uh.conj().T @ Vh
    bound = 4 * (n + 4) * U * (abs(Uh).T @ abs(Vh))
    assert np.all(np.abs(got - ref) <= bound)
    if mu == mv:  # U^H U is exactly Hermitian
        out2 = torch.zeros((mu, mu), dtype=torch.complex128, device="cuda")
        api.gram_z(ctx, Ud, mu, Ud, mu, out2)
        g = out2.cpu().numpy()
        assert np.array_equal(g, g.conj().T)
        assert np.all(np.abs(g - Uh.conj().T @ Uh) <= 4 * (n + 4) * U * (abs(Uh).T @ abs(Uh)))


@pytest.mark.parametrize("n,K,N", [(1, 1, 1), (1000, 7, 3), (50001, 144, 48), (3000, 300, 200)])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_update_z_is_the_product(ctx, n, K, N, beta):
    import torch

    from paper_2409_05572_amd import api

    Uh = _crand((n, K), 3)
    Ch = _crand((K, N), 4)
    O0 = _crand((n, N), 5)
    Ud = _cdev(Uh)
    Od = _cdev(O0)
    Cd = torch.from_numpy(np.ascontiguousarray(Ch)).cuda()
    api.update_z(ctx, Ud, K, Cd, N, Od, beta=beta)
    got = Od.cpu().numpy()[:, :N]
    ref = beta * O0 + Uh @ Ch
    bound = 4 * (K + 4) * U * (abs(Uh) @ abs(Ch) + beta * abs(O0))
    assert np.all(np.abs(got - ref) <= bound)


def _herm(m, seed, spectrum=None):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    lam = rng.standard_normal(m) if spectrum is None else spectrum
    A = (Q * lam[None, :]) @ Q.conj().T
    return 0.5 * (A + A.conj().T)


@pytest.mark.parametrize("m,k", [(1, 1), (2, 2), (3, 1), (17, 9), (80, 80), (81, 40), (200, 64), (300, 300),
                                 (512, 96)])
def test_heev_lowest_z(ctx, m, k):
    import torch

    from paper_2409_05572_amd import api

    A = _herm(m, m)
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    w = torch.zeros(k, dtype=torch.float64, device="cuda")
    Z = torch.zeros((m, k), dtype=torch.complex128, device="cuda")
    api.heev_lowest_z(ctx, Ad, k, w, Z)
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    ref = np.linalg.eigvalsh(A)[:k]
    nrm = np.abs(np.linalg.eigvalsh(A)).max()
    assert np.max(np.abs(w - ref)) <= 1e-13 * nrm * max(1.0, m / 64)
    assert np.abs(Z.conj().T @ Z - np.eye(k)).max() <= 1e-13
    assert np.abs(A @ Z - Z * w[None, :]).max() <= 1e-12 * nrm


def test_heev_lowest_z_degenerate_clusters(ctx):
    """Exactly repeated eigenvalues (multiplicity 1 to 6): the vectors of each
    cluster stay orthonormal and span its eigenspace."""
    import torch

    from paper_2409_05572_amd import api

    m, k = 120, 60
    spec = np.sort(np.repeat(np.linspace(-2.0, 3.0, 40), ([1, 2, 3, 4, 5, 6] * 7)[:40])[:m])
    assert spec.size == m
    A = _herm(m, 9, spec)
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    w = torch.zeros(k, dtype=torch.float64, device="cuda")
    Z = torch.zeros((m, k), dtype=torch.complex128, device="cuda")
    api.heev_lowest_z(ctx, Ad, k, w, Z)
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    assert np.max(np.abs(w - spec[:k])) <= 1e-13 * 3.0
    assert np.abs(Z.conj().T @ Z - np.eye(k)).max() <= 1e-12
    assert np.abs(A @ Z - Z * w[None, :]).max() <= 1e-12 * 3.0


def _check(A, lam, V, exact, ref=None):
    assert np.iscomplexobj(V)
    assert np.max(np.abs(lam - exact) / np.abs(exact)) <= 1e-10
    S = A.to_scipy()
    R = S @ V - V * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))) <= 1e-8 * 1.0001
    assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() <= 1e-12
    if ref is not None:
        assert np.max(np.abs(lam - ref.lam) / np.abs(ref.lam)) <= 1e-10
        assert cluster_angles(lam, V, ref.V) <= 1e-6


@pytest.mark.parametrize("strategy", ["none", "fix", "slopek"])
def test_lobpcg_hermitian_2d(ctx, strategy):
    from paper_2409_05572_amd import api

    m, n_ev, nb = 32, 8, 16
    A = W.magnetic_laplacian(m, PH2)
    X0 = W.gaussian_block_complex(A.n, nb, 11)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve_z(ctx, M, X0, n_ev, nb - n_ev, strategy=strategy, history_cap=2000, r_warm=1e-2)
    ref = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 5, se=O.SEParams(strategy, r_warm=1e-2))
    assert info.converged and ref.converged
    _check(A, lam, V, W.magnetic_spectrum(m, PH2)[:n_ev], ref)
    assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // 10)
    if strategy != "none":
        assert info.n_shrinks >= 1


def test_lobpcg_hermitian_3d_with_expansions(ctx):
    from paper_2409_05572_amd import api

    m, n_ev, nb = 16, 16, 24
    A = W.magnetic_laplacian(m, PH3)
    X0 = W.gaussian_block_complex(A.n, nb, 12)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve_z(ctx, M, X0, n_ev, nb - n_ev, strategy="fix", r_warm=1e-2, history_cap=2000)
    ref = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 5, se=O.SEParams("fix", r_warm=1e-2))
    assert info.converged and info.n_shrinks >= 1 and info.n_expands >= 1
    _check(A, lam, V, W.magnetic_spectrum(m, PH3)[:n_ev], ref)
    flags = info.history[:, 7].astype(int)
    shr_gpu = info.history[(flags & 2) != 0, 0].astype(int)
    shr_ref = np.array([h["j"] for h in ref.history if h["shrink"]])
    k = min(len(shr_gpu), len(shr_ref), 3)
    assert k >= 1 and np.array_equal(shr_gpu[:k], shr_ref[:k])


@pytest.mark.parametrize("strategy", ["none", "fix"])
def test_si_hermitian(ctx, strategy):
    from paper_2409_05572_amd import api

    m, n_ev, nb = 12, 4, 8
    A = W.magnetic_laplacian(m, PH2)
    X0 = W.gaussian_block_complex(A.n, nb, 13)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve_z(ctx, M, X0, n_ev, nb - n_ev, solver="si", strategy=strategy, n_es=n_ev + 2,
                               history_cap=20000)
    ref = O.subspace_iteration(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2, se=O.SEParams(strategy),
                               max_iter=20000)
    assert info.converged and ref.converged
    _check(A, lam, V, W.magnetic_spectrum(m, PH2)[:n_ev], ref)
    r_gpu = info.history[:, 1]
    r_ref = np.array([h["r"] for h in ref.history])
    L = min(len(r_gpu), len(r_ref))
    big = r_ref[:L] > 1e-6
    assert big.sum() >= 10
    np.testing.assert_allclose(r_gpu[:L][big], r_ref[:L][big], rtol=1e-5)


def test_hermitian_random_matrix_and_seeded_start(ctx):
    """A random sparse Hermitian matrix (no closed form: brute force) from the
    library's seeded real start block, and device pointers."""
    import torch

    from paper_2409_05572_amd import api

    A = W.random_sparse_hermitian(400, 0.02, 21)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve_z(ctx, M, None, 6, 6, seed=77, strategy="fix", r_warm=1e-2, max_iter=2000)
    assert info.converged
    exact = np.linalg.eigvalsh(A.to_scipy().toarray())[:6]
    assert np.max(np.abs(lam - exact)) <= 1e-10 * A.anorm
    X0 = W.gaussian_block_complex(A.n, 12, 22)
    Xd = torch.from_numpy(np.ascontiguousarray(X0.T)).cuda()
    lam2, V2, info2 = api.solve_z(ctx, M, Xd, 6, 6, max_iter=2000)
    assert info2.converged
    assert np.max(np.abs(lam2.cpu().numpy() - exact)) <= 1e-10 * A.anorm
    V2 = V2.cpu().numpy().T
    R = A.to_scipy() @ V2 - V2 * lam2.cpu().numpy()[None, :]
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-8 * A.anorm * 1.0001


def test_larger_3d_magnetic_lobpcg(ctx):
    """n = 110,592 (48^3 torus), 32 wanted + 16 extra, fix: every eigenvalue
    against the closed form, all residuals on the host, orthonormality."""
    from paper_2409_05572_amd import api

    m, n_ev, nb = 48, 32, 48
    A = W.magnetic_laplacian(m, PH3)
    X0 = W.gaussian_block_complex(A.n, nb, 14)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve_z(ctx, M, X0, n_ev, nb - n_ev, strategy="fix")
    assert info.converged and info.n_shrinks >= 1
    _check(A, lam, V, W.magnetic_spectrum(m, PH3)[:n_ev])


def test_complex_entry_points_reject_what_they_do_not_support(ctx):
    from paper_2409_05572_amd import api
    from paper_2409_05572_amd._lib import SeError

    A = W.magnetic_laplacian(8, PH2)
    M = api.Matrix.from_csr(ctx, A)
    X0 = W.gaussian_block_complex(A.n, 8, 1)
    for kw in (dict(precision="fp32"), dict(solver="sd"), dict(solver="tracemin"), dict(precond="jacobi"),
               dict(expand_vectors="random")):
        with pytest.raises(SeError):
            api.solve_z(ctx, M, X0, 4, 4, **kw)
    import ctypes as C

    from paper_2409_05572_amd import _lib

    Ar = W.laplacian_2d(8)
    Mr = api.Matrix.from_csr(ctx, Ar)
    p = api.params(4, 4)
    V = np.zeros((Ar.n, 4), dtype=np.complex128, order="F")
    lam = np.zeros(4)
    X0f = np.asfortranarray(X0)
    st = _lib.lib().se_solve_z(ctx.handle, Mr.handle, C.byref(p), C.c_void_p(X0f.ctypes.data),
                               C.c_void_p(V.ctypes.data), C.c_void_p(lam.ctypes.data), None)
    assert st == _lib.SE_ERR_INVALID_ARG  # a real matrix is not taken by the complex solver ...
    with pytest.raises(SeError):  # ... nor a complex one by the real solver
        api.solve(ctx, M, np.asfortranarray(X0.real), 4, 4)
