"""Pins of the oracle on complex Hermitian matrices (CPU).

The paper states the eigenproblem for Hermitian A in C^{n x n} (Section 1)
and writes X^H throughout its algorithms. Pins: the closed-form spectrum of
the magnetic torus Laplacian (a periodic grid with a uniform phase per step,
whose eigenvalues are sums of 2 - 2 cos(2 pi k / m + phi)), brute force on
random sparse Hermitian matrices, orthonormality in the complex inner
product, monotone Ritz values, and planted mistakes (a plain transpose where
the conjugate transpose belongs) that must fail them.
"""
import numpy as np
import pytest

import oracle as O
import oracle.solvers as OS
import workloads as W

PH2 = (0.3, 0.7)
PH3 = (0.3, 0.7, 1.1)


def _check(A, res, exact, tol=1e-8, lam_rtol=1e-10):
    assert res.converged
    assert np.iscomplexobj(res.V)
    assert np.max(np.abs(res.lam - exact) / np.abs(exact)) <= lam_rtol
    S = A.to_scipy()
    R = S @ res.V - res.V * res.lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(res.V, axis=0))) <= tol
    V = res.V
    assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() <= 1e-12


def test_magnetic_spectrum_is_the_closed_form():
    A = W.magnetic_laplacian(10, PH2)
    S = A.to_scipy().toarray()
    assert np.abs(S - S.conj().T).max() == 0.0 and np.abs(S.imag).max() > 0.1
    ev = np.linalg.eigvalsh(S)
    np.testing.assert_allclose(ev, W.magnetic_spectrum(10, PH2), atol=1e-13)
    # plane wave v_j = exp(i theta j) in the fastest direction: eigenvector
    m = 10
    th = 2 * np.pi * 3 / m
    ring = W._magnetic_ring(m, 0.3).toarray()
    v = np.exp(1j * th * np.arange(m))
    np.testing.assert_allclose(ring @ v, (2 - 2 * np.cos(th + 0.3)) * v, atol=1e-13)


@pytest.mark.parametrize("strategy", ["none", "fix", "slopek"])
def test_lobpcg_hermitian_reaches_closed_form(strategy):
    m, n_ev, nb = 16, 8, 12
    A = W.magnetic_laplacian(m, PH2)
    X0 = W.gaussian_block_complex(A.n, nb, 5)
    res = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2, se=O.SEParams(strategy, r_warm=1e-2))
    _check(A, res, W.magnetic_spectrum(m, PH2)[:n_ev])
    if strategy != "none":
        assert res.n_shrinks >= 1
    thetas = [h["theta"] for h in res.history if "theta" in h]
    for a, b in zip(thetas, thetas[1:]):  # Ritz values never increase (LOBPCG)
        assert np.all(b <= a + 1e-12 * np.abs(a))


def test_lobpcg_hermitian_3d_with_expansion():
    m, n_ev, nb = 8, 16, 24
    A = W.magnetic_laplacian(m, PH3)
    X0 = W.gaussian_block_complex(A.n, nb, 6)
    res = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 5, se=O.SEParams("fix", r_warm=1e-2))
    _check(A, res, W.magnetic_spectrum(m, PH3)[:n_ev])
    assert res.n_shrinks >= 1 and res.n_expands >= 1


@pytest.mark.parametrize("strategy", ["none", "fix"])
def test_subspace_iteration_hermitian_reaches_closed_form(strategy):
    m, n_ev, nb = 8, 4, 8
    A = W.magnetic_laplacian(m, PH2)
    X0 = W.gaussian_block_complex(A.n, nb, 7)
    res = O.subspace_iteration(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                               se=O.SEParams(strategy), max_iter=20000)
    _check(A, res, W.magnetic_spectrum(m, PH2)[:n_ev])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_lobpcg_hermitian_brute_force(seed):
    n, n_ev, nb = 150, 6, 10
    A = W.random_sparse_hermitian(n, 0.05, seed)
    X0 = W.gaussian_block_complex(n, nb, seed)
    res = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, max_iter=2000)
    ev = np.linalg.eigvalsh(A.to_scipy().toarray())[:n_ev]
    assert res.converged
    assert np.max(np.abs(res.lam - ev)) <= 1e-9 * A.anorm


def test_real_start_block_on_a_hermitian_matrix():
    A = W.magnetic_laplacian(12, PH2)
    X0 = W.gaussian_block(A.n, 10, 3)  # real block: complex arithmetic starts at A X
    res = O.lobpcg(A.to_scipy(), X0, 6, A.anorm, tol=1e-8)
    _check(A, res, W.magnetic_spectrum(12, PH2)[:6])


def test_plain_transpose_in_rayleigh_ritz_is_caught(monkeypatch):
    """Planted mistake: A_p = S^T (A S) instead of S^H (A S)."""
    def bad_rr(S, AS):
        Ap = S.T @ AS
        Ap = 0.5 * (Ap + Ap.conj().T)
        return np.linalg.eigh(Ap)

    monkeypatch.setattr(OS, "rayleigh_ritz", bad_rr)
    A = W.magnetic_laplacian(12, PH2)
    X0 = W.gaussian_block_complex(A.n, 10, 3)
    res = O.lobpcg(A.to_scipy(), X0, 6, A.anorm, tol=1e-8, max_iter=100)
    ex = W.magnetic_spectrum(12, PH2)[:6]
    assert not res.converged or np.max(np.abs(res.lam - ex) / ex) > 1e-6


def test_plain_transpose_in_projection_is_caught(monkeypatch):
    """Planted mistake: the orthogonalization projects with X^T."""
    monkeypatch.setattr(OS, "_H", lambda M: M.T)
    A = W.magnetic_laplacian(12, PH2)
    X0 = W.gaussian_block_complex(A.n, 10, 3)
    res = O.lobpcg(A.to_scipy(), X0, 6, A.anorm, tol=1e-8, max_iter=100)
    ex = W.magnetic_spectrum(12, PH2)[:6]
    bad = (not res.converged) or np.max(np.abs(res.lam - ex) / ex) > 1e-6
    V = res.V
    bad = bad or np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() > 1e-8
    assert bad
