"""Plausible mistakes planted in the oracle (on the CPU) must fail a pin.

Each case monkeypatches one oracle function with a wrong variant and checks
that the independent facts of ``tests/_pins.py`` (or the scripted strategy
sequences) no longer hold.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.solvers as OS
import oracle.strategy as OST
import workloads as W
from tests import _pins as pins


def _solve_small(strategy="none", max_iter=300):
    m, n_ev = 10, 8
    A = W.laplacian_3d(m)
    X0 = W.gaussian_block(A.n, 12, 4)
    res = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                   se=O.SEParams(strategy, r_warm=1e-2), max_iter=max_iter)
    fails = pins.eigen_failures(res.lam, res.V, A.to_scipy(), A.anorm,
                                pins.laplacian_spectrum(m, 3, n_ev), 1e-8, 1e-9)
    thetas = [h["theta"] for h in res.history if "theta" in h]
    for a, b in zip(thetas, thetas[1:]):
        if np.any(b > a + 1e-12 * np.abs(a)):
            fails.append("Ritz value increased")
            break
    if not res.converged:
        fails.append("not converged")
    return fails


def test_unmutated_oracle_passes():
    assert _solve_small() == []
    assert _solve_small("fix") == []


def test_residual_sign_error_is_caught(monkeypatch):
    orig = OS.residual_measures

    def bad(A, X, lam, anorm):
        R, stop, paper = orig(A, X, -lam, anorm)
        return R, stop, paper

    monkeypatch.setattr(OS, "residual_measures", bad)
    assert _solve_small(max_iter=100) != []


def test_descending_ritz_order_is_caught(monkeypatch):
    orig = OS.rayleigh_ritz

    def bad(S, AS):
        theta, Z = orig(S, AS)
        return theta[::-1].copy(), Z[:, ::-1].copy()

    monkeypatch.setattr(OS, "rayleigh_ritz", bad)
    assert _solve_small(max_iter=60) != []


def test_wrong_block_in_hl_basis_is_caught(monkeypatch):
    def bad(Z, k, active, drop_tol=1e-12):
        Z1 = Z[:, :k]
        B = Z1[np.asarray(active), :].T  # used Z1 instead of Z2
        QB, _ = OS.orth(B, drop_tol)
        return Z1, Z1 @ QB

    monkeypatch.setattr(OS, "hl_basis", bad)
    assert _solve_small(max_iter=100) != []


def test_shrink_keeping_wrong_columns_is_caught(monkeypatch):
    orig = OS.hl_basis

    def reverse_then(Z, k, active, drop_tol=1e-12):
        Z1, CP = orig(Z, k, active, drop_tol)
        return Z1[:, ::-1].copy(), CP  # X columns no longer ascending

    monkeypatch.setattr(OS, "hl_basis", reverse_then)
    assert _solve_small("fix", max_iter=100) != []


def test_single_pass_gram_schmidt_is_caught(monkeypatch):
    """Orthogonalizing with one classical Gram-Schmidt pass (no second pass, no
    Householder) loses orthogonality on an ill-conditioned block; the
    orthonormality pin detects it."""
    def bad_orth(Y, drop_tol=1e-12):
        basis = []
        for i in range(Y.shape[1]):
            v = Y[:, i].copy()
            if basis:
                B = np.stack(basis, 1)
                v -= B @ (B.T @ v)
            basis.append(v / np.linalg.norm(v))
        return np.stack(basis, 1), np.arange(Y.shape[1])

    rng = np.random.default_rng(0)
    U, _ = np.linalg.qr(rng.standard_normal((400, 10)))
    V, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    Y = U @ np.diag(np.logspace(0, -10, 10)) @ V.T
    good, _ = O.orth(Y)
    assert np.abs(good.T @ good - np.eye(10)).max() < 1e-12
    monkeypatch.setattr(O, "orth", bad_orth)
    bad, _ = O.orth(Y)
    assert np.abs(bad.T @ bad - np.eye(10)).max() > 1e-12


def test_slope_sign_error_is_caught(monkeypatch):
    def bad_slope(self, j):
        if j - 1 not in self.log_r or j not in self.log_r:
            return None
        return self.log_r[j] - self.log_r[j - 1]

    monkeypatch.setattr(OST.SEController, "slope", bad_slope)
    rs, lr = [], 0.0
    for j in range(1, 31):
        lr -= 1.0 if j <= 12 else 0.5
        rs.append(10.0 ** lr)
    ctl = O.SEController(O.SEParams("slope"))
    exp = []
    for j, r in enumerate(rs, start=1):
        ctl.observe(j, r)
        if ctl.ifexpand(j):
            ctl.did_expand(j)
            exp.append(j)
        if ctl.ifshrink(j):
            ctl.did_shrink(j)
    assert exp != [13]


# --- Chebyshev filter, TraceMIN's inner CG, Jacobi preconditioner -------------------------

def _cheb_pin_failures(filt):
    """The diagonal closed form of T_d (as in the oracle pins) against `filt`."""
    import scipy.sparse as sp

    rng = np.random.default_rng(5)
    a = np.sort(rng.uniform(0.0, 8.0, 40))
    A = sp.diags(a).tocsr()
    Y = rng.standard_normal((40, 3))
    lower, cut, upper, d = a[0], a[8], 8.0, 5
    c, e = 0.5 * (upper + cut), 0.5 * (upper - cut)

    def T(x):
        x = np.asarray(x, dtype=np.float64)
        return np.where(np.abs(x) <= 1, np.cos(d * np.arccos(np.clip(x, -1, 1))),
                        np.sign(x) ** d * np.cosh(d * np.arccosh(np.maximum(np.abs(x), 1))))

    rho = T((a - c) / e) / T((lower - c) / e)
    return not np.allclose(filt(A, Y, d, lower, cut, upper), rho[:, None] * Y, rtol=1e-10, atol=1e-12)


def test_unmutated_chebyshev_filter_passes():
    assert not _cheb_pin_failures(O.chebyshev_filter)


@pytest.mark.parametrize("mistake", ["centre", "normalization", "recurrence_sign"])
def test_chebyshev_filter_mistakes_are_caught(mistake):
    def bad(A, Y, degree, lower, cut, upper):
        c = 0.5 * (upper + cut) if mistake != "centre" else 0.5 * (upper - cut)
        e = 0.5 * (upper - cut)
        L = lambda Z: (A @ Z - c * Z) / e  # noqa: E731
        l0 = (lower - c) / e
        T_prev, T_ = Y, L(Y)
        t_prev, t = 1.0, l0
        sgn = -1.0 if mistake == "recurrence_sign" else 1.0
        for _ in range(2, degree + 1):
            T_prev, T_ = T_, 2.0 * L(T_) - sgn * T_prev
            t_prev, t = t, 2.0 * l0 * t - sgn * t_prev
        return T_ if mistake == "normalization" else T_ / t

    assert _cheb_pin_failures(bad)


def _projected_cg_pin_failures(cg):
    import scipy.sparse as sp

    rng = np.random.default_rng(3)
    n = 30
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    X, _ = np.linalg.qr(rng.standard_normal((n, 3)))
    B = rng.standard_normal((n, 4))
    D = cg(sp.csr_matrix(A), X, B, n)
    Qf, _ = np.linalg.qr(np.hstack([X, rng.standard_normal((n, n - 3))]))
    Q = Qf[:, 3:]
    ref = Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ B)
    return not (np.allclose(D, ref, rtol=1e-8, atol=1e-10) and np.abs(X.T @ D).max() < 1e-10)


def test_unmutated_projected_cg_passes():
    assert not _projected_cg_pin_failures(O.projected_cg)


@pytest.mark.parametrize("mistake", ["no_projection", "no_conjugation"])
def test_projected_cg_mistakes_are_caught(mistake):
    def bad(A, X, B, steps):
        P = lambda Z: Z - X @ (X.T @ Z)  # noqa: E731
        r = P(B)
        d = r.copy()
        D = np.zeros_like(B)
        rr = np.einsum("ij,ij->j", r, r)
        for _ in range(steps):
            q = A @ d if mistake == "no_projection" else P(A @ d)
            dq = np.einsum("ij,ij->j", d, q)
            alpha = np.where(dq > 0, rr / np.where(dq > 0, dq, 1.0), 0.0)
            D = D + d * alpha
            r = r - q * alpha
            rr_new = np.einsum("ij,ij->j", r, r)
            beta = 0.0 if mistake == "no_conjugation" else rr_new / np.where(rr > 0, rr, 1.0)
            d = r + d * beta
            rr = rr_new
        return D

    assert _projected_cg_pin_failures(bad)


def test_inverted_jacobi_preconditioner_is_caught(monkeypatch):
    """T = diag(|a_ii|) instead of its inverse no longer pays on the badly
    scaled Laplacian (the preconditioning pin's speed-up fails)."""
    import scipy.sparse as sp

    L = W.laplacian_2d(24).to_scipy()
    d = np.exp(np.random.default_rng(3).uniform(-2.0, 2.0, L.shape[0]))
    S = (sp.diags(np.sqrt(d)) @ L @ sp.diags(np.sqrt(d))).tocsr()
    anorm = float(abs(S).sum(axis=1).max())
    X0 = W.gaussian_block(S.shape[0], 12, 5)
    plain = O.lobpcg(S, X0, 6, anorm, tol=1e-8, n_es=8, se=O.SEParams("fix"), max_iter=600)
    diag = np.abs(S.diagonal())
    bad = O.lobpcg(S, X0, 6, anorm, tol=1e-8, n_es=8, se=O.SEParams("fix"), max_iter=600,
                   precond=lambda R: diag[:, None] * R)
    assert not (bad.converged and 2 * bad.iterations < plain.iterations)
