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
