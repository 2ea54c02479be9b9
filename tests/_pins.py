"""Independent facts the oracle (and then the GPU path) is checked against.

Everything here comes from mathematics or from numbers printed in the paper,
not from the oracle: closed-form Dirichlet-Laplacian spectra, principal angles,
the Proposition 1 rate (Section 4, eq. (rhopm)) and the Theorem 1 bound
(Section 5, eq. (convergerate)).
"""
from __future__ import annotations

import math

import numpy as np


def laplacian_spectrum(m: int, dim: int, count: int) -> np.ndarray:
    """The ``count`` smallest eigenvalues of the dim-D m-point Dirichlet Laplacian.

    The spectrum is every sum of ``2 - 2 cos(k pi / (m + 1))`` over the dim grid
    directions, k = 1..m.
    """
    one = 2.0 - 2.0 * np.cos(np.arange(1, m + 1) * math.pi / (m + 1))
    vals = one
    for _ in range(dim - 1):
        vals = (vals[:, None] + one[None, :]).ravel()
        vals = np.sort(vals)[: max(count, 1) * 4 + 64]
    return np.sort(vals)[:count]


def normalize_signs(V: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry is positive."""
    V = np.array(V, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[idx, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return V * sgn[None, :]


def matches_printed(value: float, printed: float, digits: int = 5) -> bool:
    """True when ``value`` rounds to ``printed`` at the given significant digits."""
    if printed == 0.0:
        return abs(value) < 10.0 ** (-digits)
    e = math.floor(math.log10(abs(printed)))
    return abs(value - printed) <= 0.51 * 10.0 ** (e - digits + 1)


def prop1_rate(A: np.ndarray, x: np.ndarray) -> float:
    """Proposition 1: rho = lambda_1 ||A^{-1} x_check|| for the inverse power method."""
    lam, V = np.linalg.eigh(A)
    v1 = V[:, 0]
    xc = x - v1 * (v1 @ x)
    xc = xc / np.linalg.norm(xc)
    return float(lam[0] * np.linalg.norm(np.linalg.solve(A, xc)))


def tan_angle(Vk: np.ndarray, Vperp: np.ndarray, Y: np.ndarray) -> float:
    """tan of the largest principal angle between range(Vk) and range(Y), dim k."""
    Yk = Vk.T @ Y
    Yp = Vperp.T @ Y
    return float(np.linalg.norm(Yp @ np.linalg.inv(Yk), 2))


def theorem1_bound(sig: np.ndarray, coeff: np.ndarray, k: int, l: int) -> float:
    """Right-hand side of eq. (convergerate) for X written in B's eigenbasis.

    ``sig`` descending eigenvalues of B, ``coeff`` = V^T X (n x k).
    """
    Xk = coeff[:k]
    Xlk = coeff[k:l]
    Xrest = coeff[k:]
    inv = np.linalg.inv(Xk)
    num = np.linalg.norm(Xlk @ inv, 2)
    den = np.linalg.norm(Xrest @ inv, 2)
    return float(sig[l] / sig[k - 1] + (sig[k] - sig[l]) / sig[k - 1] * num / den)


def subspace_gap(U: np.ndarray, V: np.ndarray) -> float:
    """sin of the largest principal angle between ranges of orthonormal U and V."""
    s = np.linalg.svd(U.T @ V, compute_uv=False)
    return float(math.sqrt(max(0.0, 1.0 - min(1.0, float(np.min(s))) ** 2)))


def eigen_failures(lam, V, A_dense_or_sparse, anorm, exact, tol=1e-8,
                   lam_rtol=1e-10, orth_tol=1e-12):
    """List of violated facts for a computed (lam, V) against exact eigenvalues.

    Checks: each eigenvalue against the exact one, the stopping test recomputed
    from scratch, orthonormality of V, ascending order.
    """
    out = []
    lam = np.asarray(lam)
    exact = np.asarray(exact)
    rel = np.abs(lam - exact) / np.maximum(np.abs(exact), 1e-300)
    if not np.all(rel <= lam_rtol):
        out.append(f"eigenvalue rel err {rel.max():.3e} > {lam_rtol}")
    R = A_dense_or_sparse @ V - V * lam[None, :]
    ratio = np.linalg.norm(R, axis=0) / (anorm * np.linalg.norm(V, axis=0))
    if not np.all(ratio <= tol * 1.0001):
        out.append(f"residual ratio {ratio.max():.3e} > {tol}")
    G = V.T @ V - np.eye(V.shape[1])
    if np.abs(G).max() > orth_tol:
        out.append(f"orthonormality {np.abs(G).max():.3e}")
    if np.any(np.diff(lam) < -1e-14 * np.abs(lam[:-1]).max()):
        out.append("not ascending")
    return out
