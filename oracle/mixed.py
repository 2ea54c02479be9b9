"""Mixed-precision LOBPCG and subspace iteration (oracle; test infrastructure only).

The paper points to lower-precision arithmetic for the bulk of the work as
future work (concluding section) and gives no scheme. This oracle computes,
in plain NumPy, the scheme fixed by the readings below (the whitening drop
threshold and the rule for leaving the low-precision phase are stated, with
their grounds, beside their constants):

* Low-precision phase. Every n-length block (X, P, W, their images under A,
  the dropped blocks) is stored rounded to FP32 or BF16 right after the step
  that produces it; the matrix values are rounded to FP32. Gram matrices of the
  stored blocks and all small dense work are FP64.
* The stored basis S is orthonormal only to the storage precision, so the
  Rayleigh-Ritz step solves A_p z = theta M z with M = S^T S. Here M is
  whitened through its eigendecomposition after unit column scaling,
  directions whose eigenvalue falls below 450 * 2^-24 being dropped (a
  different factorization from the library's Cholesky, on purpose).
* The Hetmaniuk-Lehoucq basis (Section 2.3) is built in the whitened
  coordinates from the old X columns.
* The phase ends by ``SwitchRule`` (below); then the FP64 solver continues
  from [X, X_drop] (LOBPCG also keeps P).
* Subspace iteration: Y = sigma X - A X (plus X_drop at an expansion), then
  the same generalized Rayleigh-Ritz step on span(Y). With a Chebyshev filter
  of degree d (``filter_degree``) Y is p(A) X for the filter of
  ``solvers.chebyshev_filter``; every intermediate block Y_i = T_i(L) X /
  T_i(l0) (normalized at each degree so that it stays of order one in the
  storage format) is stored rounded, and A Y_i uses the rounded matrix. A
  powered X_drop (``expand_vectors="powered"``) takes the same step (or the
  shifted step divided by sigma - theta_1) while it is held, also stored
  rounded.

Shrink-and-expand follows Algorithm 5 with the strategies of Section 3.2, as
in ``solvers.py``. The final result is that of the FP64 solver and so has the
same plain definition (the n_ev smallest eigenpairs).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import solvers as S_
from .strategy import SEController, SEParams

U32 = 2.0 ** -24
# Whitening drop threshold on the eigenvalues of the unit-scaled M = S^T S.
# A stored column is known only to the storage format's relative rounding u,
# so the part of a new column that is independent of the others, of relative
# size delta, carries a relative error of about u / delta. Directions are kept
# while delta^2 >= 450 u, the same threshold in units of u as the FP64
# solvers' column drop (1e-13 ~ 450 u_64), so the kept directions are accurate
# to u / delta <= sqrt(u) / 21.
DROP = 450.0 * U32
# Leaving the low-precision phase (the paper names lower precision for the
# bulk work only as an outlook, so these are readings, not the paper's):
# * r(j) <= r_switch. r(j) of a block stored with unit roundoff u cannot fall
#   much below u: on the test workloads the phase floors at 0.5-1 u for BF16
#   (u = 2^-9) and at 1.5-35 u for FP32 (u = 2^-24; the power-law graph is
#   the worst). r_switch sits at least five times above the worst floor: FP32
#   1e-5, BF16 4e-2 (about ten times BF16's machine epsilon 2^-8), so the phase
#   ends on the threshold rather than on rounding noise.
# * Once r(j) is within DIVERGE_ZONE r_switch of the threshold (the best value
#   so far), two signs that the floor was reached after all also end it:
#   r(j) > DIVERGE x best (noise drives the iteration away from its best
#   iterate), or no new best for STALL iterations. STALL exceeds one
#   shrink-and-expand cycle (j_e + j_s = 14 with the paper's parameters), so
#   the transient of an expansion cannot trigger it.
DEFAULT_SWITCH = {"fp32": 1e-5, "bf16": 4e-2}
DIVERGE_ZONE = 100.0
DIVERGE = 10.0
STALL = 15


class SwitchRule:
    """When the low-precision phase ends, fed r(1), r(2), ... in order.

    ``observe(j, r)`` records r(j) (the best value so far includes it) and
    returns True at the iteration where the phase ends.
    """

    def __init__(self, r_switch):
        self.r_switch = float(r_switch)
        self.best = np.inf
        self.j_best = 0

    def observe(self, j, r):
        if r < self.best:
            self.best, self.j_best = r, j
        if r <= self.r_switch:
            return True
        if self.best > DIVERGE_ZONE * self.r_switch:
            return False  # early iterations may rise and stall far from the floor
        return r > DIVERGE * self.best or j - self.j_best >= STALL


def round_to(Y, fmt):
    """Values of Y as stored in format fmt ('fp64', 'fp32' or 'bf16'), as FP64.

    BF16 keeps the upper 16 bits of the FP32 pattern, rounded to nearest even
    (after rounding to FP32, as a value computed in FP32 would be).
    """
    Y = np.asarray(Y, dtype=np.float64)
    if fmt == "fp64":
        return Y.copy()
    f = Y.astype(np.float32)
    if fmt == "fp32":
        return f.astype(np.float64)
    if fmt != "bf16":
        raise ValueError(fmt)
    u = np.ascontiguousarray(f).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def whiten(M, drop=DROP):
    """B (m x r) with B^T M B = I spanning M's numerically independent part.

    Columns are scaled to unit norm (D M D), the scaled matrix is
    diagonalized, and eigenvalues below ``drop`` are discarded.
    """
    d = np.sqrt(np.maximum(np.diag(M), 0.0))
    Dinv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    Ms = (M * Dinv[:, None]) * Dinv[None, :]
    Ms = 0.5 * (Ms + Ms.T)
    mu, U = np.linalg.eigh(Ms)
    keep = mu > drop
    return (Dinv[:, None] * U[:, keep]) / np.sqrt(mu[keep])[None, :]


def generalized_rr(S, AS, k, active=None, drop=DROP):
    """Rayleigh-Ritz of A on range(S) for a non-orthonormal stored basis S.

    M = S^T S, A_p = S^T (A S); with B from ``whiten``, the k lowest pairs of
    B^T A_p B give theta and Y1. With ``active`` (positions in S of the old X
    columns) the HL directions are C_P' = Y2 orth(Y2^T E'), E' = B^T M E.
    Returns (theta[:k], C_X, C_P) with X_new = S C_X, P_new = S C_P.
    """
    M = S.T @ S
    Ap = S.T @ AS
    Ap = 0.5 * (Ap + Ap.T)
    B = whiten(M, drop)
    k = min(k, B.shape[1])
    theta, Y = np.linalg.eigh(B.T @ Ap @ B)
    CX = B @ Y[:, :k]
    if active is None or len(active) == 0:
        return theta[:k], CX, CX[:, :0]
    E = (M @ B)[np.asarray(active, dtype=np.int64), :].T  # B^T M E
    Y2 = Y[:, k:]
    QB, _ = S_.orth(Y2.T @ E, 1e-12)
    return theta[:k], CX, B @ (Y2 @ QB)


def _measures(X, AX, lam, anorm, n_ev):
    R = AX - X * lam[None, :]
    rn = np.linalg.norm(R, axis=0)
    xn = np.linalg.norm(X, axis=0)
    stop = rn / (anorm * xn)
    paper = rn / (anorm * xn + xn * np.abs(lam))
    return R, stop, paper


def lobpcg_mixed(A, X0, n_ev, anorm, fmt="fp32", tol=1e-8, n_es=None, se: SEParams | None = None,
                 r_switch=None, max_iter=1000):
    """LOBPCG (Algorithm 3) with a low-precision phase, then FP64 LOBPCG.

    Returns (result, lp_iterations, lp_history) where ``result`` is the FP64
    phase's ``SolveResult`` (its history continues after the low-precision
    phase) unless the low-precision phase already met the stopping test.
    """
    se = se or SEParams()
    r_switch = DEFAULT_SWITCH[fmt] if r_switch is None else r_switch
    rd = lambda Y: round_to(Y, fmt)  # noqa: E731
    A32 = sp.csr_matrix(A).astype(np.float32).astype(np.float64)
    nb = X0.shape[1]
    ctl = SEController(se if S_._se_enabled(se, n_ev, n_es, nb) else SEParams("none"))

    X = rd(X0)
    AX = rd(A32 @ X)
    lam, CX, _ = generalized_rr(X, AX, nb)
    X, AX = rd(X @ CX), rd(AX @ CX)
    P = X[:, :0]
    AP = P.copy()
    Xd = Pd = AXd = APd = None
    rule = SwitchRule(r_switch)
    hist = []
    j = 0
    for j in range(1, max_iter + 1):
        R, stop, paper = _measures(X, AX, lam, anorm, n_ev)
        r = float(np.max(paper[:n_ev]))
        ctl.observe(j, r)
        hist.append(dict(j=j, r=r, k=X.shape[1], p=P.shape[1]))
        leave = rule.observe(j, r)
        if np.all(stop[:n_ev] <= tol):
            res = S_.SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), j, True, hist)
            return res, j, hist
        if leave:
            break
        expand = ctl.ifexpand(j)
        k = X.shape[1]
        W = rd(R)
        AW = rd(A32 @ W)
        blocks, images = [X, P], [AX, AP]
        active = list(range(k))
        k_keep = k
        if expand and Xd is not None:
            active += [k + P.shape[1] + q for q in range(Xd.shape[1])]
            blocks += [Xd, Pd]
            images += [AXd, APd]
            k_keep = k + Xd.shape[1]
            Xd = Pd = AXd = APd = None
            ctl.did_expand(j)
        blocks.append(W)
        images.append(AW)
        S = np.hstack(blocks)
        AS = np.hstack(images)
        lam, CX, CP = generalized_rr(S, AS, k_keep, active)
        X, P = rd(S @ CX), rd(S @ CP)
        AX, AP = rd(AS @ CX), rd(AS @ CP)
        if ctl.ifshrink(j) and X.shape[1] > n_es:
            Xd, AXd = X[:, n_es:], AX[:, n_es:]
            Pd, APd = P[:, n_es:], AP[:, n_es:]
            X, AX, P, AP = X[:, :n_es], AX[:, :n_es], P[:, :n_es], AP[:, :n_es]
            lam = lam[:n_es]
            ctl.did_shrink(j)
    X0_64 = X if Xd is None else np.hstack([X, Xd[:, : nb - X.shape[1]]])
    res = S_.lobpcg(A, X0_64, n_ev, anorm, tol=tol, n_es=n_es, se=se, max_iter=max_iter, P0=P)
    return res, j, hist


def _filter_rounded(A32, Y, degree, lower, cut, upper, rd):
    """p(A) Y for the Chebyshev filter damping [cut, upper], one at `lower`,
    with each normalized intermediate T_i(L) Y / T_i(l0) stored rounded:
    Y_{i+1} = (2 t_i L Y_i - t_{i-1} Y_{i-1}) / t_{i+1}, t_i = T_i(l0)."""
    c = 0.5 * (upper + cut)
    e = 0.5 * (upper - cut)
    l0 = (lower - c) / e
    L = lambda Z: (rd(A32 @ Z) - c * Z) / e  # noqa: E731
    t_prev, t = 1.0, l0
    Y_prev, Yc = Y, rd(L(Y) / t)
    for _ in range(2, degree + 1):
        t_next = 2.0 * l0 * t - t_prev
        Y_prev, Yc = Yc, rd((2.0 * t * L(Yc) - t_prev * Y_prev) / t_next)
        t_prev, t = t, t_next
    return Yc


def subspace_iteration_mixed(A, X0, n_ev, anorm, fmt="fp32", sigma=None, tol=1e-8, n_es=None,
                             se: SEParams | None = None, r_switch=None, max_iter=20000,
                             filter_degree=0, expand_vectors="xdrop"):
    """Subspace iteration (Algorithm 1) with a low-precision phase, then FP64."""
    if expand_vectors not in ("xdrop", "powered"):
        raise ValueError("mixed precision appends X_drop or the powered X_drop")
    se = se or SEParams()
    r_switch = DEFAULT_SWITCH[fmt] if r_switch is None else r_switch
    sigma = anorm if sigma is None else sigma
    rd = lambda Y: round_to(Y, fmt)  # noqa: E731
    A32 = sp.csr_matrix(A).astype(np.float32).astype(np.float64)
    nb = X0.shape[1]
    ctl = SEController(se if S_._se_enabled(se, n_ev, n_es, nb) else SEParams("none"))

    def rr(Y):
        AY = rd(A32 @ Y)
        lam, C, _ = generalized_rr(Y, AY, Y.shape[1])
        return lam, rd(Y @ C), rd(AY @ C)

    lam, X, AX = rr(rd(X0))
    Xd = None
    rule = SwitchRule(r_switch)
    hist = []
    j = 0
    for j in range(1, max_iter + 1):
        _, stop, paper = _measures(X, AX, lam, anorm, n_ev)
        r = float(np.max(paper[:n_ev]))
        ctl.observe(j, r)
        hist.append(dict(j=j, r=r, k=X.shape[1]))
        leave = rule.observe(j, r)
        if np.all(stop[:n_ev] <= tol):
            return S_.SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), j, True, hist), j, hist
        if leave:
            break
        expand = ctl.ifexpand(j)
        filt = filter_degree > 0 and sigma > lam[-1]
        if filt:
            Y = _filter_rounded(A32, X, filter_degree, lam[0], lam[-1], sigma, rd)
        else:
            Y = rd(sigma * X - AX)
        if expand_vectors == "powered" and Xd is not None:
            if filt:
                Xd = _filter_rounded(A32, Xd, filter_degree, lam[0], lam[-1], sigma, rd)
            else:
                scale = 1.0 / (sigma - lam[0]) if sigma - lam[0] > 0.0 else 1.0
                Xd = rd(scale * (sigma * Xd - rd(A32 @ Xd)))
        if expand and Xd is not None:
            Y = np.hstack([Y, Xd])
            Xd = None
            ctl.did_expand(j)
        lam, X, AX = rr(Y)
        if ctl.ifshrink(j) and X.shape[1] > n_es:
            Xd = X[:, n_es:]
            X, AX, lam = X[:, :n_es], AX[:, :n_es], lam[:n_es]
            ctl.did_shrink(j)
    X0_64 = X if Xd is None else np.hstack([X, Xd[:, : nb - X.shape[1]]])
    res = S_.subspace_iteration(A, X0_64, n_ev, anorm, sigma=sigma, tol=tol, n_es=n_es, se=se,
                                max_iter=max_iter, filter_degree=filter_degree,
                                expand_vectors=expand_vectors)
    return res, j, hist
