"""Block eigensolvers with shrink-and-expand, plain FP64 (oracle; test infrastructure only).

Follows the paper (arXiv 2409.05572):
* subspace iteration, Algorithm 1 (Section 2.1);
* steepest descent, Algorithm 2 (Section 2.2);
* LOBPCG, Algorithm 3 (Section 2.3), with soft locking and the improved
  Hetmaniuk-Lehoucq choice of P (Section 2.3 text), preconditioner T = I as in
  the experiments (Section 6.2);
* TraceMIN, Algorithm 4 (Section 2.4), with a projected conjugate-gradient
  inner solve;
* the shrink-and-expand framework, Algorithm 5 (Section 3.1), with the
  strategies of Section 3.2 (see ``strategy.py``);
* the per-pair stopping test, eq. (conv), and the overall relative residual
  r(j), eq. (rk) (Section 6.1).

Readings of points the paper leaves open (each also listed in the design notes):
* Stopping test: a pair i <= n_ev is converged when
  ``||A x_i - lambda_i x_i|| <= tol ||A|| ||x_i||``, which implies eq. (conv);
  r(j) for the strategies is eq. (rk) over i <= n_ev.
* Ordering: Ritz values are kept algebraically ascending.
* Subspace iteration operator: one shifted power step ``X <- sigma X - A X``
  with ``sigma >= lambda_max`` replaces the shift-invert solve of Algorithm 1,
  so the dominant eigenvectors of ``sigma I - A`` are the smallest of ``A``;
  Rayleigh-Ritz is done with ``A`` itself. Any other operator can be passed.
* Soft locking: pairs i <= n_ev that pass the stopping test are locked; they
  stay in X for the Rayleigh-Ritz step but leave W and P. The lock set is
  re-evaluated at every iteration.
* Hetmaniuk-Lehoucq basis: with S = [X, P, W] orthonormal and A_p = Z Theta Z^T,
  X_new = S Z1 (Z1 = first k columns). In coefficient space the old active X
  columns are unit vectors E; their part orthogonal to Z1 is Z2 (Z2^T E), so
  P_new = S Z2 Q_B with Q_B an orthonormal basis of range(Z2^T E). Then
  [X_new, P_new] is an orthonormal basis of span{X_new, X_old(active)}.
* LOBPCG expansion: S_drop = [X_drop, P_drop] is orthogonalized against S and
  orthonormalized; columns that come from X_drop go to X, the rest to P.
* Orthogonalization drops columns whose norm after projection falls below
  ``drop_tol`` times their norm before it.
* Beyond the paper's experiments: a Chebyshev filter for subspace iteration
  (Zhou and Saad) in place of its shift-invert operator, and a diagonal
  (Jacobi) preconditioner T for the W <- T R step of LOBPCG and SD.
* Expansion vectors (Section 6, the vectors appended in the expansion):
  ``expand_vectors="xdrop"`` appends the vectors dropped at the last shrink;
  ``"random"`` appends a normally distributed block of the same width,
  ``random_block(e, d)`` for the e-th expansion (LOBPCG: its first columns
  take the place of X_drop, the rest that of P_drop); ``"powered"`` (subspace
  iteration only) applies the iteration operator to X_drop at every iteration
  it is held, without orthogonalization, divided by ``sigma - theta_1``
  (theta_1 the current smallest Ritz value) so that its largest component
  stays of order one however long it waits.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from .strategy import SEController, SEParams


@dataclass
class SolveResult:
    lam: np.ndarray
    V: np.ndarray
    iterations: int
    converged: bool
    history: list = field(default_factory=list)
    n_shrinks: int = 0
    n_expands: int = 0
    max_stop_ratio: float = np.inf
    max_paper_ratio: float = np.inf


def _apply(A, X):
    """Sparse (or dense) matrix times block; a library product."""
    return A @ X


def _H(M):
    """Conjugate transpose. The paper states the problem for Hermitian A in
    C^{n x n} (Section 1) and writes X^H in its algorithms; for real blocks
    this is the plain transpose."""
    return M.conj().T


def _block(X0):
    """The start block in FP64: complex128 when X0 is complex, else float64."""
    return np.asarray(X0, dtype=np.complex128 if np.iscomplexobj(X0) else np.float64)


def residual_measures(A, X, lam, anorm):
    """Residual block R = A X - X diag(lam) and the two per-column ratios.

    ``stop``:  ||r_i|| / (||A|| ||x_i||)                 (stopping test)
    ``paper``: ||r_i|| / (||A|| ||x_i|| + ||x_i|| |lam_i|) (eq. (conv) / (rk))
    """
    AX = _apply(A, X)
    R = AX - X * lam[None, :]
    rn = np.linalg.norm(R, axis=0)
    xn = np.linalg.norm(X, axis=0)
    stop = rn / (anorm * xn)
    paper = rn / (anorm * xn + xn * np.abs(lam))
    return R, stop, paper


def orth(Y, drop_tol=1e-12):
    """Orthonormal basis of range(Y), column order kept, dependent columns dropped.

    Returns (Q, kept) where ``kept`` lists the columns of Y that contributed.
    Fast path: Householder QR when no column is numerically dependent.
    Otherwise: classical Gram-Schmidt applied twice per column, dropping a
    column whose projected norm is below ``drop_tol`` times its own norm.
    """
    k = Y.shape[1]
    if k == 0:
        return Y.copy(), np.zeros(0, dtype=np.int64)
    norms = np.linalg.norm(Y, axis=0)
    if k <= Y.shape[0]:  # a wider block has dependent columns: no fast path
        Q, R = np.linalg.qr(Y, mode="reduced")
        if np.all(np.abs(np.diag(R)) > drop_tol * norms) and np.all(norms > 0):
            return Q, np.arange(k)
    basis = []
    kept = []
    for i in range(k):
        v = Y[:, i].copy()
        if norms[i] == 0.0:
            continue
        for _ in range(2):
            if basis:
                Bm = np.stack(basis, axis=1)
                v -= Bm @ (_H(Bm) @ v)
        nv = np.linalg.norm(v)
        if nv > drop_tol * norms[i]:
            basis.append(v / nv)
            kept.append(i)
    if not basis:
        return Y[:, :0].copy(), np.zeros(0, dtype=np.int64)
    return np.stack(basis, axis=1), np.asarray(kept, dtype=np.int64)


def rayleigh_ritz(S, AS):
    """Ritz pairs of A on range(S) for orthonormal S: A_p = S^T (A S) = Z Theta Z^T.

    Theta ascending (LAPACK ``eigh``); returns (theta, Z).
    """
    Ap = _H(S) @ AS
    Ap = 0.5 * (Ap + _H(Ap))
    theta, Z = np.linalg.eigh(Ap)
    return theta, Z


def chebyshev_filter(A, Y, degree, lower, cut, upper):
    """p(A) Y with p(t) = T_d((t - c) / e) / T_d((lower - c) / e), the Chebyshev
    filter of degree d >= 1 that damps [cut, upper] and is one at ``lower``
    (c and e the centre and half-width of [cut, upper]; Zhou and Saad's filter
    for subspace iteration, 2007). Written as its definition: the textbook
    three-term recurrence T_{i+1}(L) = 2 L T_i(L) - T_{i-1}(L) on
    L = (A - cI) / e applied to Y, divided by the same recurrence on the
    scalar (lower - c) / e."""
    c = 0.5 * (upper + cut)
    e = 0.5 * (upper - cut)
    L = lambda Z: (_apply(A, Z) - c * Z) / e  # noqa: E731
    l0 = (lower - c) / e
    T_prev, T = Y, L(Y)
    t_prev, t = 1.0, l0
    for _ in range(2, degree + 1):
        T_prev, T = T, 2.0 * L(T) - T_prev
        t_prev, t = t, 2.0 * l0 * t - t_prev
    return T / t


def si_step(apply_op, A, X):
    """One subspace-iteration step (Algorithm 1 body without shrink/expand).

    X <- op(X); orthogonalize; Rayleigh-Ritz with A. Returns (theta, X_new).
    """
    Y = apply_op(X)
    Q, _ = orth(Y)
    theta, Z = rayleigh_ritz(Q, _apply(A, Q))
    return theta, Q @ Z


def hl_basis(Z, k, active, drop_tol=1e-12):
    """Coefficients [Z1, C_P] of the improved Hetmaniuk-Lehoucq basis (Section 2.3).

    ``Z`` (m x m) are the Ritz vectors of A_p in the basis S, ``k`` the width of
    X and ``active`` the positions (within the first k columns of S) of the old
    X columns that are not locked. Returns (Z1, C_P) with C_P = Z2 Q_B, where
    Q_B is an orthonormal basis of range(Z2^T E).
    """
    Z1 = Z[:, :k]
    Z2 = Z[:, k:]
    B = _H(Z2[np.asarray(active, dtype=np.int64), :])
    QB, _ = orth(B, drop_tol)
    return Z1, Z2 @ QB


def _expansion_source(expand_vectors, random_block, powered_ok):
    if expand_vectors not in ("xdrop", "random", "powered"):
        raise ValueError(f"unknown expand_vectors {expand_vectors!r}")
    if expand_vectors == "powered" and not powered_ok:
        raise ValueError("powered X_drop is defined for subspace iteration only")
    if expand_vectors == "random" and random_block is None:
        raise ValueError("random expansion vectors need random_block(e, d)")
    return expand_vectors


def jacobi_preconditioner(A):
    """T = diag(1 / |a_ii|) (1 where a_ii = 0): a symmetric positive definite
    diagonal preconditioner for the W <- T R step of Algorithms 2 and 3."""
    d = np.asarray(A.diagonal(), dtype=np.float64)
    t = np.where(d != 0.0, 1.0 / np.where(d != 0.0, np.abs(d), 1.0), 1.0)
    return lambda R: t[:, None] * R  # noqa: E731


def _se_enabled(params: SEParams, n_ev: int, n_es, nb: int) -> bool:
    return params.strategy != "none" and n_es is not None and n_ev <= n_es < nb


def lobpcg(
    A,
    X0,
    n_ev,
    anorm,
    tol=1e-8,
    n_es=None,
    se: SEParams | None = None,
    max_iter=1000,
    soft_lock=True,
    drop_tol=1e-12,
    time_limit_s=None,
    P0=None,
    expand_vectors="xdrop",
    random_block=None,
    precond=None,
):
    """LOBPCG with soft locking, HL basis and shrink-and-expand (Algorithm 3).

    ``P0``: search directions to continue with (e.g. after a low-precision
    phase); they are orthogonalized against the starting X. ``precond``: the
    preconditioner T of W <- T R as a function of the residual block (None is
    T = I, the paper's experiments).
    """
    _expansion_source(expand_vectors, random_block, False)
    se = se or SEParams()
    nb = X0.shape[1]
    ctl = SEController(se if _se_enabled(se, n_ev, n_es, nb) else SEParams("none"))
    t0 = time.perf_counter()

    # Initial Rayleigh-Ritz on the orthogonalized starting block.
    X, _ = orth(_block(X0), drop_tol)
    theta, Z = rayleigh_ritz(X, _apply(A, X))
    X = X @ Z
    lam = theta
    P = X[:, :0]
    if P0 is not None and P0.shape[1] > 0:
        P = np.asarray(P0, dtype=np.float64)
        for _ in range(2):
            P = P - X @ (_H(X) @ P)
        P, _ = orth(P, drop_tol)
    Xdrop = Pdrop = None
    history = []
    n_shr = n_exp = 0
    stop = paper = None

    for j in range(1, max_iter + 1):
        R, stop, paper = residual_measures(A, X, lam, anorm)
        r_j = float(np.max(paper[:n_ev]))
        ctl.observe(j, r_j)
        conv = stop[:n_ev] <= tol
        rec = dict(j=j, t=time.perf_counter() - t0,  # seconds since the call began
                   r=r_j, max_stop=float(np.max(stop[:n_ev])), k=X.shape[1],
                   p=P.shape[1], locked=0, a=0, expand=False, shrink=False)
        history.append(rec)
        if np.all(conv):
            return SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), j, True, history,
                               n_shr, n_exp, float(np.max(stop[:n_ev])), r_j)
        if time_limit_s is not None and time.perf_counter() - t0 > time_limit_s:
            break

        k = X.shape[1]
        locked = np.zeros(k, dtype=bool)
        if soft_lock:
            locked[:n_ev] = conv
        active = np.flatnonzero(~locked)
        expand = ctl.ifexpand(j)

        # W <- T R, restricted to the active columns; orthogonalize against
        # [X, P] (projection applied twice) and orthonormalize.
        W = R[:, active] if precond is None else precond(R[:, active])
        XP = np.hstack([X, P])
        for _ in range(2):
            W = W - XP @ (_H(XP) @ W)
        W, _ = orth(W, drop_tol)

        if expand and Xdrop is not None:
            S = np.hstack([X, P, W])
            d = Xdrop.shape[1]
            if expand_vectors == "random":
                Sd = random_block(n_exp + 1, d + Pdrop.shape[1])
            else:
                Sd = np.hstack([Xdrop, Pdrop])
            for _ in range(2):
                Sd = Sd - S @ (_H(S) @ Sd)
            Sd, kept = orth(Sd, drop_tol)
            to_x = kept < d
            new_x = np.arange(k, k + int(np.count_nonzero(to_x)))
            X = np.hstack([X, Sd[:, to_x]])
            P = np.hstack([P, Sd[:, ~to_x]])
            active = np.concatenate([active, new_x])
            Xdrop = Pdrop = None
            ctl.did_expand(j)
            n_exp += 1
            rec["expand"] = True

        S = np.hstack([X, P, W])
        k = X.shape[1]
        theta, Z = rayleigh_ritz(S, _apply(A, S))
        Z1, CP = hl_basis(Z, k, active, drop_tol)
        X = S @ Z1
        P = S @ CP
        lam = theta[:k].copy()
        rec.update(locked=int(np.count_nonzero(locked)), a=W.shape[1],
                   theta=lam[:n_ev].copy())

        if ctl.ifshrink(j):
            Xdrop = X[:, n_es:]
            Pdrop = P[:, n_es:]
            X = X[:, :n_es]
            P = P[:, :n_es]
            lam = lam[:n_es]
            ctl.did_shrink(j)
            n_shr += 1
            rec["shrink"] = True

    ms = float(np.max(stop[:n_ev])) if stop is not None else np.inf
    mp = float(np.max(paper[:n_ev])) if paper is not None else np.inf
    return SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), len(history), False, history,
                       n_shr, n_exp, ms, mp)


def steepest_descent(
    A,
    X0,
    n_ev,
    anorm,
    tol=1e-8,
    n_es=None,
    se: SEParams | None = None,
    max_iter=1000,
    soft_lock=True,
    drop_tol=1e-12,
    time_limit_s=None,
    expand_vectors="xdrop",
    random_block=None,
    precond=None,
):
    """Block steepest descent with shrink-and-expand (Algorithm 2, Section 2.2):
    X_new is the Ritz basis of span{X, T R} for the current width (T = I unless
    ``precond`` gives it as a function of the residual block).

    Readings: soft locking as in LOBPCG (locked pairs leave W); at an
    expansion X_drop is orthogonalized against X and orthonormalized before it
    is appended (the algorithm appends it as is, but the Rayleigh-Ritz step
    needs an orthonormal basis).
    """
    _expansion_source(expand_vectors, random_block, False)
    se = se or SEParams()
    nb = X0.shape[1]
    ctl = SEController(se if _se_enabled(se, n_ev, n_es, nb) else SEParams("none"))
    t0 = time.perf_counter()

    # X <- orth(X0); A_p = X^T A X = Z Lambda Z^T; X <- X Z
    X, _ = orth(_block(X0), drop_tol)
    lam, Z = rayleigh_ritz(X, _apply(A, X))
    X = X @ Z
    Xdrop = None
    history = []
    n_shr = n_exp = 0
    stop = paper = None

    for j in range(1, max_iter + 1):
        # R <- A X - X Lambda; convergence of the n_ev smallest pairs
        R, stop, paper = residual_measures(A, X, lam, anorm)
        r_j = float(np.max(paper[:n_ev]))
        ctl.observe(j, r_j)
        conv = stop[:n_ev] <= tol
        rec = dict(j=j, t=time.perf_counter() - t0,  # seconds since the call began
                   r=r_j, max_stop=float(np.max(stop[:n_ev])), k=X.shape[1], p=0,
                   locked=0, a=0, expand=False, shrink=False)
        history.append(rec)
        if np.all(conv):
            return SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), j, True, history,
                               n_shr, n_exp, float(np.max(stop[:n_ev])), r_j)
        if time_limit_s is not None and time.perf_counter() - t0 > time_limit_s:
            break
        k = X.shape[1]
        locked = np.zeros(k, dtype=bool)
        if soft_lock:
            locked[:n_ev] = conv
        active = np.flatnonzero(~locked)

        # if ifexpand(): X <- [X, X_drop]
        if ctl.ifexpand(j) and Xdrop is not None:
            Xd = random_block(n_exp + 1, Xdrop.shape[1]) if expand_vectors == "random" else Xdrop
            for _ in range(2):
                Xd = Xd - X @ (_H(X) @ Xd)
            Xd, _ = orth(Xd, drop_tol)
            X = np.hstack([X, Xd])
            Xdrop = None
            ctl.did_expand(j)
            n_exp += 1
            rec["expand"] = True

        # W <- T R (active columns); W <- W - X (X^T W), orthonormalized
        W = R[:, active] if precond is None else precond(R[:, active])
        for _ in range(2):
            W = W - X @ (_H(X) @ W)
        W, _ = orth(W, drop_tol)

        # S = [X, W]; A_p = S^T A S = Z Lambda Z^T; X <- S Z(:, 1:n_now)
        S = np.hstack([X, W])
        k = X.shape[1]
        theta, Z = rayleigh_ritz(S, _apply(A, S))
        X = S @ Z[:, :k]
        lam = theta[:k].copy()
        rec.update(locked=int(np.count_nonzero(locked)), a=W.shape[1], theta=lam[:n_ev].copy())

        # if ifshrink(): X_drop <- X(:, n_es+1:end), X <- X(:, 1:n_es)
        if ctl.ifshrink(j):
            Xdrop = X[:, n_es:]
            X = X[:, :n_es]
            lam = lam[:n_es]
            ctl.did_shrink(j)
            n_shr += 1
            rec["shrink"] = True

    ms = float(np.max(stop[:n_ev])) if stop is not None else np.inf
    mp = float(np.max(paper[:n_ev])) if paper is not None else np.inf
    return SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), len(history), False, history,
                       n_shr, n_exp, ms, mp)


def projected_cg(A, X, B, steps):
    """Approximate solution of P A P D = P B, P = I - X X^T (X orthonormal), by
    ``steps`` conjugate-gradient iterations from D = 0, each column on its own
    (TraceMIN's inexact inner solve, Section 2.4). A column stops (its step
    length is zero) once its residual vanishes or its curvature d^T P A P d is
    not positive."""
    P = lambda Z: Z - X @ (X.T @ Z)  # noqa: E731
    r = P(B)
    d = r.copy()
    D = np.zeros_like(B)
    rr = np.einsum("ij,ij->j", r, r)
    for _ in range(steps):
        q = P(_apply(A, d))
        dq = np.einsum("ij,ij->j", d, q)
        ok = (dq > 0.0) & (rr > 0.0)
        alpha = np.where(ok, rr / np.where(ok, dq, 1.0), 0.0)
        D = D + d * alpha
        r = r - q * alpha
        rr_new = np.einsum("ij,ij->j", r, r)
        beta = np.where(rr > 0.0, rr_new / np.where(rr > 0.0, rr, 1.0), 0.0)
        d = r + d * beta
        rr = rr_new
    return D


def tracemin(
    A,
    X0,
    n_ev,
    anorm,
    tol=1e-8,
    n_es=None,
    se: SEParams | None = None,
    max_iter=1000,
    cg_steps=5,
    drop_tol=1e-12,
    time_limit_s=None,
    expand_vectors="xdrop",
    random_block=None,
):
    """TraceMIN with shrink-and-expand (Algorithm 4, Section 2.4): X <- X - D
    with D from ``cg_steps`` projected CG iterations on P A P D = P R (five in
    the paper's experiments), then [X, X_drop] at an expansion, orthonormalize,
    Rayleigh-Ritz, shrink.

    Reading: the projector written I - X^H X in Algorithm 4 is I - X X^H (the
    one in the text above it); the inner solve needs P A P positive definite on
    range(P), i.e. A positive definite (as in the paper's experiments).
    ``expand_vectors="random"`` appends ``random_block(e, d)`` instead of X_drop."""
    _expansion_source(expand_vectors, random_block, False)
    se = se or SEParams()
    nb = X0.shape[1]
    ctl = SEController(se if _se_enabled(se, n_ev, n_es, nb) else SEParams("none"))
    t0 = time.perf_counter()

    X, _ = orth(_block(X0), drop_tol)
    lam, Z = rayleigh_ritz(X, _apply(A, X))
    X = X @ Z
    Xdrop = None
    history = []
    n_shr = n_exp = 0
    stop = paper = None

    for j in range(1, max_iter + 1):
        R, stop, paper = residual_measures(A, X, lam, anorm)
        r_j = float(np.max(paper[:n_ev]))
        ctl.observe(j, r_j)
        rec = dict(j=j, t=time.perf_counter() - t0,  # seconds since the call began
                   r=r_j, max_stop=float(np.max(stop[:n_ev])), k=X.shape[1],
                   trace=float(np.sum(lam)), expand=False, shrink=False)
        history.append(rec)
        if np.all(stop[:n_ev] <= tol):
            return SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), j, True, history,
                               n_shr, n_exp, float(np.max(stop[:n_ev])), r_j)
        if time_limit_s is not None and time.perf_counter() - t0 > time_limit_s:
            break

        # X <- X - D, P A P D = P R solved inexactly
        X = X - projected_cg(A, X, R, cg_steps)
        if ctl.ifexpand(j) and Xdrop is not None:
            if expand_vectors == "random":
                Xdrop = random_block(n_exp + 1, Xdrop.shape[1])
            X = np.hstack([X, Xdrop])
            Xdrop = None
            ctl.did_expand(j)
            n_exp += 1
            rec["expand"] = True
        X, _ = orth(X, drop_tol)
        lam, Z = rayleigh_ritz(X, _apply(A, X))
        X = X @ Z

        if ctl.ifshrink(j):
            Xdrop = X[:, n_es:]
            X = X[:, :n_es]
            lam = lam[:n_es]
            ctl.did_shrink(j)
            n_shr += 1
            rec["shrink"] = True

    ms = float(np.max(stop[:n_ev])) if stop is not None else np.inf
    mp = float(np.max(paper[:n_ev])) if paper is not None else np.inf
    return SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), len(history), False, history,
                       n_shr, n_exp, ms, mp)


def subspace_iteration(
    A,
    X0,
    n_ev,
    anorm,
    sigma=None,
    tol=1e-8,
    n_es=None,
    se: SEParams | None = None,
    max_iter=20000,
    apply_op=None,
    drop_tol=1e-12,
    time_limit_s=None,
    expand_vectors="xdrop",
    random_block=None,
    filter_degree=0,
):
    """Subspace iteration with Rayleigh-Ritz and shrink-and-expand (Algorithm 1).

    ``apply_op`` defaults to the shifted power step X -> sigma X - A X with
    ``sigma = anorm`` when not given. With a custom ``apply_op`` the powered
    X_drop is not rescaled. ``filter_degree`` d >= 1 replaces the operator by
    the Chebyshev filter of degree d that damps [theta_k, sigma] and is one at
    theta_1 (theta the current Ritz values of the k-column X); the powered
    X_drop then takes the same filter.
    """
    _expansion_source(expand_vectors, random_block, True)
    se = se or SEParams()
    nb = X0.shape[1]
    ctl = SEController(se if _se_enabled(se, n_ev, n_es, nb) else SEParams("none"))
    shift = None
    if apply_op is None:
        s = anorm if sigma is None else sigma
        shift = s
        apply_op = lambda Y: s * Y - _apply(A, Y)  # noqa: E731
    t0 = time.perf_counter()

    X, _ = orth(_block(X0), drop_tol)
    theta, Z = rayleigh_ritz(X, _apply(A, X))
    X = X @ Z
    lam = theta
    Xdrop = None
    history = []
    n_shr = n_exp = 0
    stop = paper = None

    for j in range(1, max_iter + 1):
        _, stop, paper = residual_measures(A, X, lam, anorm)
        r_j = float(np.max(paper[:n_ev]))
        ctl.observe(j, r_j)
        rec = dict(j=j, t=time.perf_counter() - t0,  # seconds since the call began
                   r=r_j, max_stop=float(np.max(stop[:n_ev])), k=X.shape[1],
                   expand=False, shrink=False)
        history.append(rec)
        if np.all(stop[:n_ev] <= tol):
            return SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), j, True, history,
                               n_shr, n_exp, float(np.max(stop[:n_ev])), r_j)
        if time_limit_s is not None and time.perf_counter() - t0 > time_limit_s:
            break

        if filter_degree > 0:
            up = anorm if sigma is None else sigma
            if up > lam[-1]:
                step = lambda Z: chebyshev_filter(A, Z, filter_degree, lam[0], lam[-1], up)  # noqa: E731
            else:  # no interval to damp: the plain shifted step
                step = apply_op
        else:
            step = apply_op
        Y = step(X)
        if expand_vectors == "powered" and Xdrop is not None:
            # one power step on the held X_drop, no orthogonalization
            scale = 1.0
            if step is apply_op and shift is not None and shift - lam[0] > 0.0:
                scale = 1.0 / (shift - lam[0])
            Xdrop = step(Xdrop) * scale
        if ctl.ifexpand(j) and Xdrop is not None:
            if expand_vectors == "random":
                Xdrop = random_block(n_exp + 1, Xdrop.shape[1])
            Y = np.hstack([Y, Xdrop])
            Xdrop = None
            ctl.did_expand(j)
            n_exp += 1
            rec["expand"] = True
        X, _ = orth(Y, drop_tol)
        theta, Z = rayleigh_ritz(X, _apply(A, X))
        X = X @ Z
        lam = theta.copy()
        rec["theta"] = lam[:n_ev].copy()

        if ctl.ifshrink(j):
            Xdrop = X[:, n_es:]
            X = X[:, :n_es]
            lam = lam[:n_es]
            ctl.did_shrink(j)
            n_shr += 1
            rec["shrink"] = True

    ms = float(np.max(stop[:n_ev])) if stop is not None else np.inf
    mp = float(np.max(paper[:n_ev])) if paper is not None else np.inf
    return SolveResult(lam[:n_ev].copy(), X[:, :n_ev].copy(), len(history), False, history,
                       n_shr, n_exp, ms, mp)
