"""The FP64 oracle against facts fixed by the paper and by mathematics (CPU only)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from tests import _pins as pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --- Section 4 worked example (3 x 3), values printed in the paper -----------

def _inverse_op(A):
    return lambda X: np.linalg.solve(A, X)


def test_worked_example_si_step_matches_printed_values():
    g = _golden("worked_example_3x3.json")
    A = np.diag(g["A_diag"])
    X0 = np.array(g["X0"])
    theta, X1 = O.si_step(_inverse_op(A), A, X0)
    X1 = pins.normalize_signs(X1)
    printed = np.array(g["si_step_X1"])
    for v, p in zip(X1.ravel(), printed.ravel()):
        assert pins.matches_printed(v, p), (v, p)
    assert np.all(np.diff(theta) > 0)
    assert pins.matches_printed(pins.prop1_rate(A, X1[:, 0]), g["si_step_rho_x1"])


def test_worked_example_power_step_and_rate():
    g = _golden("worked_example_3x3.json")
    A = np.diag(g["A_diag"])
    x0 = np.array(g["X0"])[:, :1]
    _, x1 = O.si_step(_inverse_op(A), A, x0)
    x1 = pins.normalize_signs(x1)[:, 0]
    ref = np.array(g["power_step_x1_times_sqrt10101"]) / math.sqrt(10101.0)
    assert np.allclose(x1, ref, rtol=1e-14, atol=1e-16)
    assert pins.matches_printed(pins.prop1_rate(A, x1), g["power_step_rho"], digits=3)


def test_worked_example_expanded_step_matches_printed_values():
    g = _golden("worked_example_3x3.json")
    A = np.diag(g["A_diag"])
    X0 = np.array(g["X0"])
    _, x1 = O.si_step(_inverse_op(A), A, X0[:, :1])
    Xexp = np.hstack([x1, X0[:, 1:2]])
    _, X2 = O.si_step(_inverse_op(A), A, Xexp)
    X2 = pins.normalize_signs(X2)
    printed = np.array(g["expanded_step_X2"])
    for v, p in zip(X2.ravel(), printed.ravel()):
        assert pins.matches_printed(v, p), (v, p)
    rho = pins.prop1_rate(A, X2[:, 0])
    assert pins.matches_printed(rho, g["expanded_step_rho_x1"])
    assert rho < 0.5 * g["asymptotic_rate"]


# --- Closed-form spectra ------------------------------------------------------

def _check(res, A, exact, tol=1e-8, lam_rtol=1e-10):
    return pins.eigen_failures(res.lam, res.V, A.to_scipy(), A.anorm, exact, tol, lam_rtol)


def test_config1_lobpcg_matches_closed_form():
    A = W.laplacian_2d(32)
    X0 = W.gaussian_block(A.n, 16, 201)
    res = O.lobpcg(A.to_scipy(), X0, 8, A.anorm, tol=1e-8)
    assert res.converged
    assert _check(res, A, pins.laplacian_spectrum(32, 2, 8)) == []


def test_config1_subspace_iteration_matches_closed_form():
    A = W.laplacian_2d(32)
    X0 = W.gaussian_block(A.n, 16, 201)
    res = O.subspace_iteration(A.to_scipy(), X0, 8, A.anorm, tol=1e-8)
    assert res.converged
    # |dlambda| <~ ||r||^2 / gap with ||r|| <= 1e-8 ||A||; gap(lam_8, lam_17) ~ 0.11
    assert _check(res, A, pins.laplacian_spectrum(32, 2, 8), lam_rtol=1e-9) == []


@pytest.mark.parametrize("strategy", ["none", "fix", "slope", "slopek"])
def test_lobpcg_shrink_expand_matches_closed_form_3d(strategy):
    m, n_ev, nb, n_es = 14, 24, 36, 29
    A = W.laplacian_3d(m)
    X0 = W.gaussian_block(A.n, nb, 11)
    res = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_es,
                   se=O.SEParams(strategy))
    assert res.converged
    assert _check(res, A, pins.laplacian_spectrum(m, 3, n_ev), lam_rtol=1e-9) == []
    if strategy != "none":
        assert res.n_shrinks >= 1


@pytest.mark.parametrize("strategy", ["fix", "slopek"])
def test_si_shrink_expand_matches_closed_form(strategy):
    m, n_ev, nb = 20, 6, 12
    A = W.laplacian_2d(m)
    X0 = W.gaussian_block(A.n, nb, 5)
    res = O.subspace_iteration(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                               se=O.SEParams(strategy))
    assert res.converged
    assert res.n_shrinks >= 1
    assert _check(res, A, pins.laplacian_spectrum(m, 2, n_ev), lam_rtol=1e-9) == []


@pytest.mark.parametrize("strategy", ["none", "fix", "slope", "slopek"])
def test_steepest_descent_matches_closed_form(strategy):
    m, n_ev, nb = 16, 6, 12
    A = W.laplacian_2d(m)
    X0 = W.gaussian_block(A.n, nb, 7)
    res = O.steepest_descent(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                             se=O.SEParams(strategy), max_iter=3000)
    assert res.converged
    assert _check(res, A, pins.laplacian_spectrum(m, 2, n_ev), lam_rtol=1e-9) == []
    if strategy != "none":
        assert res.n_shrinks >= 1


def test_steepest_descent_ritz_values_bound_from_above_and_decrease():
    """span{X, R} contains X, so the Ritz values never increase (a shrink keeps
    the first n_es), and they bound the eigenvalues from above (Courant-Fischer)."""
    m, n_ev = 8, 6
    A = W.laplacian_3d(m)
    exact = pins.laplacian_spectrum(m, 3, n_ev)
    X0 = W.gaussian_block(A.n, 12, 13)
    res = O.steepest_descent(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-9, n_es=n_ev + 2,
                             se=O.SEParams("fix", r_warm=1e-2), max_iter=3000)
    assert res.converged and res.n_shrinks >= 1
    thetas = [h["theta"] for h in res.history if "theta" in h]
    for t in thetas:
        assert np.all(t >= exact * (1 - 1e-13) - 1e-15)
    for a, b in zip(thetas, thetas[1:]):
        assert np.all(b <= a + 1e-13 * np.abs(a))


# --- Invariants -----------------------------------------------------------------

def test_lobpcg_ritz_values_bound_from_above_and_decrease():
    """Courant-Fischer: theta_i >= lambda_i; the LOBPCG space keeps all of X, so
    theta_i never increases (shrink keeps the first n_es, expansion only adds)."""
    m, n_ev = 12, 16
    A = W.laplacian_3d(m)
    exact = pins.laplacian_spectrum(m, 3, n_ev)
    X0 = W.gaussian_block(A.n, 24, 3)
    res = O.lobpcg(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-9, n_es=n_ev + 3,
                   se=O.SEParams("fix", r_warm=1e-2))
    assert res.converged and res.n_shrinks >= 1
    thetas = [h["theta"] for h in res.history if "theta" in h]
    for t in thetas:
        assert np.all(t >= exact * (1 - 1e-13) - 1e-15)
    for a, b in zip(thetas, thetas[1:]):
        assert np.all(b <= a + 1e-13 * np.abs(a))


def test_si_ritz_values_bound_from_above():
    A = W.laplacian_2d(16)
    exact = pins.laplacian_spectrum(16, 2, 4)
    X0 = W.gaussian_block(A.n, 8, 2)
    res = O.subspace_iteration(A.to_scipy(), X0, 4, A.anorm, tol=1e-8)
    for h in res.history:
        if "theta" in h:
            assert np.all(h["theta"] >= exact * (1 - 1e-13))


def test_orth_is_orthonormal_and_spans_input():
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((500, 12)) @ np.diag(np.logspace(0, -9, 12))
    Q, kept = O.orth(Y)
    assert kept.tolist() == list(range(12))
    assert np.abs(Q.T @ Q - np.eye(12)).max() < 1e-12
    assert np.linalg.norm(Y - Q @ (Q.T @ Y)) < 1e-12 * np.linalg.norm(Y)


def test_orth_drops_dependent_columns_in_order():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((300, 4))
    Y = np.hstack([B[:, :2], B[:, :1] * 3 - B[:, 1:2], B[:, 2:]])  # column 2 dependent
    Q, kept = O.orth(Y)
    assert kept.tolist() == [0, 1, 3, 4]
    assert np.abs(Q.T @ Q - np.eye(4)).max() < 1e-12
    assert np.linalg.norm(Y - Q @ (Q.T @ Y)) < 1e-11 * np.linalg.norm(Y)


def test_hl_basis_spans_new_and_old_active_x():
    """[Z1, C_P] orthonormal and its span equals span{Z1, E_active} (Section 2.3)."""
    rng = np.random.default_rng(2)
    m, k = 30, 8
    Z, _ = np.linalg.qr(rng.standard_normal((m, m)))
    active = np.array([1, 2, 4, 5, 7])
    Z1, CP = O.hl_basis(Z, k, active)
    assert CP.shape == (m, active.size)
    C = np.hstack([Z1, CP])
    assert np.abs(C.T @ C - np.eye(C.shape[1])).max() < 1e-13
    E = np.eye(m)[:, active]
    # E lies in span(C), and span(C) has exactly dim k + |active|
    assert np.linalg.norm(E - C @ (C.T @ E)) < 1e-12
    assert np.linalg.matrix_rank(np.hstack([Z1, E]), tol=1e-10) == C.shape[1]


# --- Brute force on tiny inputs ----------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_random_sparse_spd(seed):
    A = W.random_sparse_spd(150, 0.05, seed)
    dense = A.to_scipy().toarray()
    exact = np.linalg.eigvalsh(dense)[:6]
    X0 = W.gaussian_block(A.n, 10, 100 + seed)
    for res in (
        O.lobpcg(A.to_scipy(), X0, 6, A.anorm, tol=1e-10),
        O.lobpcg(A.to_scipy(), X0, 6, A.anorm, tol=1e-10, n_es=8,
                 se=O.SEParams("slopek", r_warm=1e-1)),
        O.subspace_iteration(A.to_scipy(), X0, 6, A.anorm, tol=1e-10, max_iter=50000),
    ):
        assert res.converged
        assert pins.eigen_failures(res.lam, res.V, dense, A.anorm, exact, 1e-10, 1e-9) == []


# --- Theorem 1 (Section 5, eq. (convergerate)) on random SPD matrices -----------------

@pytest.mark.parametrize("seed", range(5))
def test_theorem1_rate_bound_for_one_si_step(seed):
    rng = np.random.default_rng(seed)
    n, k, l = 40, 3, 7
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sig = np.sort(rng.uniform(0.1, 10.0, size=n))[::-1]
    B = (V * sig) @ V.T
    X, _ = np.linalg.qr(rng.standard_normal((n, k)))
    _, Xn = O.si_step(lambda Y: B @ Y, B, X)
    lhs = pins.tan_angle(V[:, :k], V[:, k:], Xn) / pins.tan_angle(V[:, :k], V[:, k:], X)
    rhs = pins.theorem1_bound(sig, V.T @ X, k, l)
    assert lhs <= rhs * (1 + 1e-10)


# --- Shrink-and-expand leaves the answer unchanged ------------------------------------

def test_shrink_expand_does_not_change_the_answer():
    A = W.laplacian_3d(12)
    X0 = W.gaussian_block(A.n, 24, 9)
    base = O.lobpcg(A.to_scipy(), X0, 16, A.anorm, tol=1e-9)
    for s in ("fix", "slope", "slopek"):
        r = O.lobpcg(A.to_scipy(), X0, 16, A.anorm, tol=1e-9, n_es=19, se=O.SEParams(s))
        assert r.converged
        assert np.max(np.abs(r.lam - base.lam) / base.lam) < 1e-10


# --- Vectors appended at an expansion (Section 6) --------------------------------------

def _expand_case(m=40, n_ev=10, n_extra=10, seed=1):
    A = W.laplacian_2d(m)
    nb = n_ev + n_extra
    X0 = W.gaussian_block(A.n, nb, seed)
    draw = lambda e, d: W.seeded_expansion_block(A.n, d, nb, e, seed + 100)  # noqa: E731
    return A, X0, nb, n_ev + min(5, n_extra - 1), draw


@pytest.mark.parametrize("solver", ["si", "lobpcg", "sd"])
@pytest.mark.parametrize("kind", ["random", "powered"])
def test_expansion_vectors_reach_the_closed_form_spectrum(solver, kind):
    if kind == "powered" and solver != "si":
        pytest.skip("powered X_drop is defined for subspace iteration")
    m, n_ev = 20, 6
    A, X0, nb, n_es, draw = _expand_case(m, n_ev, 6, 5)
    f = {"si": O.subspace_iteration, "lobpcg": O.lobpcg, "sd": O.steepest_descent}[solver]
    res = f(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_es, se=O.SEParams("fix"),
            max_iter=20000, expand_vectors=kind, random_block=draw)
    assert res.converged and res.n_expands >= 1
    assert _check(res, A, pins.laplacian_spectrum(m, 2, n_ev), lam_rtol=1e-9) == []


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_expansion_vector_choice_orders_as_the_paper_reports(seed):
    """Section 6 (the vectors appended in the expansion, and its figure of SI
    and LOBPCG under fix): reusing X_drop converges in fewer iterations than
    appending random vectors, and powering X_drop (SI) in fewer still. Checked
    on the 40 x 40 Dirichlet Laplacian, n_ev = 10, block 20, n_es = 15."""
    A, X0, nb, n_es, draw = _expand_case(seed=seed)
    it = {}
    for kind in ("xdrop", "random", "powered"):
        r = O.subspace_iteration(A.to_scipy(), X0, 10, A.anorm, tol=1e-8, n_es=n_es,
                                 se=O.SEParams("fix"), expand_vectors=kind, random_block=draw)
        assert r.converged
        it["si", kind] = r.iterations
    for kind in ("xdrop", "random"):
        r = O.lobpcg(A.to_scipy(), X0, 10, A.anorm, tol=1e-8, n_es=n_es, se=O.SEParams("fix"),
                     expand_vectors=kind, random_block=draw)
        assert r.converged
        it["lobpcg", kind] = r.iterations
    assert it["si", "random"] > it["si", "xdrop"] > it["si", "powered"], it
    assert it["lobpcg", "random"] > it["lobpcg", "xdrop"], it


def test_expansion_vectors_leave_the_fix_schedule_unchanged():
    """fix decides shrinks and expansions from the iteration count alone
    (Algorithm 6), so every choice of vectors gives the same schedule over the
    iterations both runs make."""
    A, X0, nb, n_es, draw = _expand_case(16, 4, 4, 3)
    runs = [O.subspace_iteration(A.to_scipy(), X0, 4, A.anorm, tol=1e-8, n_es=n_es,
                                 se=O.SEParams("fix"), expand_vectors=k, random_block=draw)
            for k in ("xdrop", "random", "powered")]
    L = min(len(r.history) for r in runs)
    sched = [[(h["expand"], h["shrink"]) for h in r.history[:L]] for r in runs]
    assert sched[0] == sched[1] == sched[2]
    assert any(e for e, _ in sched[0])


def test_powered_xdrop_on_a_diagonal_matrix_is_a_scaled_power():
    """On A = diag(a) the held X_drop after t power steps is, row by row,
    X_drop(shrink) times prod over the steps of (sigma - a_i) / (sigma - theta_1):
    the expansion then appends exactly that block. Checked through the first
    expansion of a run whose expansion basis is recorded by the apply hook."""
    rng = np.random.default_rng(4)
    a = np.sort(rng.uniform(0.5, 10.0, 60))
    A = sp.diags(a).tocsr()
    sigma = 10.0
    X0 = rng.standard_normal((60, 8))
    seen = []

    def op(Y):
        seen.append(Y.copy())
        return sigma * Y - A @ Y

    r = O.subspace_iteration(A, X0, 3, sigma, tol=1e-13, n_es=5,
                             se=O.SEParams("fix", r_warm=1.0, j_warm=2), apply_op=op,
                             expand_vectors="powered", max_iter=40)
    # With a custom operator the power step is not rescaled: X_drop(t) is
    # (sigma I - A)^t X_drop(shrink), so consecutive held blocks differ by
    # the row factors sigma - a_i exactly.
    shr = next(h["j"] for h in r.history if h["shrink"])
    exp = next(h["j"] for h in r.history if h["expand"])
    assert exp > shr + 1
    held = [Y for Y in seen if Y.shape[1] == 3][:exp - shr]  # the first wait
    assert len(held) == exp - shr
    for prev, nxt in zip(held, held[1:]):
        np.testing.assert_allclose(nxt, (sigma - a)[:, None] * prev, rtol=1e-12, atol=1e-12)


# --- Chebyshev-filtered subspace iteration ------------------------------------------------

def _cheb_closed(x, d):
    """T_d(x) from its trigonometric / hyperbolic closed form."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(d * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** d * np.cosh(d * np.arccosh(np.abs(xo)))
    return out


@pytest.mark.parametrize("degree", [1, 2, 5, 12])
def test_chebyshev_filter_on_a_diagonal_matrix_is_the_closed_form(degree):
    rng = np.random.default_rng(degree)
    a = np.sort(rng.uniform(0.0, 8.0, 50))
    A = sp.diags(a).tocsr()
    Y = rng.standard_normal((50, 4))
    lower, cut, upper = a[0], a[9], 8.0
    c, e = 0.5 * (upper + cut), 0.5 * (upper - cut)
    rho = _cheb_closed((a - c) / e, degree) / _cheb_closed(np.array([(lower - c) / e]), degree)[0]
    np.testing.assert_allclose(O.chebyshev_filter(A, Y, degree, lower, cut, upper), rho[:, None] * Y,
                               rtol=1e-10, atol=1e-12)
    # the filter is one at `lower` and at most one in modulus on [cut, upper] relative to it
    assert abs(rho[0] - 1.0) < 1e-12
    assert np.all(np.abs(rho[a >= cut]) <= 1.0 / abs(_cheb_closed(np.array([(lower - c) / e]), degree)[0]) + 1e-12)


@pytest.mark.parametrize("strategy", ["none", "fix"])
def test_filtered_subspace_iteration_matches_closed_form_in_fewer_iterations(strategy):
    """Degree-8 Chebyshev filtering reaches the closed-form spectrum, and its
    per-iteration damping 1/T_8 makes it need far fewer iterations than the
    degree-one shifted step (here more than 8x fewer SpMM-weighted steps)."""
    m, n_ev, nb = 20, 6, 12
    A = W.laplacian_2d(m)
    X0 = W.gaussian_block(A.n, nb, 5)
    plain = O.subspace_iteration(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                                 se=O.SEParams(strategy))
    filt = O.subspace_iteration(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                                se=O.SEParams(strategy), filter_degree=8)
    assert filt.converged and plain.converged
    assert _check(filt, A, pins.laplacian_spectrum(m, 2, n_ev), lam_rtol=1e-9) == []
    assert 8 * filt.iterations < plain.iterations


# --- TraceMIN (Algorithm 4) ------------------------------------------------------------

def test_projected_cg_reaches_the_projected_solution():
    """Enough CG steps solve P A P D = P B on range(P) exactly: compare with the
    solution in an orthonormal basis Q of range(P), D = Q (Q^T A Q)^-1 Q^T B."""
    rng = np.random.default_rng(3)
    n = 30
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    X, _ = np.linalg.qr(rng.standard_normal((n, 3)))
    B = rng.standard_normal((n, 4))
    D = O.projected_cg(sp.csr_matrix(A), X, B, n)
    Qf, _ = np.linalg.qr(np.hstack([X, rng.standard_normal((n, n - 3))]))
    Q = Qf[:, 3:]
    ref = Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ B)
    np.testing.assert_allclose(D, ref, rtol=1e-8, atol=1e-10)
    assert np.abs(X.T @ D).max() < 1e-10
    # one step is the steepest-descent step along the projected right-hand side
    r = B - X @ (X.T @ B)
    q = A @ r - X @ (X.T @ (A @ r))
    np.testing.assert_allclose(O.projected_cg(sp.csr_matrix(A), X, B, 1),
                               r * (np.sum(r * r, 0) / np.sum(r * q, 0)), rtol=1e-12)


@pytest.mark.parametrize("strategy", ["none", "fix", "slopek"])
def test_tracemin_matches_closed_form(strategy):
    m, n_ev, nb = 20, 6, 12
    A = W.laplacian_2d(m)
    X0 = W.gaussian_block(A.n, nb, 5)
    res = O.tracemin(A.to_scipy(), X0, n_ev, A.anorm, tol=1e-8, n_es=n_ev + 2,
                     se=O.SEParams(strategy, r_warm=1e-2))
    assert res.converged
    assert _check(res, A, pins.laplacian_spectrum(m, 2, n_ev), lam_rtol=1e-9) == []
    if strategy != "none":
        assert res.n_shrinks >= 1


def test_tracemin_trace_decreases_and_bounds_from_above():
    """Sameh and Wisniewski: each TraceMIN step lowers the trace of the Ritz
    values (a CG solve from zero lowers the quadratic, and orthonormalizing
    X - D with X^T D = 0 lowers it further); Courant-Fischer bounds every
    Ritz value from below by the exact eigenvalue."""
    A = W.laplacian_3d(10)
    X0 = W.gaussian_block(A.n, 14, 2)
    res = O.tracemin(A.to_scipy(), X0, 10, A.anorm, tol=1e-10)
    tr = np.array([h["trace"] for h in res.history])
    assert res.converged and np.all(np.diff(tr) <= 1e-12 * abs(tr[0]))
    exact = np.sort(np.linalg.eigvalsh(A.to_scipy().toarray()))[:10]
    assert np.all(res.lam >= exact - 1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_tracemin_brute_force_random_sparse_spd(seed):
    A = W.random_sparse_spd(150, 0.04, seed)
    X0 = W.gaussian_block(A.n, 10, seed + 30)
    res = O.tracemin(A.to_scipy(), X0, 6, A.anorm, tol=1e-9, max_iter=3000)
    exact = np.sort(np.linalg.eigvalsh(A.to_scipy().toarray()))[:6]
    assert res.converged
    np.testing.assert_allclose(res.lam, exact, rtol=1e-10)


# --- Preconditioned LOBPCG / SD (W <- T R, Algorithms 2 and 3) -----------------------------

def _scaled_laplacian(m=24, seed=3):
    """D^1/2 L D^1/2 with log-uniform D over e^[-2, 2]: badly scaled, SPD."""
    L = W.laplacian_2d(m).to_scipy()
    d = np.exp(np.random.default_rng(seed).uniform(-2.0, 2.0, L.shape[0]))
    S = (sp.diags(np.sqrt(d)) @ L @ sp.diags(np.sqrt(d))).tocsr()
    return S, float(abs(S).sum(axis=1).max())


def test_orth_of_a_wide_block_keeps_a_basis():
    Y = np.random.default_rng(0).standard_normal((5, 8))
    Q, kept = O.orth(Y)
    assert Q.shape == (5, 5) and list(kept) == [0, 1, 2, 3, 4]
    assert np.abs(Q.T @ Q - np.eye(5)).max() < 1e-14


@pytest.mark.parametrize("solver", ["lobpcg", "sd"])
def test_jacobi_preconditioning_speeds_up_a_badly_scaled_problem(solver):
    """With T = diag(A)^-1 on D^1/2 L D^1/2 the iteration needs far fewer
    steps and still reaches the brute-force spectrum."""
    S, anorm = _scaled_laplacian()
    f = O.lobpcg if solver == "lobpcg" else O.steepest_descent
    X0 = W.gaussian_block(S.shape[0], 12, 5)
    exact = np.sort(np.linalg.eigvalsh(S.toarray()))[:6]
    plain = f(S, X0, 6, anorm, tol=1e-8, n_es=8, se=O.SEParams("fix"), max_iter=3000)
    pre = f(S, X0, 6, anorm, tol=1e-8, n_es=8, se=O.SEParams("fix"), max_iter=3000,
            precond=O.jacobi_preconditioner(S))
    assert pre.converged
    np.testing.assert_allclose(pre.lam, exact, rtol=1e-10)
    assert 2 * pre.iterations < plain.iterations


def test_scalar_preconditioner_leaves_lobpcg_unchanged():
    """T = c I changes no subspace: the residual history is that of T = I."""
    A = W.laplacian_2d(16)
    X0 = W.gaussian_block(A.n, 12, 4)
    a = O.lobpcg(A.to_scipy(), X0, 6, A.anorm, tol=1e-8, n_es=8, se=O.SEParams("fix"))
    b = O.lobpcg(A.to_scipy(), X0, 6, A.anorm, tol=1e-8, n_es=8, se=O.SEParams("fix"),
                 precond=O.jacobi_preconditioner(A.to_scipy()))  # the diagonal is 4 everywhere
    ra = np.array([h["r"] for h in a.history])
    rb = np.array([h["r"] for h in b.history])
    assert len(ra) == len(rb)
    np.testing.assert_allclose(ra, rb, rtol=1e-6)


def test_tracemin_with_random_expansion_vectors_reaches_the_closed_form():
    A, X0, nb, n_es, draw = _expand_case(20, 6, 6, 5)
    res = O.tracemin(A.to_scipy(), X0, 6, A.anorm, tol=1e-8, n_es=n_es,
                     se=O.SEParams("fix", r_warm=1e-2), expand_vectors="random", random_block=draw)
    assert res.converged and res.n_expands >= 1
    assert _check(res, A, pins.laplacian_spectrum(20, 2, 6), lam_rtol=1e-9) == []
