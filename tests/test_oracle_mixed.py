"""Pins of the mixed-precision oracle (CPU).

Storage rounding is checked against hand-derived values; the generalized
Rayleigh-Ritz step against SciPy's generalized symmetric eigensolver and
against plain Rayleigh-Ritz on an orthonormalized basis; the HL directions
against their defining properties; whole solves against the closed-form
Laplacian spectrum; the rule that ends the low-precision phase against
hand-derived exit iterations on scripted r(j) histories. Planted mistakes
(ignoring M; variants of the exit rule) must fail the checks.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W
from tests import _pins as pins

M_ = O.mixed


def test_bf16_rounding_hand_values():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3.0 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8, -2.5,
                  3.14159265, 65504.0, 2.0 ** -130])
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0);
    # 1 + 3*2^-9 is above halfway; 1 + 2^-7 + 2^-8 is halfway and rounds up to
    # the even 1 + 2^-6; pi has 8 significant bits 1.1001001 (x 2) = 3.140625.
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -6, -2.5, 3.140625, 65536.0,
                     2.0 ** -130])
    assert np.array_equal(M_.round_to(x, "bf16"), want)
    assert M_.round_to(np.array([0.1]), "fp32")[0] == 0.100000001490116119384765625
    assert np.array_equal(M_.round_to(x, "fp64"), x)


def _basis(n, m, seed, fmt):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, m)))
    return M_.round_to(Q @ (np.eye(m) + 0.05 * rng.standard_normal((m, m))), fmt)


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
def test_generalized_rr_equals_library_generalized_eigensolver(fmt):
    A = W.laplacian_2d(20).to_scipy()
    S = _basis(A.shape[0], 24, 3, fmt)
    AS = A @ S
    theta, CX, _ = M_.generalized_rr(S, AS, 10)
    ref = sla.eigh(S.T @ AS, S.T @ S, eigvals_only=True)[:10]
    assert np.max(np.abs(theta - ref)) <= 1e-12 * np.abs(ref).max()
    # and plain Rayleigh-Ritz on an orthonormal basis of the same space
    Q, _ = np.linalg.qr(S)
    assert np.max(np.abs(theta - np.linalg.eigvalsh(Q.T @ (A @ Q))[:10])) <= 1e-12 * np.abs(ref).max()
    X = S @ CX  # M-orthonormal coefficients give orthonormal Ritz vectors
    assert np.abs(X.T @ X - np.eye(10)).max() <= 1e-12


def test_generalized_rr_drops_a_dependent_column():
    A = W.laplacian_2d(16).to_scipy()
    S = _basis(A.shape[0], 12, 4, "fp32")
    S2 = np.hstack([S, S[:, 3:4]])  # exactly dependent
    theta, CX, _ = M_.generalized_rr(S2, A @ S2, 6)
    Q, _ = np.linalg.qr(S)
    ref = np.linalg.eigvalsh(Q.T @ (A @ Q))[:6]
    assert np.max(np.abs(theta - ref)) <= 1e-12 * np.abs(ref).max()
    assert M_.whiten(S2.T @ S2).shape[1] == 12


def test_hl_directions_in_whitened_coordinates():
    A = W.laplacian_2d(16).to_scipy()
    S = _basis(A.shape[0], 18, 5, "bf16")
    k, active = 6, [0, 2, 3, 5]
    theta, CX, CP = M_.generalized_rr(S, A @ S, k, active)
    XN, PN = S @ CX, S @ CP
    B = np.hstack([XN, PN])
    assert np.abs(B.T @ B - np.eye(B.shape[1])).max() <= 1e-11  # orthonormal
    old = S[:, active]
    resid = old - B @ (B.T @ old)  # span{X_new, P_new} contains the old X columns
    assert np.linalg.norm(resid) <= 1e-10 * np.linalg.norm(old)
    assert PN.shape[1] <= len(active)


def test_ignoring_m_is_caught(monkeypatch):
    """Planted mistake: treat the stored basis as orthonormal (B = I)."""
    A = W.laplacian_2d(20).to_scipy()
    S = _basis(A.shape[0], 24, 6, "bf16")
    AS = A @ S
    ref = sla.eigh(S.T @ AS, S.T @ S, eigvals_only=True)[:10]
    monkeypatch.setattr(M_, "whiten", lambda M, drop=M_.DROP: np.eye(M.shape[0]))
    theta, _, _ = M_.generalized_rr(S, AS, 10)
    assert np.max(np.abs(theta - ref)) > 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
def test_mixed_lobpcg_reaches_closed_form(fmt):
    A = W.laplacian_2d(32)
    X0 = W.gaussian_block(A.n, 16, 201)
    res, lp, hist = M_.lobpcg_mixed(A.to_scipy(), X0, 8, A.anorm, fmt=fmt)
    ex = pins.laplacian_spectrum(32, 2, 8)
    assert res.converged and lp >= 1
    assert np.max(np.abs(res.lam - ex) / ex) <= 1e-10
    _, stop, _ = O.residual_measures(A.to_scipy(), res.V, res.lam, A.anorm)
    assert stop.max() <= 1e-8
    r = np.array([h["r"] for h in hist])
    assert r.min() <= 100 * M_.DEFAULT_SWITCH[fmt]  # left at r_switch or at its floor near it


def test_mixed_lobpcg_with_shrink_expand_and_si():
    A = W.laplacian_3d(12)
    X0 = W.gaussian_block(A.n, 24, 205)
    res, lp, _ = M_.lobpcg_mixed(A.to_scipy(), X0, 16, A.anorm, fmt="fp32", n_es=21,
                                 se=O.SEParams("fix"))
    ex = pins.laplacian_spectrum(12, 3, 16)
    assert res.converged and np.max(np.abs(res.lam - ex) / ex) <= 1e-10
    A2 = W.laplacian_2d(32)
    X2 = W.gaussian_block(A2.n, 16, 201)
    res2, lp2, _ = M_.subspace_iteration_mixed(A2.to_scipy(), X2, 8, A2.anorm, fmt="fp32")
    ex2 = pins.laplacian_spectrum(32, 2, 8)
    assert res2.converged and lp2 >= 1 and np.max(np.abs(res2.lam - ex2) / ex2) <= 1e-10


@pytest.mark.parametrize("degree", [1, 2, 7])
def test_normalized_filter_recurrence_is_the_filter_definition(degree):
    """Without rounding, the per-degree normalized recurrence of the mixed
    oracle is the filter as defined (T_d(L) Y / T_d(l0) by the textbook
    recurrence)."""
    from oracle import mixed as OM

    A = W.laplacian_2d(12).to_scipy()
    Y = np.random.default_rng(degree).standard_normal((A.shape[0], 5))
    lo, cut, up = 0.06, 1.2, 8.0
    got = OM._filter_rounded(A, Y, degree, lo, cut, up, lambda Z: Z)
    np.testing.assert_allclose(got, O.chebyshev_filter(A, Y, degree, lo, cut, up), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
@pytest.mark.parametrize("degree,kind", [(8, "xdrop"), (3, "powered"), (0, "powered")])
def test_mixed_filtered_and_powered_si_reach_closed_form(fmt, degree, kind):
    from oracle import mixed as OM

    m, n_ev = 20, 6
    A = W.laplacian_2d(m)
    X0 = W.gaussian_block(A.n, 12, 5)
    res, j_lp, _ = OM.subspace_iteration_mixed(A.to_scipy(), X0, n_ev, A.anorm, fmt=fmt, n_es=8,
                                               se=O.SEParams("fix"), filter_degree=degree,
                                               expand_vectors=kind)
    assert res.converged and j_lp >= 2
    exact = pins.laplacian_spectrum(m, 2, n_ev)
    np.testing.assert_allclose(res.lam, exact, rtol=1e-9)


# --- the rule that ends the low-precision phase, on scripted r(j) histories ---
#
# Each expected iteration below is worked out by hand from the rule as stated
# beside the oracle's constants: leave at the first j with r(j) <= r_switch;
# once the best r so far is within 100 r_switch, also leave when r(j) exceeds
# ten times that best or when no new best has come for 15 iterations.


def _leave_at(rs, r_switch, rule_cls=None):
    rule = (rule_cls or M_.SwitchRule)(r_switch)
    for j, r in enumerate(rs, start=1):
        if rule.observe(j, r):
            return j
    return None


def test_switch_on_threshold():
    # 2^-j <= 1e-3 first at j = 10 (2^-10 = 9.77e-4; 2^-9 = 1.95e-3)
    assert _leave_at([2.0 ** -j for j in range(1, 40)], 1e-3) == 10
    # equality leaves: r(4) = r_switch exactly
    assert _leave_at([0.5, 0.25, 0.125, 0.0625, 0.03], 0.0625) == 4


def test_switch_on_divergence_near_the_floor():
    # best 2e-3 at j = 5 (within 100 x 1e-3); 4e-3, 1e-2 and 1.5e-2 stay at or
    # below 10 x best = 2e-2; 2.5e-2 at j = 9 exceeds it.
    rs = [1e-1, 5e-2, 1e-2, 5e-3, 2e-3, 4e-3, 1e-2, 1.5e-2, 2.5e-2, 1e-3]
    assert _leave_at(rs, 1e-3) == 9
    # exactly ten times the best does not leave (strict); the next rise does
    rs = [1e-1, 2e-3, 2e-2, 2.0000001e-2]
    assert _leave_at(rs, 1e-3) == 4


def test_switch_on_stall_near_the_floor():
    # best 5e-3 at j = 3; then 6e-3 forever: 15 iterations without a new best
    # is j = 3 + 15 = 18.
    rs = [1e-1, 1e-2, 5e-3] + [6e-3] * 30
    assert _leave_at(rs, 1e-3) == 18
    # a new best at j = 10 restarts the count: 10 + 15 = 25
    rs = [1e-1, 1e-2, 5e-3] + [6e-3] * 6 + [4e-3] + [6e-3] * 30
    assert _leave_at(rs, 1e-3) == 25
    # a new best exactly when the count would run out (j = 18 = 3 + 15) counts
    # first: the phase goes on until 18 + 15 = 33
    rs = [1e-1, 1e-2, 5e-3] + [6e-3] * 14 + [4e-3] + [6e-3] * 30
    assert _leave_at(rs, 1e-3) == 33


def test_no_divergence_or_stall_exit_far_from_the_floor():
    # best stays above 100 x 1e-3 = 0.1 until j = 25: the rise at j = 2 (20 x
    # best) and the 20-iteration plateau do not end the phase; the threshold
    # does, at j = 27.
    rs = [1.0, 20.0] + [1.5] * 22 + [0.05, 0.01, 5e-4]
    assert _leave_at(rs, 1e-3) == 27
    # with the best at exactly 100 r_switch the near-floor exits are armed:
    # best 0.1 at j = 1, then 0.2 for 15 iterations -> j = 16
    assert _leave_at([0.1] + [0.2] * 20, 1e-3) == 16


def test_default_thresholds_are_above_the_format_floor():
    # floor of r(j) in the low-precision phase is of order the unit roundoff
    # (2^-24, 2^-9); each threshold is at least a decade above it
    assert M_.DEFAULT_SWITCH["fp32"] >= 10 * 2.0 ** -24 * 16
    assert M_.DEFAULT_SWITCH["bf16"] >= 10 * 2.0 ** -8


class _NoStrictDivergence(M_.SwitchRule):
    def observe(self, j, r):
        if r < self.best:
            self.best, self.j_best = r, j
        if r <= self.r_switch:
            return True
        if self.best > M_.DIVERGE_ZONE * self.r_switch:
            return False
        return r >= M_.DIVERGE * self.best or j - self.j_best >= M_.STALL


class _StallOffByOne(M_.SwitchRule):
    def observe(self, j, r):
        if r < self.best:
            self.best, self.j_best = r, j
        if r <= self.r_switch:
            return True
        if self.best > M_.DIVERGE_ZONE * self.r_switch:
            return False
        return r > M_.DIVERGE * self.best or j - self.j_best > M_.STALL


class _NoZoneGate(M_.SwitchRule):
    def observe(self, j, r):
        if r < self.best:
            self.best, self.j_best = r, j
        return r <= self.r_switch or r > M_.DIVERGE * self.best or j - self.j_best >= M_.STALL


class _BestAfterTest(M_.SwitchRule):
    def observe(self, j, r):
        leave = r <= self.r_switch or (self.best <= M_.DIVERGE_ZONE * self.r_switch and (
            r > M_.DIVERGE * self.best or j - self.j_best >= M_.STALL))
        if r < self.best:
            self.best, self.j_best = r, j
        return leave


class _StrictThreshold(M_.SwitchRule):
    def observe(self, j, r):
        if r < self.best:
            self.best, self.j_best = r, j
        if r < self.r_switch:
            return True
        if self.best > M_.DIVERGE_ZONE * self.r_switch:
            return False
        return r > M_.DIVERGE * self.best or j - self.j_best >= M_.STALL


@pytest.mark.parametrize("bad", [_NoStrictDivergence, _StallOffByOne, _NoZoneGate, _BestAfterTest,
                                 _StrictThreshold])
def test_planted_switch_rule_mistakes_fail_a_pin(bad):
    cases = [
        ([2.0 ** -j for j in range(1, 40)], 1e-3, 10),
        ([0.5, 0.25, 0.125, 0.0625, 0.03], 0.0625, 4),
        ([1e-1, 5e-2, 1e-2, 5e-3, 2e-3, 4e-3, 1e-2, 1.5e-2, 2.5e-2, 1e-3], 1e-3, 9),
        ([1e-1, 2e-3, 2e-2, 2.0000001e-2], 1e-3, 4),
        ([1e-1, 1e-2, 5e-3] + [6e-3] * 30, 1e-3, 18),
        ([1e-1, 1e-2, 5e-3] + [6e-3] * 6 + [4e-3] + [6e-3] * 30, 1e-3, 25),
        ([1e-1, 1e-2, 5e-3] + [6e-3] * 14 + [4e-3] + [6e-3] * 30, 1e-3, 33),
        ([1.0, 20.0] + [1.5] * 22 + [0.05, 0.01, 5e-4], 1e-3, 27),
        ([0.1] + [0.2] * 20, 1e-3, 16),
    ]
    for rs, rsw, want in cases:  # the oracle's rule passes all of them ...
        assert _leave_at(rs, rsw) == want
    # ... and each planted variant fails at least one
    assert any(_leave_at(rs, rsw, bad) != want for rs, rsw, want in cases)


def test_low_precision_phase_ends_where_the_rule_fires_on_its_history():
    """The solver stops its low-precision phase exactly at the rule's
    iteration on the r(j) it recorded (BF16 on the 2-D Laplacian: the phase
    ends on the threshold, not on rounding noise)."""
    A = W.laplacian_2d(32)
    X0 = W.gaussian_block(A.n, 16, 201)
    res, lp, hist = M_.lobpcg_mixed(A.to_scipy(), X0, 8, A.anorm, fmt="bf16")
    r = [h["r"] for h in hist]
    assert _leave_at(r, M_.DEFAULT_SWITCH["bf16"]) == lp
    assert r[lp - 1] <= M_.DEFAULT_SWITCH["bf16"] and min(r[: lp - 1]) > M_.DEFAULT_SWITCH["bf16"]
