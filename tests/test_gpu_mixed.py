"""Mixed precision on the GPU (FP32 / BF16 panels, FP64 reductions and
refinement): the low-precision bulk kernels against FP64 products of the same
stored values, and whole solves against closed forms and the FP64 oracle.

Error bounds of the kernels follow from their arithmetic: FP32 products and
FP32 accumulation runs of at most 64 terms (folded into FP64 after that),
the FP64 coefficient matrix of an update rounded to FP32, and one rounding of
every output to its storage format.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import _pins as pins
from tests.gpu_util import gpu_ctx, to_dev

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
UNIT = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _dtype(fmt):
    import torch

    return torch.float32 if fmt == "fp32" else torch.bfloat16


def _block(a, fmt, ld=None):
    """Device block of the given format with leading dimension ld (padding
    columns hold garbage on purpose); returns (tensor, stored values as
    float64)."""
    import torch

    n, w = a.shape
    ld = ld or (w + 7) // 8 * 8
    full = np.full((n, ld), 7.0e3)
    full[:, :w] = a
    t = torch.from_numpy(full.astype(np.float32)).to(_dtype(fmt)).cuda()
    return t, t[:, :w].float().double().cpu().numpy()


def _read(t, w):
    return t[:, :w].float().double().cpu().numpy()


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
@pytest.mark.parametrize("w", [1, 3, 4, 16, 48, 69, 96, 250])
def test_spmm_lp_matches_product_of_stored_values(ctx, fmt, w):
    import torch

    from paper_2409_05572_amd import api

    A = W.anderson_3d(11, 4.0, 7)  # non-integer diagonal: FP32 rounding of A matters
    rng = np.random.default_rng(w)
    X, Xs = _block(rng.standard_normal((A.n, w)), fmt)
    Y = torch.zeros_like(X)
    M = api.Matrix.from_csr(ctx, A)
    api.spmm_lp(ctx, M, X, Y, w)
    got = _read(Y, w)
    A32 = A.to_scipy().astype(np.float32).astype(np.float64)
    ref = A32 @ Xs
    absA = abs(A32)
    nnz_row = int(np.diff(A.rowptr).max())
    bound = (nnz_row + 2) * U32 * (absA @ abs(Xs)) + UNIT[fmt] * abs(ref) + 1e-300
    assert np.all(np.abs(got - ref) <= bound)
    assert np.all(Y[:, w:].float().cpu().numpy() == 0.0)  # padding columns untouched


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
@pytest.mark.parametrize("w", [1, 2, 7, 96, 129, 250])
def test_spmm_lp_empty_rows(ctx, fmt, w):
    import torch

    from paper_2409_05572_amd import api
    from tests.gpu_util import matrix_with_empty_runs

    A = matrix_with_empty_runs()
    rng = np.random.default_rng(w + 5)
    X, Xs = _block(rng.standard_normal((A.n, w)), fmt)
    Y = torch.full_like(X, 3.0)
    api.spmm_lp(ctx, api.Matrix.from_csr(ctx, A), X, Y, w)
    got = _read(Y, w)
    A32 = A.to_scipy().astype(np.float32).astype(np.float64)
    ref = A32 @ Xs
    deg = np.diff(A.rowptr)
    assert np.all(got[deg == 0] == 0.0)
    bound = (deg.max() + 2) * U32 * (abs(A32) @ abs(Xs)) + UNIT[fmt] * abs(ref) + 1e-300
    assert np.all(np.abs(got - ref) <= bound)
    assert np.all(Y[:, w:].float().cpu().numpy() == 3.0)  # padding columns untouched


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
@pytest.mark.parametrize("w", [3, 48, 130])
def test_spmm_lp_power_law_rows(ctx, fmt, w):
    import torch

    from paper_2409_05572_amd import api

    A = W.chung_lu_laplacian(20000, 16.0, 2.5, 11)
    deg = np.diff(A.rowptr)
    rng = np.random.default_rng(w)
    X, Xs = _block(rng.standard_normal((A.n, w)), fmt)
    Y = torch.zeros_like(X)
    api.spmm_lp(ctx, api.Matrix.from_csr(ctx, A), X, Y, w)
    A32 = A.to_scipy().astype(np.float32).astype(np.float64)
    ref = A32 @ Xs
    bound = (deg.max() + 2) * U32 * (abs(A32) @ abs(Xs)) + UNIT[fmt] * abs(ref) + 1e-300
    assert np.all(np.abs(_read(Y, w) - ref) <= bound)


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
@pytest.mark.parametrize("n,mu,mv", [(1000, 1, 1), (1000, 17, 5), (20001, 96, 96), (20001, 150, 250),
                                     (70001, 250, 250), (5000, 750, 33)])
def test_gram_lp_within_fp32_accumulation_bound(ctx, fmt, n, mu, mv):
    import torch

    from paper_2409_05572_amd import api

    rng = np.random.default_rng(n + mu + mv)
    U, Us = _block(rng.standard_normal((n, mu)), fmt)
    V, Vs = _block(rng.standard_normal((n, mv)), fmt)
    C = torch.zeros((mu, mv), dtype=torch.float64, device="cuda")
    api.gram_lp(ctx, U, mu, V, mv, C)
    ref = Us.T @ Vs
    bound = 70 * U32 * (abs(Us).T @ abs(Vs))
    assert np.all(np.abs(C.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
@pytest.mark.parametrize("n,m", [(1000, 5), (20001, 96), (20001, 150), (30001, 250)])
def test_symmetric_gram_lp_within_bound(ctx, fmt, n, m):
    """U^T U (the same block twice): only output tiles on or above the
    diagonal are formed and the reduction mirrors them; the result is
    symmetric and within the FP32 accumulation bound of the stored values."""
    import torch

    from paper_2409_05572_amd import api

    rng = np.random.default_rng(n + m)
    U, Us = _block(rng.standard_normal((n, m)), fmt)
    C = torch.zeros((m, m), dtype=torch.float64, device="cuda")
    api.gram_lp(ctx, U, m, U, m, C)
    got = C.cpu().numpy()
    ref = Us.T @ Us
    assert np.all(np.abs(got - ref) <= 70 * U32 * (abs(Us).T @ abs(Us)))
    assert np.array_equal(got, got.T)


def test_gram_lp_is_deterministic(ctx):
    import torch

    from paper_2409_05572_amd import api

    rng = np.random.default_rng(3)
    U, _ = _block(rng.standard_normal((300001, 96)), "fp32")
    C1 = torch.zeros((96, 96), dtype=torch.float64, device="cuda")
    C2 = torch.zeros_like(C1)
    api.gram_lp(ctx, U, 96, U, 96, C1)
    api.gram_lp(ctx, U, 96, U, 96, C2)
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
@pytest.mark.parametrize("n,K,N,beta", [(20001, 1, 1, 0.0), (20001, 33, 16, 1.0), (20001, 250, 69, 0.0),
                                        (5003, 750, 250, 1.0), (64, 96, 96, 0.0)])
def test_update_lp_within_bound(ctx, fmt, n, K, N, beta):
    from paper_2409_05572_amd import api

    rng = np.random.default_rng(K * 1000 + N)
    U, Us = _block(rng.standard_normal((n, K)), fmt)
    Cm = rng.standard_normal((K, N))
    Out, Olds = _block(rng.standard_normal((n, N)), fmt)
    api.update_lp(ctx, U, K, to_dev(Cm), N, Out, beta)
    got = _read(Out, N)
    ref = beta * Olds + Us @ Cm
    bound = 72 * U32 * (abs(Us) @ abs(Cm) + beta * abs(Olds)) + UNIT[fmt] * abs(ref) + 1e-300
    assert np.all(np.abs(got - ref) <= bound)


def _solve(ctx, A, X0, n_ev, n_extra, **kw):
    from paper_2409_05572_amd import api

    M = api.Matrix.from_csr(ctx, A)
    return api.solve(ctx, M, X0, n_ev, n_extra, history_cap=6000, **kw)


def _check_result(A, lam, V, info, exact, lam_rtol=1e-10):
    assert info.converged and info.status == 0
    assert info.max_stop_ratio <= 1e-8
    assert np.max(np.abs(lam - exact) / np.abs(exact)) <= lam_rtol
    R = A.to_scipy() @ V - V * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))) <= 1e-8 * 1.0001
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() <= 1e-12


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
@pytest.mark.parametrize("solver", ["lobpcg", "si"])
def test_config1_mixed_matches_closed_form(ctx, fmt, solver):
    A = W.laplacian_2d(32)
    X0 = W.gaussian_block(A.n, 16, 201)
    lam, V, info = _solve(ctx, A, X0, 8, 8, solver=solver, precision=fmt)
    _check_result(A, lam, V, info, pins.laplacian_spectrum(32, 2, 8))
    h = info.history
    lp_rows = (h[:, 7].astype(int) & 4) != 0
    assert info.lp_iterations >= 1 and lp_rows.sum() == info.lp_iterations
    assert np.all(lp_rows[: info.lp_iterations]) and not lp_rows[info.lp_iterations:].any()
    # the low-precision phase got r(j) down to r_switch or stalled there
    r_lp = h[lp_rows, 1]
    assert r_lp.min() <= O.mixed.DEFAULT_SWITCH[fmt] * 100


@pytest.mark.parametrize("fmt,strategy", [("fp32", "fix"), ("fp32", "slopek"), ("bf16", "fix")])
def test_3d_laplacian_mixed_with_shrink_expand(ctx, fmt, strategy):
    m = 16
    A = W.laplacian_3d(m)
    X0 = W.gaussian_block(A.n, 48, 203)
    lam, V, info = _solve(ctx, A, X0, 32, 16, precision=fmt, strategy=strategy)
    _check_result(A, lam, V, info, pins.laplacian_spectrum(m, 3, 32))
    assert info.n_shrinks >= 1
    if fmt == "fp32":  # r(j) passes r_warm inside the FP32 phase, so it shrinks there too
        lp = (info.history[:, 7].astype(int) & 4) != 0
        assert ((info.history[lp, 7].astype(int) & 2) != 0).any()


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
def test_anderson_mixed_matches_fp64_oracle(ctx, fmt):
    """The indefinite Anderson matrix (3-D Laplacian plus a diagonal potential
    U[-4, 4]) with a low-precision phase in FP32 or BF16: the pairs against
    the FP64 oracle at the FP64 bars."""
    A = W.anderson_3d(14, 4.0, 103)
    X0 = W.gaussian_block(A.n, 30, 204)
    lam, V, info = _solve(ctx, A, X0, 20, 10, precision=fmt, strategy="fix")
    ref = O.lobpcg(A.to_scipy(), X0, 20, A.anorm, tol=1e-8)
    assert info.converged and info.lp_iterations >= 1
    scale = np.maximum(np.abs(ref.lam), 1e-3 * A.anorm)
    assert np.max(np.abs(lam - ref.lam) / scale) <= 1e-10
    R = A.to_scipy() @ V - V * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))) <= 1e-8 * 1.0001


def test_mixed_solve_is_bitwise_reproducible(ctx):
    A = W.laplacian_3d(12)
    X0 = W.gaussian_block(A.n, 24, 205)
    lam1, V1, i1 = _solve(ctx, A, X0, 16, 8, precision="fp32", strategy="fix")
    lam2, V2, i2 = _solve(ctx, A, X0, 16, 8, precision="fp32", strategy="fix")
    assert i1.iterations == i2.iterations and i1.lp_iterations == i2.lp_iterations
    assert np.array_equal(lam1, lam2) and np.array_equal(V1, V2)


def test_mixed_rejects_negative_switch_threshold(ctx):
    from paper_2409_05572_amd._lib import SeError

    A = W.laplacian_2d(8)
    X0 = W.gaussian_block(A.n, 6, 1)
    with pytest.raises(SeError):
        _solve(ctx, A, X0, 3, 3, precision="fp32", r_switch=-1.0)


def _switch_iteration(r, r_switch):
    """First iteration (1-based) at which the oracle's rule for leaving the
    low-precision phase (pinned on scripted histories in the CPU tests) fires
    on the sequence r(1), r(2), ..."""
    rule = O.mixed.SwitchRule(r_switch)
    for j, v in enumerate(r, start=1):
        if rule.observe(j, v):
            return j
    return None


# r(j) of the GPU and the oracle are compared where both lie well above the
# floor of the stored format (FP32 <= 2e-6, BF16 <= 2e-3 on these workloads),
# so that rounding differences between the two whitening factorizations do
# not matter.
ABOVE_FLOOR = {"fp32": 1e-4, "bf16": 2e-2}


@pytest.mark.parametrize("fmt,solver", [("fp32", "lobpcg"), ("bf16", "lobpcg"), ("fp32", "si")])
def test_mixed_matches_mixed_oracle(ctx, fmt, solver):
    """Same scheme on both sides (different whitening factorizations): the
    final pairs agree to the FP64 bar; r(j) of the two low-precision phases
    agrees while it is well above the format's floor, each phase ends exactly
    where the switch rule fires on its own history, and the two phases have
    the same length up to the iteration at which r(j) crosses r_switch (both
    thresholds lie well above the floor)."""
    from tests.gpu_util import cluster_angles

    A = W.laplacian_2d(32)
    X0 = W.gaussian_block(A.n, 16, 201)
    lam, V, info = _solve(ctx, A, X0, 8, 8, solver=solver, precision=fmt)
    run = O.mixed.lobpcg_mixed if solver == "lobpcg" else O.mixed.subspace_iteration_mixed
    ref, lp_ref, hist = run(A.to_scipy(), X0, 8, A.anorm, fmt=fmt)
    assert info.converged and ref.converged
    assert np.max(np.abs(lam - ref.lam) / np.abs(ref.lam)) <= 1e-10
    assert cluster_angles(lam, V, ref.V) <= 1e-6
    rsw = O.mixed.DEFAULT_SWITCH[fmt]
    h = info.history
    r_gpu = h[(h[:, 7].astype(int) & 4) != 0, 1]
    r_ref = np.array([q["r"] for q in hist])[:lp_ref]
    assert len(r_gpu) == info.lp_iterations
    assert _switch_iteration(r_gpu, rsw) == info.lp_iterations
    assert _switch_iteration(r_ref, rsw) == lp_ref
    both = min(len(r_gpu), len(r_ref))
    above = (r_gpu[:both] > ABOVE_FLOOR[fmt]) & (r_ref[:both] > ABOVE_FLOOR[fmt])
    assert above.sum() >= 5
    ratio = r_gpu[:both][above] / r_ref[:both][above]
    assert np.all((ratio > 0.8) & (ratio < 1.25))
    if fmt == "fp32":
        assert abs(info.lp_iterations - lp_ref) <= max(5, 0.3 * lp_ref)
    else:
        assert abs(info.lp_iterations - lp_ref) <= 1


@pytest.mark.parametrize("fmt,degree,kind,strategy", [("fp32", 3, "xdrop", "fix"), ("fp32", 3, "powered", "fix"),
                                                      ("bf16", 3, "powered", "fix"), ("fp32", 8, "xdrop", "none"),
                                                      ("fp32", 0, "powered", "fix")])
def test_mixed_filtered_and_powered_si_match_mixed_oracle(ctx, fmt, degree, kind, strategy):
    """Chebyshev-filtered SI and the powered X_drop with a low-precision phase
    (every intermediate block stored in FP32 / BF16) against the mixed
    oracle: the final pairs to the FP64 bar and the closed form; r(j) of the
    two low-precision phases agrees while it is well above r_switch, and the
    GPU's phase ends where the switch rule fires on its own history."""
    from tests.gpu_util import cluster_angles

    A = W.laplacian_2d(20)
    X0 = W.gaussian_block(A.n, 12, 5)
    lam, V, info = _solve(ctx, A, X0, 6, 6, solver="si", precision=fmt, strategy=strategy, n_es=8,
                          filter_degree=degree, expand_vectors=kind)
    ref, lp_ref, hist = O.mixed.subspace_iteration_mixed(A.to_scipy(), X0, 6, A.anorm, fmt=fmt, n_es=8,
                                                         se=O.SEParams(strategy), filter_degree=degree,
                                                         expand_vectors=kind)
    assert info.converged and ref.converged and info.lp_iterations >= 2
    exact = pins.laplacian_spectrum(20, 2, 6)
    assert np.max(np.abs(lam - exact) / exact) <= 1e-10
    assert np.max(np.abs(lam - ref.lam) / np.abs(ref.lam)) <= 1e-10
    assert cluster_angles(lam, V, ref.V) <= 1e-6
    rsw = O.mixed.DEFAULT_SWITCH[fmt]
    h = info.history
    r_gpu = h[(h[:, 7].astype(int) & 4) != 0, 1]
    r_ref = np.array([q["r"] for q in hist])[:lp_ref]
    assert _switch_iteration(r_gpu, rsw) == info.lp_iterations
    both = min(len(r_gpu), len(r_ref))
    above = (r_gpu[:both] > ABOVE_FLOOR[fmt]) & (r_ref[:both] > ABOVE_FLOOR[fmt])
    assert above.sum() >= 3
    ratio = r_gpu[:both][above] / r_ref[:both][above]
    assert np.all((ratio > 0.8) & (ratio < 1.25))


def test_full_size_fp32_filtered_si(ctx):
    """The 128^3 Laplacian with a degree-32 filter and an FP32 phase (fused
    low-precision product-and-step), fixed block: every eigenvalue against the
    closed form, sampled stopping test on the host, orthonormality."""
    from paper_2409_05572_amd import api

    A = W.laplacian_3d(128)
    X0 = W.gaussian_block(A.n, 96, 202)
    M = api.Matrix.from_csr(ctx, A)
    lam, V, info = api.solve(ctx, M, X0, 64, 32, solver="si", precision="fp32", filter_degree=32,
                             max_iter=500)
    assert info.converged and info.lp_iterations >= 2
    exact = pins.laplacian_spectrum(128, 3, 64)
    assert np.max(np.abs(lam - exact) / exact) <= 1e-10
    cols = np.array([0, 1, 17, 40, 63])
    R = A.to_scipy() @ V[:, cols] - V[:, cols] * lam[cols][None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V[:, cols], axis=0))) <= 1e-8 * 1.0001
    assert np.abs(V.T @ V - np.eye(64)).max() <= 1e-12
