"""The Gram entry point that allocates nothing (library-held scratch) against
se_op_gram on the same inputs: two calls in a row, the second smaller; and
the widest blocks, whose row chunking the fixed scratch limits."""
import numpy as np
import pytest

from tests.gpu_util import gpu_ctx, to_dev

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _row_major(n, w, ld, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, ld))
    X[:, :w] = rng.standard_normal((n, w))
    return X


def _both(ctx, U, mu, V, mv, same):
    from paper_2409_05572_amd import api

    Ud = to_dev(U)
    Vd = Ud if same else to_dev(V)
    C1 = to_dev(np.full((mu, mv), np.nan))
    C2 = to_dev(np.full((mu, mv), np.nan))
    api.gram(ctx, Ud, mu, Vd, mv, C1)
    api.gram_noalloc(ctx, Ud, mu, Vd, mv, C2)
    return C1.cpu().numpy(), C2.cpu().numpy()


def _bound(U, mu, V, mv):
    n = U.shape[0]
    return 2 * n * U64 * (np.abs(U[:, :mu]).T @ np.abs(V[:, :mv]))


def test_noalloc_gram_matches_se_op_gram_twice(ctx):
    # 1) tall symmetric product: the scratch limits the row chunks (the
    #    summation order differs from se_op_gram's), both within the bound of
    #    the definition and exactly symmetric
    n, m = 1_000_003, 96
    print(f"[no_alloc] call 1: n={n} m={m} symmetric", flush=True)
    U = _row_major(n, m, m, 11)
    C1, C2 = _both(ctx, U, m, U, m, True)
    ref = U.T @ U
    bound = _bound(U, m, U, m)
    assert np.all(np.abs(C1 - ref) <= bound)
    assert np.all(np.abs(C2 - ref) <= bound)
    assert np.all(np.abs(C2 - C1) <= 2 * bound)
    assert np.array_equal(C2, C2.T)
    # 2) smaller, non-symmetric, ragged widths and leading dimensions: the
    #    chunk plan fits the scratch unchanged, so the result is bitwise
    #    se_op_gram's, and nothing of call 1 leaks into it
    n, mu, mv = 30_001, 41, 70
    print(f"[no_alloc] call 2: n={n} mu={mu} mv={mv}", flush=True)
    U = _row_major(n, mu, mu + 1, 12)
    V = _row_major(n, mv, mv + 2, 13)
    C1, C2 = _both(ctx, U, mu, V, mv, False)
    assert np.array_equal(C1, C2)
    assert np.all(np.abs(C2 - U[:, :mu].T @ V[:, :mv]) <= _bound(U, mu, V, mv))


def test_noalloc_gram_widest_blocks(ctx):
    # mu = mv = 1024: 121 output tiles, the chunks limited to 4 (4 x 1024^2
    # doubles = the whole scratch)
    n, m = 5001, 1024
    print(f"[no_alloc] widest: n={n} mu=mv={m}", flush=True)
    U = _row_major(n, m, m, 14)
    V = _row_major(n, m, m, 15)
    C1, C2 = _both(ctx, U, m, V, m, False)
    ref = U.T @ V
    bound = _bound(U, m, V, m)
    assert np.all(np.abs(C1 - ref) <= bound)
    assert np.all(np.abs(C2 - ref) <= bound)


def test_noalloc_gram_rejects_bad_arguments(ctx):
    from paper_2409_05572_amd import _lib, api

    U = to_dev(np.zeros((10, 1026)))
    C = to_dev(np.zeros((1025, 1025)))
    with pytest.raises(_lib.SeError) as e:
        api.gram_noalloc(ctx, U, 1025, U, 1025, C)
    assert e.value.status == _lib.SE_ERR_INVALID_ARG
