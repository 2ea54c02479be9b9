"""Seeded input generators: sizes, symmetry, norms and reproducibility (CPU only)."""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import workloads as W
from tests import _pins as pins


def _is_symmetric(A):
    S = A.to_scipy()
    return abs(S - S.T).max() == 0


def test_laplacian_nnz_counts_and_layout():
    a2 = W.laplacian_2d(32)
    assert a2.n == 1024 and a2.nnz == 4992
    a3 = W.laplacian_3d(20)
    assert a3.n == 8000 and a3.nnz == 7 * 20**3 - 6 * 20**2
    for a in (a2, a3):
        assert a.rowptr.dtype == np.int64 and a.colind.dtype == np.int32
        assert _is_symmetric(a)
        for i in range(0, a.n, 97):
            row = a.colind[a.rowptr[i]:a.rowptr[i + 1]]
            assert np.all(np.diff(row) > 0)


def test_config2_nnz_formula():
    # 7 m^3 - 6 m^2 at m = 128 (the full config is built by the benchmark)
    m = 128
    assert 7 * m**3 - 6 * m**2 == 14_581_760


def test_laplacian_norm_is_exact_max_eigenvalue():
    for m, dim in ((8, 2), (6, 3)):
        a = W.laplacian_2d(m) if dim == 2 else W.laplacian_3d(m)
        ev = np.linalg.eigvalsh(a.to_scipy().toarray())
        assert abs(ev[-1] - a.anorm) < 1e-12
        assert np.allclose(ev[:5], pins.laplacian_spectrum(m, dim, 5), rtol=1e-12)


def test_anderson_potential_and_bound():
    a = W.anderson_3d(10, 4.0, 103)
    base = W.laplacian_3d(10).to_scipy()
    pot = (a.to_scipy() - base).diagonal()
    assert pot.min() >= -4.0 and pot.max() <= 4.0 and pot.std() > 1.0
    ev = np.linalg.eigvalsh(a.to_scipy().toarray())
    assert max(abs(ev[0]), abs(ev[-1])) <= a.anorm
    assert _is_symmetric(a)
    b = W.anderson_3d(10, 4.0, 103)
    assert np.array_equal(a.val, b.val)


def test_gaussian_block_seeded_and_fortran():
    x = W.gaussian_block(1000, 7, 5)
    y = W.gaussian_block(1000, 7, 5)
    assert x.flags.f_contiguous and x.shape == (1000, 7)
    assert np.array_equal(x, y)
    assert abs(x.mean()) < 0.05 and abs(x.std() - 1) < 0.05


def test_chung_lu_is_connected_normalized_laplacian():
    a = W.chung_lu_laplacian(3000, 16.0, 2.5, 104)
    S = a.to_scipy()
    assert _is_symmetric(a)
    g = (sp.identity(a.n) - S)
    g.data[np.abs(g.data) < 1e-15] = 0
    g.eliminate_zeros()
    ncomp, _ = connected_components(g, directed=False)
    assert ncomp == 1
    d = S.toarray()
    ev, V = np.linalg.eigh(d)
    assert abs(ev[0]) < 1e-10 and ev[1] > 1e-8 and ev[-1] <= 2.0 + 1e-12
    # zero eigenvector is D^{1/2} 1 (up to sign)
    adj = (np.abs(d) > 0).astype(float) - np.eye(a.n)
    deg = adj.sum(1)
    v = np.sqrt(deg) / np.linalg.norm(np.sqrt(deg))
    assert abs(abs(v @ V[:, 0]) - 1) < 1e-8
    assert 10 < deg.mean() < 22


def test_splitmix64_published_outputs():
    """First outputs of SplitMix64 seeded with 0 (Steele, Lea and Flood 2014)."""
    z = W.splitmix64(np.array([0, 1], dtype=np.uint64), 0)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]


def test_seeded_uniform_block_layout_and_range():
    B = W.seeded_uniform_block(5, 3, 7)
    assert B.shape == (5, 3) and B.flags.f_contiguous
    assert np.all((B >= -1.0) & (B < 1.0))
    # entry (i, j) uses counter j n + i
    z = W.splitmix64(np.array([1 * 5 + 2], dtype=np.uint64), 7)
    assert B[2, 1] == float(int(z[0]) >> 11) * 2.0 ** -52 - 1.0
    assert np.linalg.matrix_rank(W.seeded_uniform_block(200, 12, 1)) == 12


def test_seeded_expansion_block_is_standard_normal_and_independent():
    """Box-Muller of uniform pairs gives independent standard normals: the
    draws pass a Kolmogorov-Smirnov test against N(0, 1), and different
    expansions, columns and seeds are uncorrelated."""
    from scipy import stats

    B = W.seeded_expansion_block(4000, 20, 40, 3, 9)
    assert B.shape == (4000, 20) and B.flags.f_contiguous
    assert stats.kstest(B.ravel(), "norm").pvalue > 1e-3
    C = np.corrcoef(B.T)
    assert np.abs(C - np.eye(20)).max() < 0.08
    B4 = W.seeded_expansion_block(4000, 20, 40, 4, 9)
    B9 = W.seeded_expansion_block(4000, 20, 40, 3, 10)
    for other in (B4, B9):
        assert abs(np.corrcoef(B.ravel(), other.ravel())[0, 1]) < 0.02
    # column j of draw e is column nb + j of draw e - 1 (one counter space)
    np.testing.assert_array_equal(W.seeded_expansion_block(50, 45, 40, 2, 1)[:, 0],
                                  W.seeded_expansion_block(50, 45, 40, 1, 1)[:, 40])
