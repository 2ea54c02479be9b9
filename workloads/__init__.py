"""Seeded synthetic inputs for the shrink-and-expand eigensolvers.

This module is shared by the FP64 oracle, the tests and the benchmark. It only
builds inputs: sparse symmetric matrices in CSR form, an upper bound on their
2-norm (the ``||A||_2`` that the per-pair stopping test of the paper's
numerical section scales the residual by), and seeded Gaussian starting blocks.
It contains none of the eigensolver arithmetic.

Matrix families (shapes of the workloads the solvers are measured on):

* ``laplacian_2d(m)``: 5-point Dirichlet Laplacian on an m x m grid,
  ``T_m (x) I + I (x) T_m`` with ``T_m = tridiag(-1, 2, -1)``, lexicographic
  order with the first grid index fastest.
* ``laplacian_3d(m)``: 7-point Dirichlet Laplacian on an m^3 grid, same order.
* ``anderson_3d(m, w, seed)``: ``laplacian_3d(m)`` plus a diagonal potential
  drawn uniformly from [-w, w] (Anderson-type model, indefinite for w > 0).
* ``chung_lu_laplacian(n, mean_degree, exponent, seed)``: normalized graph
  Laplacian ``I - D^{-1/2} A_g D^{-1/2}`` of a connected Chung-Lu power-law
  graph with unit weights.
* ``magnetic_laplacian(m, phases)``: complex Hermitian Laplacian of a periodic
  grid (torus) with a uniform phase per step in each direction (a uniform
  vector potential); its spectrum is known in closed form (``magnetic_spectrum``).
* ``random_sparse_hermitian(n, density, seed)``: small complex Hermitian
  matrices for brute-force checks.
Complex matrices come as ``CSRMatrix`` with complex128 values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSRMatrix:
    """Real symmetric or complex Hermitian sparse matrix in CSR form with its
    full pattern stored."""

    n: int
    rowptr: np.ndarray  # int64, n + 1
    colind: np.ndarray  # int32, nnz, sorted within each row
    val: np.ndarray  # float64 (or complex128 for a Hermitian matrix), nnz
    anorm: float  # an upper bound of ||A||_2 (exact where a closed form exists)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.val)

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix(
            (self.val, self.colind.astype(np.int64), self.rowptr), shape=(self.n, self.n)
        )


def _from_scipy(a: sp.spmatrix, anorm: float, name: str) -> CSRMatrix:
    a = sp.csr_matrix(a, dtype=np.float64)
    a.sum_duplicates()
    a.sort_indices()
    return CSRMatrix(
        n=a.shape[0],
        rowptr=np.ascontiguousarray(a.indptr, dtype=np.int64),
        colind=np.ascontiguousarray(a.indices, dtype=np.int32),
        val=np.ascontiguousarray(a.data, dtype=np.float64),
        anorm=float(anorm),
        name=name,
    )


def _from_scipy_complex(a: sp.spmatrix, anorm: float, name: str) -> CSRMatrix:
    a = sp.csr_matrix(a, dtype=np.complex128)
    a.sum_duplicates()
    a.sort_indices()
    return CSRMatrix(
        n=a.shape[0],
        rowptr=np.ascontiguousarray(a.indptr, dtype=np.int64),
        colind=np.ascontiguousarray(a.indices, dtype=np.int32),
        val=np.ascontiguousarray(a.data, dtype=np.complex128),
        anorm=float(anorm),
        name=name,
    )


def _magnetic_ring(m: int, phi: float) -> sp.csr_matrix:
    """m-point periodic ring: 2 on the diagonal, -e^{i phi} at (j, j + 1) and
    -e^{-i phi} at (j + 1, j), indices mod m (m >= 3)."""
    j = np.arange(m)
    rows = np.concatenate([j, j, (j + 1) % m])
    cols = np.concatenate([j, (j + 1) % m, j])
    vals = np.concatenate([np.full(m, 2.0 + 0j), np.full(m, -np.exp(1j * phi)),
                           np.full(m, -np.exp(-1j * phi))])
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, m))


def magnetic_laplacian(m: int, phases) -> CSRMatrix:
    """Complex Hermitian Laplacian of the periodic m^d grid (d = len(phases),
    1 to 3) with phase phases[a] on every step in direction a (first grid
    index fastest): the Kronecker sum of ``_magnetic_ring(m, phases[a])``.
    Eigenvalues sum_a (2 - 2 cos(2 pi k_a / m + phases[a])), k_a = 0..m-1
    (``magnetic_spectrum``); ``anorm`` is the exact largest one."""
    d = len(phases)
    a = None
    for ax, phi in enumerate(phases):
        slow = sp.identity(m ** (d - 1 - ax), format="csr", dtype=np.complex128)
        fast = sp.identity(m ** ax, format="csr", dtype=np.complex128)
        term = sp.kron(sp.kron(slow, _magnetic_ring(m, phi)), fast)
        a = term if a is None else a + term
    lam_max = float(magnetic_spectrum(m, phases)[-1])
    return _from_scipy_complex(a, lam_max, f"magnetic{d}d_{m}")


def magnetic_spectrum(m: int, phases) -> np.ndarray:
    """All eigenvalues of ``magnetic_laplacian(m, phases)``, ascending."""
    k = 2.0 * np.pi * np.arange(m) / m
    total = np.zeros(1)
    for phi in phases:
        one = 2.0 - 2.0 * np.cos(k + phi)
        total = (total[:, None] + one[None, :]).ravel()
    return np.sort(total)


def random_sparse_hermitian(n: int, density: float, seed: int) -> CSRMatrix:
    """Random sparse complex Hermitian matrix (B + B^H) / 2 + a real diagonal,
    entries normal; ``anorm`` is the Gershgorin bound."""
    rng = np.random.default_rng(seed)
    nnz = max(1, int(density * n * n))
    r = rng.integers(0, n, nnz)
    c = rng.integers(0, n, nnz)
    v = rng.standard_normal(nnz) + 1j * rng.standard_normal(nnz)
    b = sp.csr_matrix((v, (r, c)), shape=(n, n))
    a = 0.5 * (b + b.conj().T) + sp.diags(rng.standard_normal(n).astype(np.complex128), 0)
    a = sp.csr_matrix(a)
    gersh = float(np.max(np.asarray(abs(a).sum(axis=1)).ravel()))
    return _from_scipy_complex(a, gersh, f"randherm_{n}")


def gaussian_block_complex(n: int, nb: int, seed: int) -> np.ndarray:
    """n x nb complex start block: real and imaginary parts independent
    standard normals (``default_rng(seed)``, real part drawn first), scaled
    by 1/sqrt(2)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n, nb))
    im = rng.standard_normal((n, nb))
    return np.asfortranarray((re + 1j * im) / math.sqrt(2.0))


def _second_difference(m: int) -> sp.csr_matrix:
    off = -np.ones(m - 1)
    return sp.diags([off, 2.0 * np.ones(m), off], [-1, 0, 1], format="csr")


def dirichlet_laplacian_max_eig(m: int, dim: int) -> float:
    """Largest eigenvalue of the dim-dimensional m-point Dirichlet Laplacian.

    Used as the exact ``||A||_2`` input of the stopping test.
    """
    return dim * (2.0 - 2.0 * math.cos(m * math.pi / (m + 1)))


def laplacian_2d(m: int) -> CSRMatrix:
    t = _second_difference(m)
    eye = sp.identity(m, format="csr")
    a = sp.kron(eye, t) + sp.kron(t, eye)
    return _from_scipy(a, dirichlet_laplacian_max_eig(m, 2), f"laplace2d_{m}x{m}")


def laplacian_3d(m: int) -> CSRMatrix:
    t = _second_difference(m)
    eye = sp.identity(m, format="csr")
    a = (
        sp.kron(eye, sp.kron(eye, t))
        + sp.kron(eye, sp.kron(t, eye))
        + sp.kron(t, sp.kron(eye, eye))
    )
    return _from_scipy(a, dirichlet_laplacian_max_eig(m, 3), f"laplace3d_{m}^3")


def anderson_3d(m: int, w: float, seed: int) -> CSRMatrix:
    """3-D 7-point Laplacian plus a uniform random diagonal potential in [-w, w].

    ``anorm`` is the Gershgorin bound 12 + w.
    """
    base = laplacian_3d(m).to_scipy()
    rng = np.random.default_rng(seed)
    pot = rng.uniform(-w, w, size=base.shape[0])
    a = base + sp.diags(pot, 0, format="csr")
    return _from_scipy(a, 12.0 + w, f"anderson3d_{m}^3_w{w:g}")


def potential_laplacian(m: int, dim: int, w: float, seed: int) -> CSRMatrix:
    """2-D or 3-D Dirichlet Laplacian plus a uniform diagonal potential in [-w, w]."""
    base = (laplacian_2d(m) if dim == 2 else laplacian_3d(m)).to_scipy()
    rng = np.random.default_rng(seed)
    pot = rng.uniform(-w, w, size=base.shape[0])
    a = base + sp.diags(pot, 0, format="csr")
    return _from_scipy(a, 4.0 * dim + w, f"laplace{dim}d_{m}_w{w:g}")


def chung_lu_laplacian(n: int, mean_degree: float, exponent: float, seed: int) -> CSRMatrix:
    """Normalized Laplacian of a connected Chung-Lu graph with power-law degrees.

    Expected degrees ``w_i = c (i + i0)^(-1/(exponent-1))`` are scaled to the
    requested mean, with ``i0`` chosen so that ``max w <= sqrt(sum w)``. Each
    unordered pair {i, j} is an edge with probability ``min(1, w_i w_j / sum w)``,
    sampled per row with geometric skips (Miller and Hagberg, 2011). Self loops
    and duplicates are dropped. Every vertex outside the largest connected
    component is then joined by one edge to a uniformly chosen vertex of it, so
    the graph is connected and the Laplacian has a simple zero eigenvalue with
    eigenvector ``D^{1/2} 1``. Spectrum lies in [0, 2]; ``anorm`` = 2.
    """
    from scipy.sparse.csgraph import connected_components

    rng = np.random.default_rng(seed)
    gamma = 1.0 / (exponent - 1.0)
    # choose i0 so that the largest expected degree stays below sqrt(sum w)
    i0 = 1.0
    for _ in range(60):
        idx = np.arange(n, dtype=np.float64) + i0
        w = idx ** (-gamma)
        w *= mean_degree * n / w.sum()
        if w[0] <= math.sqrt(w.sum()):
            break
        i0 *= 1.5
    total = w.sum()
    rows: list[np.ndarray] = []
    cols: list[np.ndarray] = []
    # weights are non-increasing in i, so p_ij <= w_i w_i' / total for j >= i'
    for i in range(n - 1):
        j = i + 1
        p = min(1.0, w[i] * w[j] / total)
        out_j = []
        while j < n and p > 0.0:
            if p < 1.0:
                r = rng.random()
                j += int(math.floor(math.log(r) / math.log1p(-p)))
            if j >= n:
                break
            q = min(1.0, w[i] * w[j] / total)
            if rng.random() < q / p:
                out_j.append(j)
            p = q
            j += 1
        if out_j:
            rows.append(np.full(len(out_j), i, dtype=np.int64))
            cols.append(np.asarray(out_j, dtype=np.int64))
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    g = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n)).tocsr()
    g = g + g.T
    g.data[:] = 1.0
    ncomp, labels = connected_components(g, directed=False)
    if ncomp > 1:
        big = np.bincount(labels).argmax()
        inside = np.flatnonzero(labels == big)
        outside = np.flatnonzero(labels != big)
        targets = inside[rng.integers(0, inside.size, size=outside.size)]
        extra = sp.coo_matrix(
            (np.ones(outside.size), (outside, targets)), shape=(n, n)
        ).tocsr()
        g = g + extra + extra.T
        g.data[:] = 1.0
    deg = np.asarray(g.sum(axis=1)).ravel()
    dinv = 1.0 / np.sqrt(deg)
    lap = sp.identity(n, format="csr") - sp.diags(dinv) @ g @ sp.diags(dinv)
    return _from_scipy(lap, 2.0, f"chunglu_{n}_d{mean_degree:g}_b{exponent:g}")


def gaussian_block(n: int, nb: int, seed: int) -> np.ndarray:
    """Seeded N(0, 1) starting block, n x nb, Fortran (column-major) order."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((nb, n)).T)


def splitmix64(counter: np.ndarray, seed: int) -> np.ndarray:
    """SplitMix64 output for the Weyl-sequence states seed + (counter + 1) * 0x9E3779B97F4A7C15
    (mod 2^64): the published mixer of Steele, Lea and Flood (2014)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def seeded_uniform_block(n: int, nb: int, seed: int) -> np.ndarray:
    """The start block the library generates when se_solve gets X0 = NULL: entry
    (i, j) is 2 u - 1 with u = (splitmix64(j n + i) >> 11) 2^-53, exact in FP64,
    n x nb column-major."""
    k = (np.arange(nb, dtype=np.uint64)[None, :] * np.uint64(n) + np.arange(n, dtype=np.uint64)[:, None])
    z = splitmix64(k, seed)
    return np.asfortranarray((z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0)


def seeded_expansion_block(n: int, d: int, nb: int, e: int, seed: int) -> np.ndarray:
    """The normally distributed block the library draws for the e-th expansion
    (e = 1, 2, ...) when the expansion vectors are random: entry (i, j), j < d,
    takes counters 2t and 2t + 1 with t = (e nb + j) n + i (past the start
    block's n nb counters), u1 = ((z1 >> 11) + 1) 2^-53 in (0, 1],
    u2 = (z2 >> 11) 2^-53 in [0, 1), and the Box-Muller (1958) value
    sqrt(-2 ln u1) cos(2 pi u2). n x d column-major FP64."""
    t = ((np.uint64(e) * np.uint64(nb) + np.arange(d, dtype=np.uint64)[None, :]) * np.uint64(n)
         + np.arange(n, dtype=np.uint64)[:, None])
    z1 = splitmix64(np.uint64(2) * t, seed)
    z2 = splitmix64(np.uint64(2) * t + np.uint64(1), seed)
    u1 = ((z1 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (z2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.asfortranarray(np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2))


def random_sparse_spd(n: int, density: float, seed: int) -> CSRMatrix:
    """Small random sparse symmetric positive definite matrix (diagonally dominant)."""
    rng = np.random.default_rng(seed)
    b = sp.random(n, n, density=density, random_state=rng, format="csr")
    b = b + b.T
    absrow = np.asarray(abs(b).sum(axis=1)).ravel()
    a = b + sp.diags(absrow + rng.uniform(0.1, 1.0, size=n))
    dense = a.toarray()
    bound = float(np.max(np.abs(dense).sum(axis=1)))
    return _from_scipy(a, bound, f"rand_spd_{n}")


# Named workloads. Each entry gives the matrix builder and the solver shape.
WORKLOADS = {
    "laplace2d_32": dict(build=lambda: laplacian_2d(32), n_ev=8, n_extra=8, x0_seed=201),
    "laplace3d_128": dict(build=lambda: laplacian_3d(128), n_ev=64, n_extra=32, x0_seed=202),
    "anderson3d_100": dict(
        build=lambda: anderson_3d(100, 4.0, 103), n_ev=200, n_extra=50, x0_seed=203
    ),
    "chunglu_500k": dict(
        build=lambda: chung_lu_laplacian(500_000, 16.0, 2.5, 104), n_ev=32, n_extra=16, x0_seed=204
    ),
}


def serving_requests(count: int, seed: int = 305, n_min: float = 1e4, n_max: float = 1e6,
                     ev_min: int = 4, ev_max: int = 64) -> list:
    """A stream of eigenproblem requests for the serving workload.

    Each request is a 2-D or 3-D Dirichlet Laplacian (probability 1/2 each)
    with a diagonal potential U[-2, 2]; the target size is log-uniform in
    [n_min, n_max] and the grid side is round(n^(1/dim)), so n = m^dim;
    n_ev ~ U{ev_min..ev_max} and n_extra = n_ev // 2. Returns dicts with dim,
    m, n, n_ev, n_extra and the potential's seed (built by
    ``potential_laplacian``).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dim = 2 if rng.random() < 0.5 else 3
        target = float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        m = max(4, int(round(target ** (1.0 / dim))))
        n_ev = int(rng.integers(ev_min, ev_max + 1))
        out.append({"dim": dim, "m": m, "n": m ** dim, "n_ev": n_ev, "n_extra": n_ev // 2,
                    "pot_seed": 10000 + i})
    return out


def poisson_gaps(count: int, rate: float, seed: int = 306) -> np.ndarray:
    """Inter-arrival gaps (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return rng.exponential(1.0 / rate, size=count)
