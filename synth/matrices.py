"""Seeded synthetic CSR matrices standing in for the paper's datasets.

The paper measures on MovieLens, AMiner and SNAP matrices (Section 4, Tables 1-4); none of
them is available here, so every workload is synthetic with the shape, nonzeros per row,
column-popularity skew and value distribution of the workload it stands in for. All
generators use numpy's PCG64 with an explicit seed and return a canonical CSR matrix:
int64 row pointers, int32 column indices strictly increasing within each row, float32
values. Both the FP64 oracle and the GPU path read the same float32 values.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Csr:
    """Canonical CSR matrix (row_ptr int64[m+1], col int32[nnz], val float32[nnz])."""

    m: int
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self, dtype=np.float64):
        import scipy.sparse as sp

        return sp.csr_matrix(
            (self.val.astype(dtype), self.col.astype(np.int64), self.row_ptr),
            shape=(self.m, self.n),
        )

    def toarray(self, dtype=np.float64) -> np.ndarray:
        return self.to_scipy(dtype).toarray()

    def check(self) -> None:
        """Assert canonical form: monotone pointers, in-range sorted unique columns."""
        rp, c = self.row_ptr, self.col
        assert rp.dtype == np.int64 and c.dtype == np.int32 and self.val.dtype == np.float32
        assert rp.shape == (self.m + 1,) and rp[0] == 0 and rp[-1] == c.size == self.val.size
        assert np.all(np.diff(rp) >= 0)
        if c.size:
            assert c.min() >= 0 and c.max() < self.n
            d = np.diff(c.astype(np.int64))
            starts = np.zeros(c.size, bool)
            starts[rp[:-1][np.diff(rp) > 0]] = True
            assert np.all((d > 0) | starts[1:])
        assert np.all(np.isfinite(self.val))


def _csr_from_rows(m: int, n: int, counts: np.ndarray, cols: np.ndarray, vals: np.ndarray,
                   meta=None) -> Csr:
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Csr(m, n, row_ptr, cols.astype(np.int32), vals.astype(np.float32), meta or {})


def from_dense(d: np.ndarray) -> Csr:
    """CSR of the nonzero entries of a dense array (values rounded to float32)."""
    d = np.asarray(d)
    m, n = d.shape
    mask = d != 0
    r, c = np.nonzero(mask)
    counts = mask.sum(1)
    return _csr_from_rows(m, n, counts, c, d[r, c])


def random_sparse(m: int, n: int, density: float, seed: int, empty_rows=(), empty_cols=(),
                  integer_values: bool = False) -> Csr:
    """Bernoulli(density) pattern with N(0,1) (or small-integer) values.

    ``empty_rows`` / ``empty_cols`` force whole rows/columns to be structurally empty, for
    edge-case tests of the products.
    """
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    mask[list(empty_rows), :] = False
    mask[:, list(empty_cols)] = False
    r, c = np.nonzero(mask)
    if integer_values:
        v = rng.integers(-4, 5, size=r.size).astype(np.float32)
        v[v == 0] = 1.0
    else:
        v = rng.standard_normal(r.size)
    return _csr_from_rows(m, n, mask.sum(1), c, v)


def small_decay(m: int = 2000, n: int = 1000, density: float = 0.01, seed: int = 1001) -> Csr:
    """2,000 x 1,000, 1% Bernoulli positions, N(0,1) values, rows scaled for ~1/i decay.

    Each row is normalised to unit Euclidean norm and row r (0-based) is multiplied by
    1/(r+1); an exact sigma_i = 1/i spectrum is impossible for a random pattern, so tests
    take the true spectrum from a dense SVD.
    """
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    r, c = np.nonzero(mask)
    v = rng.standard_normal(r.size)
    counts = mask.sum(1)
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    norms = np.sqrt(np.add.reduceat(v * v, row_ptr[:-1][counts > 0]))
    scale = np.zeros(m)
    scale[counts > 0] = 1.0 / norms
    scale /= np.arange(1, m + 1)
    v = v * scale[r]
    return _csr_from_rows(m, n, counts, c, v, {"workload": "small_decay"})


def _zipf_cdf(n: int, alpha: float) -> np.ndarray:
    w = (np.arange(1, n + 1, dtype=np.float64)) ** (-alpha)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf


def _first_distinct(draws: np.ndarray, t: int):
    """Per row, keep the first t distinct values in draw order."""
    order = np.argsort(draws, axis=1, kind="stable")
    sd = np.take_along_axis(draws, order, axis=1)
    first_sorted = np.ones(sd.shape, bool)
    first_sorted[:, 1:] = sd[:, 1:] != sd[:, :-1]
    is_first = np.empty_like(first_sorted)
    np.put_along_axis(is_first, order, first_sorted, axis=1)
    rank = np.cumsum(is_first, axis=1)
    keep = is_first & (rank <= t)
    ok = rank[:, -1] >= t
    return keep, ok


class _ZipfSampler:
    """Inverse-CDF sampler of the truncated Zipf law with a bucket guide table.

    Returns exactly ``searchsorted(cdf, u, side="right")`` (clipped to n-1); the guide table
    only narrows the binary search to the few indices whose CDF interval meets u's bucket.
    """

    def __init__(self, n: int, alpha: float, buckets: int = 1 << 20):
        self.n = n
        self.cdf = _zipf_cdf(n, alpha)
        self.g = buckets
        edges = np.arange(buckets + 1, dtype=np.float64) / buckets
        self.lo = np.searchsorted(self.cdf, edges[:-1], side="right")
        self.hi = np.minimum(np.searchsorted(self.cdf, edges[1:], side="right"), n - 1)

    def __call__(self, u: np.ndarray) -> np.ndarray:
        b = np.minimum((u * self.g).astype(np.int64), self.g - 1)
        lo = np.minimum(self.lo[b], self.n - 1)
        hi = self.hi[b]
        while True:
            act = lo < hi
            if not act.any():
                break
            mid = (lo + hi) >> 1
            right = self.cdf[mid] <= u
            lo = np.where(act & right, mid + 1, lo)
            hi = np.where(act & ~right, mid, hi)
        return lo.astype(np.int32)


_ZIPF_CHUNK = 1 << 17


def zipf_rows(m: int, n: int, t: int, alpha: float, seed: int, threads: int = 0) -> tuple:
    """Column pattern with exactly t distinct columns per row, drawn from a truncated Zipf.

    P(column j) is proportional to (j+1)^-alpha over j in [0, n); each row draws until it
    holds t distinct columns (column id = popularity rank, i.e. a frequency-sorted
    vocabulary). Rows are generated in fixed chunks of 2^17 with one PCG64 stream per
    chunk, so the result does not depend on the number of worker threads. Returns
    (row_ptr, col) with columns sorted within each row.
    """
    import os
    from concurrent.futures import ThreadPoolExecutor

    assert t <= n
    sampler = _ZipfSampler(n, alpha)
    cols = np.empty(m * t, np.int32)
    d0 = t + max(t // 2, 8)

    def work(ci: int) -> None:
        r0 = ci * _ZIPF_CHUNK
        r1 = min(m, r0 + _ZIPF_CHUNK)
        rng = np.random.default_rng([seed, ci])
        rows = np.arange(r0, r1)
        d = d0
        while rows.size:
            draws = sampler(rng.random((rows.size, d)))
            keep, ok = _first_distinct(draws, t)
            sel = draws[ok][keep[ok]].reshape(-1, t)
            sel.sort(axis=1)
            okrows = rows[ok]
            cols[(okrows[:, None] * t + np.arange(t)).ravel()] = sel.ravel()
            rows = rows[~ok]
            d *= 2

    nchunks = (m + _ZIPF_CHUNK - 1) // _ZIPF_CHUNK
    nthreads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(nthreads) as ex:
        list(ex.map(work, range(nchunks)))
    row_ptr = np.arange(0, m + 1, dtype=np.int64) * t
    return row_ptr, cols


def zipf_lognormal(m: int = 1_000_000, n: int = 200_000, t: int = 40, alpha: float = 1.1,
                   seed: int = 1002) -> Csr:
    """Power-law columns (Zipf alpha=1.1), ~40 nnz/row, lognormal(0,1) values."""
    row_ptr, col = zipf_rows(m, n, t, alpha, seed)
    rng = np.random.default_rng(seed + 50_000)
    val = rng.lognormal(0.0, 1.0, size=col.size).astype(np.float32)
    return Csr(m, n, row_ptr, col, val, {"workload": "zipf_lognormal"})


def aminer_tfidf(m: int = 12_869_521, n: int = 323_899, t: int = 20, alpha: float = 1.0,
                 seed: int = 1003) -> Csr:
    """Person x keyword stand-in: Zipf(1.0) columns, 20 nnz/row, tf-idf values.

    Count ~ zero-truncated Poisson(3); value = log1p(count) * ln(m / df_c) with df_c the
    number of rows that hold column c.
    """
    row_ptr, col = zipf_rows(m, n, t, alpha, seed)
    rng = np.random.default_rng(seed + 50_000)
    cnt = rng.poisson(3.0, size=col.size)
    z = cnt == 0
    while z.any():
        cnt[z] = rng.poisson(3.0, size=int(z.sum()))
        z = cnt == 0
    df = np.bincount(col, minlength=n).astype(np.float64)
    idf = np.log(m / np.maximum(df, 1.0))
    val = (np.log1p(cnt) * idf[col]).astype(np.float32)
    return Csr(m, n, row_ptr, col, val, {"workload": "aminer_tfidf"})


def zipf_normal(m: int = 500_000, n: int = 100_000, t: int = 30, alpha: float = 1.1,
                seed: int = 1004) -> Csr:
    """Zipf(1.1) columns, 30 nnz/row, N(0,1) values (the differentiated workload)."""
    row_ptr, col = zipf_rows(m, n, t, alpha, seed)
    rng = np.random.default_rng(seed + 50_000)
    val = rng.standard_normal(col.size).astype(np.float32)
    return Csr(m, n, row_ptr, col, val, {"workload": "zipf_normal"})


def ratings_zipf(m: int = 90_230, n: int = 45_115, t: int = 24, alpha: float = 1.1, seed: int = 1006) -> Csr:
    """User x item ratings stand-in (the shape and density of the paper's Matrix 2, a
    MovieLens matrix thinned to 24 nonzeros per row): Zipf(1.1) item popularity, integer
    ratings 1..5 with probabilities 0.06, 0.11, 0.27, 0.34, 0.22."""
    row_ptr, col = zipf_rows(m, n, t, alpha, seed)
    rng = np.random.default_rng(seed + 50_000)
    val = rng.choice(np.arange(1, 6, dtype=np.float32), size=col.size, p=[0.06, 0.11, 0.27, 0.34, 0.22])
    return Csr(m, n, row_ptr, col, val.astype(np.float32), {"workload": "ratings_zipf"})


def planted_blocks(m: int = 200_000, n: int = 50_000, blocks: int = 200, seed: int = 1005,
                   decades: float = 3.0) -> Csr:
    """Block-disjoint planted spectrum: A = sum_i sigma_i u_i v_i^T, sigma_i = 10^(-3i/B).

    Rows and columns are randomly permuted into ``blocks`` groups; u_i (v_i) is a random
    unit vector supported on row (column) group i, so the u_i are orthonormal, the v_i are
    orthonormal and the singular values of A are exactly sigma_1 > ... > sigma_B. With
    200 blocks of 1,000 x 250 the density is exactly 0.5%.
    """
    rng = np.random.default_rng(seed)
    sig = 10.0 ** (-decades * np.arange(1, blocks + 1) / blocks)
    rperm = rng.permutation(m)
    cperm = rng.permutation(n)
    rblk = np.array_split(rperm, blocks)
    cblk = [np.sort(b) for b in np.array_split(cperm, blocks)]
    blk_of_row = np.empty(m, np.int64)
    u = np.empty(m)
    for i, b in enumerate(rblk):
        blk_of_row[b] = i
        g = rng.standard_normal(b.size)
        u[b] = g / np.linalg.norm(g)
    v = np.empty(n)
    for b in cblk:
        g = rng.standard_normal(b.size)
        v[b] = g / np.linalg.norm(g)
    counts = np.array([cblk[i].size for i in blk_of_row], np.int64)
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.concatenate([cblk[i] for i in blk_of_row]) if m else np.zeros(0, np.int64)
    rows = np.repeat(np.arange(m), counts)
    val = sig[blk_of_row[rows]] * u[rows] * v[col]
    meta = {"workload": "planted_blocks", "sigma": sig, "row_blocks": rblk,
            "col_blocks": cblk, "u": u, "v": v}
    return Csr(m, n, row_ptr, col.astype(np.int32), val.astype(np.float32), meta)


# Workload registry: name -> (generator, full-size kwargs, k, s, passes)
WORKLOADS = {
    "small_decay": (small_decay, {}, 10, 5, 3),
    "zipf_lognormal": (zipf_lognormal, {}, 100, 20, 5),
    "aminer_tfidf": (aminer_tfidf, {}, 100, 20, 5),
    "zipf_normal": (zipf_normal, {}, 50, 10, 4),
    "planted_blocks": (planted_blocks, {}, 100, 20, 5),
    "ratings_zipf": (ratings_zipf, {}, 100, 5, 11),
}
