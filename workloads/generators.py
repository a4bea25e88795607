"""Seeded generators for the matrix families of the paper's numerical section.

Each generator returns a :class:`Problem`: the matrix A (dense row-major or
CSR with int64 row pointers and int32 sorted, unique column indices), a
right-hand side ``b = A x* + noise`` in float64, the planted ``x*`` and, for the
differentiation workloads, a target ``x_t`` for the loss ``L = 0.5*||x - x_t||^2``.

Random streams: every quantity draws from its own numpy ``PCG64`` stream,
keyed by ``(seed, stream id[, chunk])``, so a quantity never depends on the
order in which others were drawn, and large matrices are filled chunk by chunk
with the same bytes whatever the chunk schedule.

Nothing here computes a column norm, a sampling density, a Gram matrix or a
solve: the only arithmetic is drawing the inputs and forming ``A x*`` for b.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import os

import numpy as np

# stream ids (fixed; changing one changes the inputs of every test and bench)
_S_A, _S_COLS, _S_SCALE, _S_XSTAR, _S_NOISE, _S_XT, _S_V, _S_HEAVY, _S_EDGES, _S_W = range(10)

_CHUNK_ROWS = 1 << 16


def _rng(seed: int, stream: int, chunk: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), stream, chunk])))


@dataclasses.dataclass
class Problem:
    """One least-squares instance ``min ||Ax - b||``.

    fmt:      "dense" (A is an m x n C-contiguous array) or "csr".
    A:        dense array (float64 or float32), or None for CSR.
    row_ptr:  int64[m+1] (CSR only)
    col_idx:  int32[nnz], sorted and unique within each row (CSR only)
    values:   float64 or float32 [nnz] (CSR only)
    b:        float64[m]
    x_star:   float64[n], the planted solution used to form b
    x_t:      float64[n] or None, target of the loss 0.5*||x - x_t||^2
    meta:     family name and generation parameters
    """

    fmt: str
    m: int
    n: int
    b: np.ndarray
    x_star: np.ndarray
    A: Optional[np.ndarray] = None
    row_ptr: Optional[np.ndarray] = None
    col_idx: Optional[np.ndarray] = None
    values: Optional[np.ndarray] = None
    x_t: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.values.shape[0]) if self.fmt == "csr" else self.m * self.n

    @property
    def dtype(self):
        return (self.values if self.fmt == "csr" else self.A).dtype

    def dense(self) -> np.ndarray:
        """A as a dense float64 array (small problems only)."""
        if self.fmt == "dense":
            return np.asarray(self.A, dtype=np.float64)
        out = np.zeros((self.m, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        out[rows, self.col_idx] = self.values
        return out


# ----------------------------------------------------------------------------
# helpers that only apply A to the planted x* (input construction)


def _dense_times(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    out = np.empty(A.shape[0], dtype=np.float64)

    def fill(c, r0, r1):
        out[r0:r1] = A[r0:r1].astype(np.float64) @ x

    _chunks(A.shape[0], fill)
    return out


def _csr_times(row_ptr, col_idx, values, x) -> np.ndarray:
    m = row_ptr.shape[0] - 1
    prod = values.astype(np.float64) * x[col_idx]
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    return np.bincount(rows, weights=prod, minlength=m)


def _finish(p: Problem, noise: float, seed: int, with_target: bool) -> Problem:
    ax = _dense_times(p.A, p.x_star) if p.fmt == "dense" else _csr_times(p.row_ptr, p.col_idx, p.values, p.x_star)
    p.b = ax + noise * _rng(seed, _S_NOISE).standard_normal(p.m)
    if with_target:
        p.x_t = _rng(seed, _S_XT).standard_normal(p.n)
    return p


def _chunks(m: int, fill) -> None:
    """Runs fill(c, r0, r1) over the row chunks of an m-row array on a few
    threads; every chunk has its own random stream, so the result does not
    depend on the order."""
    jobs = [(c, r0, min(m, r0 + _CHUNK_ROWS)) for c, r0 in enumerate(range(0, m, _CHUNK_ROWS))]
    if len(jobs) < 4:
        for j in jobs:
            fill(*j)
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda j: fill(*j), jobs))


def _fill_normal(m: int, n: int, seed: int, stream: int, dtype) -> np.ndarray:
    A = np.empty((m, n), dtype=dtype)

    def fill(c, r0, r1):
        A[r0:r1] = _rng(seed, stream, c).standard_normal((r1 - r0, n), dtype=np.float64).astype(dtype)

    _chunks(m, fill)
    return A


# ----------------------------------------------------------------------------
# the five families


def gaussian_dense(m: int, n: int, seed: int = 0, noise: float = 1e-4, dtype=np.float64) -> Problem:
    """Dense Gaussian family (Section 5.1): a_ij ~ N(0,1), x* ~ N(0,1)."""
    A = _fill_normal(m, n, seed, _S_A, dtype)
    x = _rng(seed, _S_XSTAR).standard_normal(n)
    p = Problem("dense", m, n, b=None, x_star=x, A=A,
                meta=dict(family="gaussian", m=m, n=n, seed=seed, noise=noise))
    return _finish(p, noise, seed, with_target=False)


def _distinct_sorted_cols(m: int, n: int, k: int, seed: int) -> np.ndarray:
    """k distinct uniform columns per row, ascending (redraw rows with repeats)."""
    cols = np.empty((m, k), dtype=np.int64)
    for c, r0 in enumerate(range(0, m, _CHUNK_ROWS)):
        r1 = min(m, r0 + _CHUNK_ROWS)
        g = _rng(seed, _S_COLS, c)
        blk = np.sort(g.integers(0, n, size=(r1 - r0, k)), axis=1)
        while True:
            bad = np.nonzero((np.diff(blk, axis=1) == 0).any(axis=1))[0]
            if bad.size == 0:
                break
            blk[bad] = np.sort(g.integers(0, n, size=(bad.size, k)), axis=1)
        cols[r0:r1] = blk
    return cols


def sparse_rowscaled(m: int, n: int, k: int = 10, seed: int = 0, noise: float = 1e-6,
                     log10_range: float = 3.0, dtype=np.float64) -> Problem:
    """Sparse random family standing in for Section 5.3's 'sprand' matrices.

    k distinct uniform columns per row, values N(0,1), row i scaled by
    10**U(-log10_range, log10_range), which makes the row norms (and hence the
    sampling density) spread over 2*log10_range decades.
    """
    if k > n:
        raise ValueError("k > n")
    cols = _distinct_sorted_cols(m, n, k, seed)
    vals = np.empty((m, k), dtype=np.float64)
    for c, r0 in enumerate(range(0, m, _CHUNK_ROWS)):
        r1 = min(m, r0 + _CHUNK_ROWS)
        vals[r0:r1] = _rng(seed, _S_A, c).standard_normal((r1 - r0, k))
    scale = 10.0 ** _rng(seed, _S_SCALE).uniform(-log10_range, log10_range, size=m)
    vals *= scale[:, None]
    row_ptr = np.arange(0, (m + 1) * k, k, dtype=np.int64)
    x = _rng(seed, _S_XSTAR).standard_normal(n)
    p = Problem("csr", m, n, b=None, x_star=x, row_ptr=row_ptr,
                col_idx=cols.reshape(-1).astype(np.int32), values=vals.reshape(-1).astype(dtype),
                meta=dict(family="sparse_rowscaled", m=m, n=n, k=k, seed=seed, noise=noise,
                          log10_range=log10_range))
    return _finish(p, noise, seed, with_target=False)


def udv_dense(m: int, n: int, seed: int = 0, noise: float = 1e-8, sigma_min: float = 1e-6,
              spacing: str = "log", dtype=np.float64) -> Problem:
    """UDV family (Section 5.4): A = U diag(sigma) V^T.

    U: Q factor of a Gaussian m x n matrix; V: Q factor of a Gaussian n x n
    matrix. sigma runs from 1 down to sigma_min, log-spaced ("log") or
    linearly spaced as in the paper's diag[1, 1+(c-1)/n, ..., c] ("linear").
    """
    G = _fill_normal(m, n, seed, _S_A, np.float64)
    U, _ = np.linalg.qr(G)
    del G
    V, _ = np.linalg.qr(_rng(seed, _S_V).standard_normal((n, n)))
    if spacing == "log":
        sig = 10.0 ** (np.log10(sigma_min) * np.arange(n) / max(n - 1, 1))
    elif spacing == "linear":
        sig = np.linspace(1.0, sigma_min, n)
    else:
        raise ValueError(spacing)
    A = np.ascontiguousarray(((U * sig[None, :]) @ V.T).astype(dtype))
    x = _rng(seed, _S_XSTAR).standard_normal(n)
    p = Problem("dense", m, n, b=None, x_star=x, A=A,
                meta=dict(family="udv", m=m, n=n, seed=seed, noise=noise, sigma_min=sigma_min,
                          spacing=spacing))
    return _finish(p, noise, seed, with_target=False)


def er_incidence(nv: int, ne: int, seed: int = 0, noise: float = 1e-6, dtype=np.float64,
                 require_connected: bool = True) -> Problem:
    """Weighted incidence matrix of an Erdos-Renyi graph (stands in for Section 5.5).

    ne distinct undirected edges without loops, drawn uniformly; edge (u, v) with
    u < v becomes the row w*(e_u - e_v), w = exp(N(0,1)); rows are ordered by
    (u, v). The column of vertex 0 is dropped so that A has full column rank
    (n = nv - 1); the rows of edges at vertex 0 keep one entry.
    """
    if ne > nv * (nv - 1) // 2:
        raise ValueError("too many edges")
    g = _rng(seed, _S_EDGES)
    keys = np.empty(0, dtype=np.int64)
    while keys.size < ne:
        need = ne - keys.size
        u = g.integers(0, nv, size=need + need // 8 + 16)
        v = g.integers(0, nv, size=u.size)
        ok = u != v
        lo, hi = np.minimum(u, v)[ok], np.maximum(u, v)[ok]
        new = lo * nv + hi
        # keep first occurrences in draw order, then top up
        allk = np.concatenate([keys, new])
        _, first = np.unique(allk, return_index=True)
        keys = allk[np.sort(first)][:ne]
    keys = np.sort(keys)
    u, v = keys // nv, keys % nv
    deg = np.bincount(u, minlength=nv) + np.bincount(v, minlength=nv)
    if (deg == 0).any():
        raise ValueError("isolated vertex; draw more edges")
    if require_connected:
        import scipy.sparse as sp
        from scipy.sparse.csgraph import connected_components
        G = sp.coo_matrix((np.ones(ne), (u, v)), shape=(nv, nv))
        ncomp, _ = connected_components(G, directed=False)
        if ncomp != 1:
            raise ValueError("graph not connected")
    w = np.exp(_rng(seed, _S_W).standard_normal(ne))
    at0 = u == 0
    cnt = np.where(at0, 1, 2).astype(np.int64)
    row_ptr = np.zeros(ne + 1, dtype=np.int64)
    np.cumsum(cnt, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    start = row_ptr[:-1]
    # rows with both ends kept: (u-1, +w), (v-1, -w); rows at vertex 0: (v-1, -w)
    two = ~at0
    col[start[two]] = (u[two] - 1)
    val[start[two]] = w[two]
    col[start[two] + 1] = (v[two] - 1)
    val[start[two] + 1] = -w[two]
    col[start[at0]] = (v[at0] - 1)
    val[start[at0]] = -w[at0]
    n = nv - 1
    x = _rng(seed, _S_XSTAR).standard_normal(n)
    p = Problem("csr", ne, n, b=None, x_star=x, row_ptr=row_ptr, col_idx=col, values=val.astype(dtype),
                meta=dict(family="er_incidence", nv=nv, ne=ne, seed=seed, noise=noise))
    return _finish(p, noise, seed, with_target=True)


def _chung_lu_edges(nv: int, beta: float, d: float, i0: int, g: np.random.Generator):
    """Edges (i, j), i < j, of a random graph with expected degrees following a
    power law (Section 5.5): w_i = c (i0 + i)^(-1/(beta-1)) for i = 0..nv-1,
    c = (beta-2)/(beta-1) * d * nv^(-1/(beta-1)), and each pair joined with
    probability min(1, w_i w_j / sum(w)). Pairs are drawn row by row of the
    upper triangle, one uniform per pair."""
    ex = -1.0 / (beta - 1.0)
    c = (beta - 2.0) / (beta - 1.0) * d * float(nv) ** ex
    w = c * np.arange(i0, i0 + nv, dtype=np.float64) ** ex
    rho = 1.0 / w.sum()
    us, vs = [], []
    for i in range(nv - 1):
        p = np.minimum(1.0, w[i] * w[i + 1:] * rho)
        j = np.nonzero(g.random(nv - 1 - i) < p)[0] + (i + 1)
        us.append(np.full(j.size, i, dtype=np.int64))
        vs.append(j.astype(np.int64))
    return np.concatenate(us), np.concatenate(vs)


def powerlaw_laplacian(n0: int, seed: int = 0, noise: float = 1e-6, i0: int = 11, overlap: int = 5,
                       sparse_graph=(5.0, 30.0), dense_graph=(8.0, None), dtype=np.float64) -> Problem:
    """Incidence matrix of two glued power-law random graphs, not grounded
    (Section 5.5's random graph Laplacian workload).

    B1: a sparse, ill-conditioned graph on n0 vertices (beta = 5, average
    degree parameter d = 30); B2: a dense, well-conditioned one on n0 vertices
    (beta = 8, d = 5 n0); both with i0 = 11. B2's vertex k becomes vertex
    n0 - overlap + k, so the two graphs share `overlap` vertices; B1's rows
    come first, then B2's, each in (i, j) order, as (+1 at i, -1 at j).
    Vertices without edges are removed (columns renumbered in order). No
    column is dropped: A^T A is a graph Laplacian, singular with the constant
    vectors of the connected components as its null space, and the least
    squares problem is consistent in the normal equations.
    """
    b1, d1 = sparse_graph
    b2, d2 = dense_graph
    if d2 is None:
        d2 = 5.0 * n0
    u1, v1 = _chung_lu_edges(n0, b1, d1, i0, _rng(seed, _S_EDGES, 0))
    u2, v2 = _chung_lu_edges(n0, b2, d2, i0, _rng(seed, _S_EDGES, 1))
    shift = n0 - overlap
    u = np.concatenate([u1, u2 + shift])
    v = np.concatenate([v1, v2 + shift])
    nv = 2 * n0 - overlap
    used = np.zeros(nv, dtype=bool)
    used[u] = True
    used[v] = True
    newid = np.cumsum(used) - 1
    u, v = newid[u], newid[v]
    n = int(used.sum())
    m = int(u.size)
    row_ptr = np.arange(0, 2 * m + 1, 2, dtype=np.int64)
    col = np.empty(2 * m, dtype=np.int32)
    val = np.empty(2 * m, dtype=np.float64)
    col[0::2], col[1::2] = u, v
    val[0::2], val[1::2] = 1.0, -1.0
    x = _rng(seed, _S_XSTAR).standard_normal(n)
    p = Problem("csr", m, n, b=None, x_star=x, row_ptr=row_ptr, col_idx=col, values=val.astype(dtype),
                meta=dict(family="powerlaw_laplacian", n0=n0, seed=seed, noise=noise, i0=i0, overlap=overlap,
                          sparse_graph=(b1, d1), dense_graph=(b2, d2), edges_sparse=int(u1.size),
                          edges_dense=int(u2.size)))
    return _finish(p, noise, seed, with_target=True)


def semi_gaussian_dense(m: int, n: int, seed: int = 0, noise: float = 1e-6, small: float = 1e-4,
                        heavy_frac: float = 0.01, heavy_scale: float = 1e3, dtype=np.float32) -> Problem:
    """Column-scaled dense family with heavy rows (stands in for Section 5.2).

    Columns [0, n/2) are N(0,1), columns [n/2, n) are small*N(0,1); a uniform
    random heavy_frac of the rows is multiplied by heavy_scale. The heavy rows
    make the sampling density strongly non-uniform (a coherent-like matrix).
    """
    A = np.empty((m, n), dtype=dtype)
    h = n // 2

    def fill(c, r0, r1):
        blk = _rng(seed, _S_A, c).standard_normal((r1 - r0, n))
        blk[:, h:] *= small
        A[r0:r1] = blk.astype(dtype)

    _chunks(m, fill)
    nh = int(round(heavy_frac * m))
    heavy = np.sort(_rng(seed, _S_HEAVY).choice(m, size=nh, replace=False))
    for r0 in range(0, nh, 4096):
        rows = heavy[r0:r0 + 4096]
        A[rows] = (A[rows].astype(np.float64) * heavy_scale).astype(dtype)
    x = _rng(seed, _S_XSTAR).standard_normal(n)
    p = Problem("dense", m, n, b=None, x_star=x, A=A,
                meta=dict(family="semi_gaussian", m=m, n=n, seed=seed, noise=noise, small=small,
                          heavy_frac=heavy_frac, heavy_scale=heavy_scale, heavy_rows=nh))
    return _finish(p, noise, seed, with_target=True)


# ----------------------------------------------------------------------------
# tiny structured fixtures from Section 3.1


def coherent_identity(m: int, n: int, seed: int = 0) -> Problem:
    """Z = [I_n; 0] (the coherent example of Section 3.1); b ~ N(0,1)."""
    A = np.zeros((m, n))
    A[np.arange(n), np.arange(n)] = 1.0
    b = _rng(seed, _S_NOISE).standard_normal(m)
    return Problem("dense", m, n, b=b, x_star=b[:n].copy(), A=A, meta=dict(family="coherent", m=m, n=n))


def semi_coherent_block(m: int, n: int, seed: int = 0) -> Problem:
    """Y = [X 0; 0 I_{n/2}] with Gaussian X (the semi-coherent example of Section 3.1)."""
    h = n // 2
    A = np.zeros((m, n))
    A[: m - (n - h), :h] = _rng(seed, _S_A).standard_normal((m - (n - h), h))
    A[m - (n - h):, h:] = np.eye(n - h)
    x = _rng(seed, _S_XSTAR).standard_normal(n)
    p = Problem("dense", m, n, b=None, x_star=x, A=A, meta=dict(family="semi_coherent", m=m, n=n))
    return _finish(p, 1e-6, seed, with_target=False)


# ----------------------------------------------------------------------------
# named workloads


CONFIG_NAMES = ("gaussian", "sparse", "udv", "graph", "semigauss", "laplacian")

# full sizes of the five workloads: (generator, kwargs, solver settings)
_FULL = {
    "gaussian": (gaussian_dense, dict(m=20000, n=100, noise=1e-4), dict(C=4.0, sweeps=1)),
    "sparse": (sparse_rowscaled, dict(m=1_000_000, n=10_000, k=10, noise=1e-6), dict(C=4.0, sweeps=2)),
    "udv": (udv_dense, dict(m=200_000, n=1000, noise=1e-8), dict(C=4.0, sweeps=5)),
    "graph": (er_incidence, dict(nv=100_000, ne=2_000_000, noise=1e-6), dict(C=4.0, sweeps=5)),
    "semigauss": (semi_gaussian_dense, dict(m=2_000_000, n=2000, noise=1e-6), dict(C=4.0, sweeps=5)),
    "laplacian": (powerlaw_laplacian, dict(n0=2000, noise=1e-6), dict(C=4.0, sweeps=5)),
}

# reduced sizes with the same structure, for parity tests the oracle finishes in seconds
_SMALL = {
    "gaussian": dict(m=4000, n=64),
    "sparse": dict(m=40_000, n=600, k=10),
    "udv": dict(m=8000, n=160),
    "graph": dict(nv=3000, ne=30_000),
    "semigauss": dict(m=20_000, n=200),
    "laplacian": dict(n0=100),
}


def make_config(name: str, seed: int = 0, scale: str = "full", **override):
    """Return (Problem, solver settings dict) for a named workload.

    scale="full" gives the workload at its stated size; scale="small" keeps the
    family, distributions and structure at a size the oracle handles quickly.
    """
    gen, kw, solver = _FULL[name]
    kw = dict(kw)
    if scale == "small":
        kw.update(_SMALL[name])
    elif scale != "full":
        raise ValueError(scale)
    kw.update(override)
    return gen(seed=seed, **kw), dict(solver)

