"""Seeded synthetic inputs shaped like the paper's SpMM workloads.

This module only draws sparsity patterns, values and dense operands.  It
holds none of the SpMM method's arithmetic, so both the CPU oracle and the
HIP path can consume its arrays without sharing any code with each other.

Every generator draws from ``numpy.random.default_rng([seed, stream])`` with
the streams

    0 = sparsity pattern, 1 = values of A, 2 = dense B (or X),
    3 = the upstream gradient G (= dC), 4 = auxiliary choices (BFS root).

A sparse matrix is returned as a ``Csr`` with int32 ``row_ptr``/``col_idx``
(canonical: columns ascending within a row, no duplicates) and float64
``vals``.  The paper evaluates on SuiteSparse and on DGL graphs (Sec. 4.1,
Table 2, Table 4); neither is available here, so these generators stand in
for them with the shapes, sizes and row-length statistics described in the
workload recipes below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Csr", "rng", "csr_from_coo", "config1", "config2", "config3", "config4",
    "config4_fd_subgraph", "config5", "config5_spec", "powerlaw_degrees",
    "dense", "random_csr",
]

PATTERN, AVALS, DENSE, GRAD, AUX = 0, 1, 2, 3, 4


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


@dataclass
class Csr:
    m: int
    k: int
    row_ptr: np.ndarray  # int32 [m+1]
    col_idx: np.ndarray  # int32 [nnz]
    vals: np.ndarray     # float64 [nnz]
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64)."""
        return np.repeat(np.arange(self.m, dtype=np.int64), np.diff(self.row_ptr))

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.m, self.k))


def csr_from_coo(m: int, k: int, rows: np.ndarray, cols: np.ndarray,
                 vals: np.ndarray | None = None) -> Csr:
    """Sort (row, col) pairs into canonical CSR; pairs must be distinct."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * k + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate (row, col) pairs")
    r = key // k
    c = key % k
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    v = np.zeros(key.size) if vals is None else np.asarray(vals, dtype=np.float64)[order]
    return Csr(m, k, row_ptr.astype(np.int32), c.astype(np.int32), v)


def dense(seed: int, stream: int, rows: int, cols: int, dist: str = "normal") -> np.ndarray:
    g = rng(seed, stream)
    if dist == "normal":
        return g.standard_normal((rows, cols))
    if dist == "uniform":
        return g.uniform(-1.0, 1.0, (rows, cols))
    raise ValueError(dist)


# ---------------------------------------------------------------------------
# Config 1: 4096 x 4096, exactly 10 distinct uniform columns per row, FP64.
# ---------------------------------------------------------------------------
def config1(seed: int = 0, m: int = 4096, per_row: int = 10, n: int = 32):
    g = rng(seed, PATTERN)
    cols = np.stack([g.choice(m, per_row, replace=False) for _ in range(m)])
    cols = np.sort(cols, axis=1)
    rows = np.repeat(np.arange(m), per_row)
    a = csr_from_coo(m, m, rows, cols.reshape(-1))
    a.vals = rng(seed, AVALS).uniform(-1.0, 1.0, a.nnz)
    a.meta = {"name": "config1_uniform10", "seed": seed}
    b = dense(seed, DENSE, m, n, "uniform")
    return a, b


# ---------------------------------------------------------------------------
# Config 2: block stencil.  128 x 128 grid, 4 DOFs per node, 9-point
# neighbourhood (non-periodic), every coupling a dense 4x4 block; plus 5 %
# distinct uniformly scattered extra positions.  Values N(0,1).
# ---------------------------------------------------------------------------
def stencil_pattern(grid: int = 128, dofs: int = 4):
    nodes = grid * grid
    y, x = np.divmod(np.arange(nodes, dtype=np.int64), grid)
    src, dst = [], []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ny, nx = y + dy, x + dx
            ok = (ny >= 0) & (ny < grid) & (nx >= 0) & (nx < grid)
            src.append(np.nonzero(ok)[0])
            dst.append((ny * grid + nx)[ok])
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    d = np.arange(dofs, dtype=np.int64)
    rows = (src[:, None, None] * dofs + d[None, :, None]).repeat(dofs, axis=2)
    cols = (dst[:, None, None] * dofs + d[None, None, :]).repeat(dofs, axis=1)
    return nodes * dofs, rows.reshape(-1), cols.reshape(-1)


def config2(seed: int = 0, grid: int = 128, dofs: int = 4, extra_frac: float = 0.05,
            n: int = 128):
    m, rows, cols = stencil_pattern(grid, dofs)
    base = rows * m + cols
    n_extra = int(round(extra_frac * base.size))
    g = rng(seed, PATTERN)
    taken = np.sort(base)
    extra = np.empty(0, dtype=np.int64)
    while extra.size < n_extra:
        cand = g.integers(0, m * m, size=2 * (n_extra - extra.size) + 16, dtype=np.int64)
        cand = cand[~np.isin(cand, taken)]
        cand = cand[~np.isin(cand, extra)]
        _, first = np.unique(cand, return_index=True)
        cand = cand[np.sort(first)]
        extra = np.concatenate([extra, cand[: n_extra - extra.size]])
    allk = np.concatenate([base, extra])
    a = csr_from_coo(m, m, allk // m, allk % m)
    a.vals = rng(seed, AVALS).standard_normal(a.nnz)
    a.meta = {"name": f"config2_stencil{grid}x{grid}x{dofs}", "seed": seed,
              "stencil_nnz": int(base.size), "extra_nnz": int(n_extra)}
    b = dense(seed, DENSE, m, n, "normal")
    return a, b


# ---------------------------------------------------------------------------
# Power-law degrees: continuous law pdf ~ x^-alpha on [x_min, x_max], rounded
# to integers and clipped to [1, x_max]; x_min is solved so the mean of the
# rounded degrees equals `mean`.
# ---------------------------------------------------------------------------
def _pl_cdf(x, xmin, xmax, alpha):
    a1 = 1.0 - alpha
    x = np.clip(x, xmin, xmax)
    return (xmin ** a1 - x ** a1) / (xmin ** a1 - xmax ** a1)


def _rounded_mean(xmin, xmax, alpha):
    d = np.arange(1, int(xmax) + 1, dtype=np.float64)
    p = _pl_cdf(d + 0.5, xmin, xmax, alpha) - _pl_cdf(d - 0.5, xmin, xmax, alpha)
    return float((d * p).sum())


def solve_xmin(mean: float, xmax: float, alpha: float = 2.1) -> float:
    lo, hi = 0.5, float(xmax) * (1.0 - 1e-9)
    if _rounded_mean(hi, xmax, alpha) < mean:
        return hi
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if _rounded_mean(mid, xmax, alpha) < mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def powerlaw_degrees(g: np.random.Generator, m: int, mean: float, dmax: int,
                     alpha: float = 2.1) -> np.ndarray:
    xmin = solve_xmin(mean, float(dmax), alpha)
    a1 = 1.0 - alpha
    u = g.random(m)
    x = (xmin ** a1 - u * (xmin ** a1 - float(dmax) ** a1)) ** (1.0 / a1)
    d = np.clip(np.rint(x), 1, dmax).astype(np.int64)
    d[np.argmax(d)] = dmax
    return d


def _preferential_columns(g, deg, k, weights):
    """For each row i draw deg[i] distinct columns with P(j) ~ weights[j]."""
    m = deg.size
    cdf = np.cumsum(weights, dtype=np.float64)
    cdf /= cdf[-1]
    rows = np.repeat(np.arange(m, dtype=np.int64), deg)
    cols = np.searchsorted(cdf, g.random(rows.size), side="right").astype(np.int64)
    np.minimum(cols, k - 1, out=cols)
    while True:
        key = rows * k + cols
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        idx = order[dup]
        new = np.searchsorted(cdf, g.random(idx.size), side="right")
        cols[idx] = np.minimum(new, k - 1)
    return rows, cols


# ---------------------------------------------------------------------------
# Config 3: 2^20 x 2^20 power law, exponent 2.1, mean 16, max 20000, columns
# drawn preferentially by degree without replacement; a_ij = 1/sqrt(d_i d_j).
# ---------------------------------------------------------------------------
def config3(seed: int = 0, m: int = 1 << 20, mean: float = 16.0, dmax: int = 20000,
            n: int = 64):
    g = rng(seed, PATTERN)
    deg = powerlaw_degrees(g, m, mean, dmax)
    rows, cols = _preferential_columns(g, deg, m, deg.astype(np.float64))
    a = csr_from_coo(m, m, rows, cols)
    d = np.diff(a.row_ptr).astype(np.float64)
    r = a.rows()
    a.vals = 1.0 / np.sqrt(d[r] * d[a.col_idx])
    a.meta = {"name": f"config3_powerlaw{m}", "seed": seed}
    b = dense(seed, DENSE, m, n, "normal")
    return a, b


# ---------------------------------------------------------------------------
# Config 4: GCN graph.  Chung-Lu graph on 232,965 nodes with power-law expected
# degrees (exponent 2.1, mean 50, capped at sqrt(sum w)); symmetrised, self
# loops added, weights D^-1/2 (A+I) D^-1/2.
# ---------------------------------------------------------------------------
def _capped_pl_mean(xmin, cap, alpha):
    # E[min(X, cap)] for X ~ x^-alpha on [xmin, inf)
    a = alpha
    tail = (cap / xmin) ** (1.0 - a)
    body = (a - 1.0) / (a - 2.0) * xmin * (1.0 - (cap / xmin) ** (2.0 - a))
    return body + cap * tail


def config4(seed: int = 0, nodes: int = 232_965, mean: float = 50.0, n: int = 128,
            alpha: float = 2.1):
    g = rng(seed, PATTERN)
    cap = math.sqrt(nodes * mean)
    lo, hi = 1.0, mean
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _capped_pl_mean(mid, cap, alpha) < mean:
            lo = mid
        else:
            hi = mid
    xmin = 0.5 * (lo + hi)
    u = g.random(nodes)
    w = np.minimum(xmin * (1.0 - u) ** (-1.0 / (alpha - 1.0)), cap)
    n_edges = int(round(w.sum() / 2.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    s = np.minimum(np.searchsorted(cdf, g.random(n_edges), side="right"), nodes - 1)
    t = np.minimum(np.searchsorted(cdf, g.random(n_edges), side="right"), nodes - 1)
    keep = s != t
    s, t = s[keep], t[keep]
    r = np.concatenate([s, t, np.arange(nodes)])
    c = np.concatenate([t, s, np.arange(nodes)])
    key = np.unique(r.astype(np.int64) * nodes + c)
    a = csr_from_coo(nodes, nodes, key // nodes, key % nodes)
    deg = np.diff(a.row_ptr).astype(np.float64)  # rowsum(A + I), A is 0/1
    rr = a.rows()
    a.vals = 1.0 / np.sqrt(deg[rr] * deg[a.col_idx])
    a.meta = {"name": f"config4_gcn{nodes}", "seed": seed, "xmin": xmin, "cap": cap}
    x = dense(seed, DENSE, nodes, n, "normal")
    return a, x


def config4_fd_subgraph(a: Csr, size: int = 512, seed: int = 0) -> Csr:
    """Induced submatrix on a BFS ball of `size` nodes (ascending-id
    neighbour order) from a seeded root; no renormalisation."""
    g = rng(seed, AUX)
    start = int(g.integers(a.m))
    seen = {start: 0}
    order = [start]
    head = 0
    while len(order) < size and head < len(order):
        u = order[head]
        head += 1
        for v in a.col_idx[a.row_ptr[u]:a.row_ptr[u + 1]]:
            v = int(v)
            if v not in seen:
                seen[v] = len(order)
                order.append(v)
                if len(order) == size:
                    break
    nodes = np.array(sorted(order), dtype=np.int64)
    pos = -np.ones(a.m, dtype=np.int64)
    pos[nodes] = np.arange(nodes.size)
    rs, cs, vs = [], [], []
    for li, u in enumerate(nodes):
        lo, hi = a.row_ptr[u], a.row_ptr[u + 1]
        cc = pos[a.col_idx[lo:hi]]
        ok = cc >= 0
        rs.append(np.full(int(ok.sum()), li))
        cs.append(cc[ok])
        vs.append(a.vals[lo:hi][ok])
    sub = csr_from_coo(nodes.size, nodes.size, np.concatenate(rs), np.concatenate(cs),
                       np.concatenate(vs))
    sub.meta = {"name": "config4_bfs512", "root": start}
    return sub


# ---------------------------------------------------------------------------
# Config 5: structure sweep, 64 matrices.
# ---------------------------------------------------------------------------
CLASSES = ("uniform", "banded", "blockdiag", "powerlaw")
BLOCK_SIZES = (2, 4, 8, 16)
SWEEP_N = (16, 32, 64, 128, 256)


def config5_spec(i: int, max_rows: int = 500_000):
    g = rng(i, AUX)
    m = int(round(math.exp(g.uniform(math.log(1e3), math.log(max_rows)))))
    d = int(round(math.exp(g.uniform(math.log(2.0), math.log(200.0)))))
    cls = CLASSES[i % 4]
    spec = {"index": i, "class": cls, "m": m, "d": min(d, m)}
    if cls == "banded":
        spec["half_band"] = int(g.integers(1, 65))
    if cls == "blockdiag":
        spec["b"] = BLOCK_SIZES[(i // 4) % 4]
    return spec


def config5(i: int, max_rows: int = 500_000) -> Csr:
    spec = config5_spec(i, max_rows)
    m, d, cls = spec["m"], spec["d"], spec["class"]
    g = rng(i, PATTERN)
    if cls == "uniform":
        deg = np.full(m, d, dtype=np.int64)
        rows, cols = _preferential_columns(g, deg, m, np.ones(m))
    elif cls == "banded":
        hb = spec["half_band"]
        r = np.arange(m, dtype=np.int64)
        lo = np.maximum(r - hb, 0)
        hi = np.minimum(r + hb, m - 1)
        width = hi - lo + 1
        take = np.minimum(width, d)
        rows = np.repeat(r, take)
        # distinct offsets inside the band: rank of random keys
        maxw = 2 * hb + 1
        keys = g.random((m, maxw))
        keys[np.arange(maxw)[None, :] >= width[:, None]] = 2.0
        sel = np.argsort(keys, axis=1)
        mask = np.arange(maxw)[None, :] < take[:, None]
        cols = (lo[:, None] + sel)[mask]
    elif cls == "blockdiag":
        b = spec["b"]
        nb = (m + b - 1) // b
        extra = max(0, (d + b - 1) // b - 1)
        extra = min(extra, nb - 1)
        brow, bcol = [np.arange(nb)], [np.arange(nb)]
        if extra > 0:
            # extra distinct off-diagonal block columns per block row
            keys = g.random((nb, nb)) if nb <= 4096 else None
            if keys is not None:
                keys[np.arange(nb), np.arange(nb)] = 2.0
                off = np.argsort(keys, axis=1)[:, :extra]
            else:
                off = np.empty((nb, extra), dtype=np.int64)
                for q in range(nb):
                    c = g.choice(nb - 1, extra, replace=False)
                    off[q] = c + (c >= q)
            brow.append(np.repeat(np.arange(nb), extra))
            bcol.append(off.reshape(-1))
        brow = np.concatenate(brow)
        bcol = np.concatenate(bcol)
        ii, jj = np.meshgrid(np.arange(b), np.arange(b), indexing="ij")
        rows = (brow[:, None] * b + ii.reshape(-1)[None, :]).reshape(-1)
        cols = (bcol[:, None] * b + jj.reshape(-1)[None, :]).reshape(-1)
        ok = (rows < m) & (cols < m)
        rows, cols = rows[ok], cols[ok]
    else:  # powerlaw
        dmax = int(max(1, min(20000, m // 4)))
        deg = powerlaw_degrees(g, m, min(float(d), dmax * 0.5), dmax)
        deg = np.minimum(deg, m)
        rows, cols = _preferential_columns(g, deg, m, deg.astype(np.float64))
    a = csr_from_coo(m, m, rows, cols)
    a.vals = rng(i, AVALS).uniform(-1.0, 1.0, a.nnz)
    a.meta = dict(spec, name=f"config5_{i:02d}_{cls}")
    return a


def random_csr(seed: int, m: int, k: int, density: float, stream: int = PATTERN,
               dist: str = "uniform") -> Csr:
    """Small uniform random pattern for edge-case tests."""
    g = rng(seed, stream)
    mask = g.random((m, k)) < density
    r, c = np.nonzero(mask)
    a = csr_from_coo(m, k, r, c)
    if dist == "uniform":
        a.vals = rng(seed, AVALS).uniform(-1.0, 1.0, a.nnz)
    elif dist == "int":
        a.vals = rng(seed, AVALS).integers(-4, 5, a.nnz).astype(np.float64)
    else:
        raise ValueError(dist)
    return a
