"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names what it pins the oracle to; none of them re-calls the oracle
to produce its own expectation.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle
from tests.conftest import read_golden


def _dense(m, k, row_ptr, col, vals):
    A = np.zeros((m, k))
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    np.add.at(A, (rows, np.asarray(col)), np.asarray(vals))
    return A


def _rand_csr(seed, m, k, density, ints=False, dups=0, shuffle=False):
    g = np.random.default_rng(seed)
    mask = g.random((m, k)) < density
    r, c = np.nonzero(mask)
    if dups:
        pick = g.integers(0, max(1, r.size), dups) if r.size else np.zeros(0, int)
        r = np.concatenate([r, r[pick]])
        c = np.concatenate([c, c[pick]])
    order = np.lexsort((g.random(r.size) if shuffle else c, r))
    r, c = r[order], c[order]
    v = g.integers(-5, 6, r.size).astype(float) if ints else g.uniform(-1, 1, r.size)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp), c.astype(np.int32), v


# ---------------------------------------------------------------------------
# forward C = A B  (Sec. 2.1 inner-product definition)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_spmm_matches_dense_gemm_tiny(seed):
    """Pin: dense GEMM A_dense @ B (closed form) on tiny inputs."""
    g = np.random.default_rng(100 + seed)
    m, k, n = g.integers(1, 64, 3)
    rp, c, v = _rand_csr(seed, m, k, 0.2)
    B = g.standard_normal((k, n))
    C = oracle.spmm(m, k, rp, c, v, B)
    ref = _dense(m, k, rp, c, v) @ B
    assert oracle.rel_err(C, ref) <= 1e-14


def test_spmm_matches_scipy_config1():
    """Pin: scipy.sparse CSR @ dense (an independent library routine) on
    the 4096 x 4096, 10-per-row FP64 workload."""
    a, b = gen.config1()
    C = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b)
    ref = a.to_scipy() @ b
    assert oracle.rel_err(C, ref) <= 1e-14


def test_spmm_worked_example(golden):
    """Pin: the hand-worked 6 x 5 example (Sec. 2.1 definition)."""
    g = read_golden("alg1_example.txt")
    m, k, n = int(g["m"][0]), int(g["k"][0]), int(g["n"][0])
    rp = np.array(g["row_ptr"], dtype=np.int64)
    c = np.array(g["col_idx"], dtype=np.int32)
    v = np.array(g["vals"], dtype=float)
    B = np.array(g["B"], dtype=float).reshape(k, n)
    C = oracle.spmm(m, k, rp, c, v, B)
    assert np.array_equal(C, np.array(g["C"], dtype=float).reshape(m, n))


def test_identity_and_permutation_bitwise():
    """Pin: A = I gives C = B and A = P gives C = P B, bit for bit."""
    g = np.random.default_rng(7)
    m, n = 300, 17
    B = g.standard_normal((m, n))
    rp = np.arange(m + 1, dtype=np.int64)
    C = oracle.spmm(m, m, rp, np.arange(m, dtype=np.int32), np.ones(m), B)
    assert np.array_equal(C, B)
    p = g.permutation(m)
    C = oracle.spmm(m, m, rp, p.astype(np.int32), np.ones(m), B)
    assert np.array_equal(C, B[p])


def test_integer_valued_exact():
    """Pin: integer-valued A and B -- every partial sum is exact in FP64, so
    the result equals the exact integer product."""
    m, k, n = 200, 150, 33
    rp, c, v = _rand_csr(3, m, k, 0.1, ints=True)
    B = np.random.default_rng(4).integers(-7, 8, (k, n))
    C = oracle.spmm(m, k, rp, c, v, B.astype(float))
    A = _dense(m, k, rp, c, v).astype(np.int64)
    assert np.array_equal(C, (A @ B).astype(float))


def test_linearity_in_B():
    """Pin: A (a B1 + b B2) = a A B1 + b A B2 within rounding."""
    g = np.random.default_rng(9)
    m, k, n = 120, 90, 20
    rp, c, v = _rand_csr(5, m, k, 0.15)
    B1, B2 = g.standard_normal((k, n)), g.standard_normal((k, n))
    lhs = oracle.spmm(m, k, rp, c, v, 0.75 * B1 - 2.5 * B2)
    rhs = 0.75 * oracle.spmm(m, k, rp, c, v, B1) - 2.5 * oracle.spmm(m, k, rp, c, v, B2)
    assert oracle.rel_err(lhs, rhs) <= 1e-14


def test_row_permutation_equivariance_and_column_relabel():
    """Pin: (P A) B = P (A B) and (A P^T)(P B) = A B, bitwise (the stored
    order of each row is unchanged, so every sum is the same)."""
    g = np.random.default_rng(11)
    m, k, n = 80, 70, 9
    rp, c, v = _rand_csr(6, m, k, 0.2)
    B = g.standard_normal((k, n))
    C = oracle.spmm(m, k, rp, c, v, B)
    p = g.permutation(m)
    lens = np.diff(rp)[p]
    rp2 = np.concatenate([[0], np.cumsum(lens)])
    c2 = np.concatenate([c[rp[i]:rp[i + 1]] for i in p])
    v2 = np.concatenate([v[rp[i]:rp[i + 1]] for i in p])
    assert np.array_equal(oracle.spmm(m, k, rp2, c2, v2, B), C[p])
    q = g.permutation(k)             # new column q[j] holds old column j
    Bq = np.empty_like(B)
    Bq[q] = B
    assert np.array_equal(oracle.spmm(m, k, rp, q[c].astype(np.int32), v, Bq), C)


def test_duplicates_and_unsorted_rows_summed():
    """Pin: duplicated and unsorted entries contribute as a dense scatter-add
    (np.add.at) of the same triplets."""
    m, k, n = 64, 48, 5
    rp, c, v = _rand_csr(8, m, k, 0.2, dups=40, shuffle=True)
    B = np.random.default_rng(1).standard_normal((k, n))
    C = oracle.spmm(m, k, rp, c, v, B)
    assert oracle.rel_err(C, _dense(m, k, rp, c, v) @ B) <= 1e-14


def test_thread_count_independent_bitwise():
    a, b = gen.config1(m=1024)
    c1 = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b, nthreads=1)
    c8 = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b, nthreads=8)
    assert np.array_equal(c1, c8)
    g = np.random.default_rng(2).standard_normal(c1.shape)
    t1 = oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, g, nthreads=1)
    t8 = oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, g, nthreads=8)
    assert np.array_equal(t1, t8)


def test_empty_shapes():
    """Empty rows give zero rows; m = 0 and n = 0 are valid."""
    rp = np.zeros(5, dtype=np.int64)
    C = oracle.spmm(4, 3, rp, np.zeros(0, np.int32), np.zeros(0), np.ones((3, 2)))
    assert np.array_equal(C, np.zeros((4, 2)))
    assert oracle.spmm(0, 3, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0),
                       np.ones((3, 2))).shape == (0, 2)
    assert oracle.spmm(4, 3, rp, np.zeros(0, np.int32), np.zeros(0), np.ones((3, 0))).shape == (4, 0)


def test_invalid_csr_rejected():
    with pytest.raises(ValueError):
        oracle.spmm(2, 2, np.array([0, 1, 1]), np.array([5], np.int32), np.ones(1), np.ones((2, 1)))
    with pytest.raises(ValueError):
        oracle.spmm(2, 2, np.array([0, 2, 1]), np.array([0, 1], np.int32), np.ones(2), np.ones((2, 1)))


# ---------------------------------------------------------------------------
# backward: dB = A^T G (row scatter) and dA = SDDMM(G, B)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_spmm_t_dense_scipy_and_adjoint(seed):
    """Pins: dense A^T @ G, scipy A.T @ G, and the adjoint identity
    <A B, G> = <B, A^T G>."""
    g = np.random.default_rng(seed)
    m, k, n = 97, 61, 13
    rp, c, v = _rand_csr(20 + seed, m, k, 0.1, dups=5 * seed, shuffle=seed % 2 == 1)
    G = g.standard_normal((m, n))
    B = g.standard_normal((k, n))
    dB = oracle.spmm_t(m, k, rp, c, v, G)
    A = _dense(m, k, rp, c, v)
    assert oracle.rel_err(dB, A.T @ G) <= 1e-14
    S = sp.csr_matrix((v, c, rp), shape=(m, k))
    assert oracle.rel_err(dB, S.T @ G) <= 1e-14
    lhs = float(np.sum(oracle.spmm(m, k, rp, c, v, B) * G))
    rhs = float(np.sum(B * dB))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_spmm_t_integer_exact():
    m, k, n = 150, 120, 7
    rp, c, v = _rand_csr(31, m, k, 0.1, ints=True)
    G = np.random.default_rng(3).integers(-9, 10, (m, n))
    dB = oracle.spmm_t(m, k, rp, c, v, G.astype(float))
    A = _dense(m, k, rp, c, v).astype(np.int64)
    assert np.array_equal(dB, (A.T @ G).astype(float))


@pytest.mark.parametrize("seed", range(3))
def test_sddmm_dense_masked(seed):
    """Pin: dA[e] = ((G B^T) masked by the pattern)[row(e), col(e)], with
    every duplicate of a position receiving the same value."""
    g = np.random.default_rng(seed)
    m, k, n = 45, 38, 11
    rp, c, v = _rand_csr(40 + seed, m, k, 0.2, dups=7, shuffle=True)
    G = g.standard_normal((m, n))
    B = g.standard_normal((k, n))
    dA = oracle.sddmm(m, k, rp, c, G, B)
    full = G @ B.T
    rows = np.repeat(np.arange(m), np.diff(rp))
    assert oracle.rel_err(dA, full[rows, c]) <= 1e-14


def test_sddmm_is_gradient_of_bilinear_loss():
    """Pin: L(vals) = <A(vals) B, G> is linear in vals, so dL/dvals[e] is
    exactly L(e_e) -- the loss of the matrix holding 1 at entry e only."""
    g = np.random.default_rng(5)
    m, k, n = 20, 15, 6
    rp, c, v = _rand_csr(50, m, k, 0.25)
    G = g.standard_normal((m, n))
    B = g.standard_normal((k, n))
    dA = oracle.sddmm(m, k, rp, c, G, B)
    for e in range(0, c.size, 3):
        unit = np.zeros_like(v)
        unit[e] = 1.0
        L = float(np.sum(oracle.spmm(m, k, rp, c, unit, B) * G))
        assert abs(L - dA[e]) <= 1e-13 * max(1.0, abs(L))


def test_spmm_t_matches_spmm_of_explicit_transpose():
    """Pin: scipy's explicit transpose fed back through the forward oracle."""
    a, _ = gen.config1(m=512)
    g = np.random.default_rng(0).standard_normal((a.m, 8))
    T = a.to_scipy().T.tocsr()
    ref = oracle.spmm(T.shape[0], T.shape[1], T.indptr, T.indices.astype(np.int32), T.data, g)
    got = oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, g)
    assert oracle.rel_err(got, ref) <= 1e-14


# ---------------------------------------------------------------------------
# metric: the FLOP count 2 * nnz * N against Table 3
# ---------------------------------------------------------------------------
def test_flop_count_matches_table3():
    """Pin of the throughput convention: Eff * Power * Time equals about 100
    calls of 2 * nnz * 32 FLOPs on 19 of the 20 rows of Table 3, on both
    devices; m20 is the paper's own outlier."""
    rows = read_golden("table3_flops.txt")
    ok = {"a100": 0, "m4": 0}
    for mid, vals in rows.items():
        nnz = float(vals[0]) * 1e6
        per_call = 2.0 * nnz * 32 / 1e9
        for dev, off in (("a100", 1), ("m4", 4)):
            w, t, eff = (float(x) for x in vals[off:off + 3])
            ratio = eff * w * t / per_call
            if 90.0 <= ratio <= 110.0:
                ok[dev] += 1
            elif mid != "m20":
                pytest.fail(f"{mid} {dev}: ratio {ratio:.1f}")
    assert ok == {"a100": 19, "m4": 19}
