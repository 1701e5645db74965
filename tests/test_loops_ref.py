"""Pins of the CPU restatement of the format conversion (Alg. 1), the row
boundary (Eq. 1), the quadratic model (Eq. 2/3) and the FP16/BF16 storage
of A."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gen
from oracle import loops_ref as L
from tests.conftest import read_golden


def _ints(xs):
    return np.array(xs, dtype=np.int64)


def test_alg1_worked_example():
    """Pin: hand-worked instance of Alg. 1 (tests/golden/alg1_example.txt)."""
    g = read_golden("alg1_example.txt")
    m, br, rb = int(g["m"][0]), int(g["br"][0]), int(g["r_boundary"][0])
    f = L.convert_ref(m, _ints(g["row_ptr"]), _ints(g["col_idx"]),
                      np.array(g["vals"], float), rb, br)
    for key in ("csr_rows", "csr_ptr", "csr_col", "bcsr_rb", "blk_ptr", "blk_col"):
        assert np.array_equal(f[key], _ints(g[key])), key
    assert np.array_equal(f["csr_val"], np.array(g["csr_val"], float))
    assert np.array_equal(f["blk_val"].ravel(), np.array(g["blk_val"], float))
    nnz, nblk = L.rowblock_stats_ref(m, _ints(g["row_ptr"]), _ints(g["col_idx"]), br)
    assert np.array_equal(nnz, _ints(g["rb_nnz"]))
    assert np.array_equal(nblk, _ints(g["rb_nblk"]))


def test_alg1_boundary_must_align():
    """Reading: a boundary inside a row block would let a tile straddle both
    parts, so it is rejected."""
    with pytest.raises(ValueError):
        L.convert_ref(6, _ints([0, 1, 1, 1, 1, 1, 1]), _ints([0]), np.ones(1), 3, 2)


@pytest.mark.parametrize("seed", range(4))
def test_conversion_round_trip_and_conservation(seed):
    """Pins: expanding the hybrid format back to triplets gives A again for
    every boundary and every per-block assignment; stored entries are
    conserved (CSR entries + non-zero tile slots = nnz)."""
    a = gen.random_csr(seed, 53, 41, 0.15)
    trip = [(int(i), int(j), float(v)) for i, j, v in
            zip(a.rows(), a.col_idx, a.vals)]
    br = [2, 4, 8, 16][seed]
    nrb = (a.m + br - 1) // br
    cases = [q * br for q in range(nrb)] + [a.m]
    rng = np.random.default_rng(seed)
    for r_b in cases:
        f = L.convert_ref(a.m, a.row_ptr, a.col_idx, a.vals, r_b, br)
        assert L.to_coo_ref(a.m, f, br) == trip
        assert f["csr_col"].size + np.count_nonzero(f["blk_val"]) == a.nnz
    for _ in range(5):
        mask = rng.random(nrb) < 0.5
        f = L.convert_assign_ref(a.m, a.row_ptr, a.col_idx, a.vals, mask, br)
        assert L.to_coo_ref(a.m, f, br) == trip


def test_rowblock_stats_brute_force():
    """Pin: non-empty tiles per row block = non-zero columns of the dense
    br-row slab."""
    a = gen.random_csr(3, 70, 90, 0.05)
    D = a.to_scipy().toarray() != 0
    for br in (1, 4, 16):
        nnz, nblk = L.rowblock_stats_ref(a.m, a.row_ptr, a.col_idx, br)
        for q in range(nnz.size):
            slab = D[q * br:(q + 1) * br]
            assert nnz[q] == slab.sum()
            assert nblk[q] == slab.any(axis=0).sum()


def test_canonicalize_matches_scipy():
    """Pin: scipy's sum_duplicates (sorted indices, duplicates summed)."""
    g = np.random.default_rng(0)
    m, k = 30, 25
    r = g.integers(0, m, 300)
    c = g.integers(0, k, 300)
    order = np.argsort(r, kind="stable")
    r, c = r[order], c[order]
    v = g.standard_normal(300)
    rp = np.zeros(m + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    rp = np.cumsum(rp)
    ptr, col, val, canon = L.canonicalize_ref(m, k, rp, c, v)
    S = sp.csr_matrix((v, c, rp), shape=(m, k))
    S.sum_duplicates()
    assert np.array_equal(ptr, S.indptr) and np.array_equal(col, S.indices)
    assert np.allclose(val, S.data, rtol=1e-15, atol=1e-15)
    # every original entry maps to the canonical slot of its (row, col)
    rows_c = np.repeat(np.arange(m), np.diff(ptr))
    assert np.array_equal(rows_c[canon], r) and np.array_equal(col[canon], c)


def test_transpose_ref_matches_scipy_and_is_an_involution():
    a = gen.random_csr(5, 40, 33, 0.1)
    ptr, col, val, perm = L.transpose_ref(a.m, a.k, a.row_ptr, a.col_idx, a.vals)
    T = a.to_scipy().T.tocsr()
    T.sort_indices()
    assert np.array_equal(ptr, T.indptr) and np.array_equal(col, T.indices)
    assert np.array_equal(val, T.data)
    ptr2, col2, val2, perm2 = L.transpose_ref(a.k, a.m, ptr, col, val)
    assert np.array_equal(ptr2, a.row_ptr) and np.array_equal(col2, a.col_idx)
    assert np.array_equal(perm[perm2], np.arange(a.nnz))


# ---------------------------------------------------------------------------
# Eq. 1 - 3
# ---------------------------------------------------------------------------
def test_eq1_balances_predicted_times():
    """Pin: at the returned boundary the predicted times r/(TP_c t_c) and
    (R - r)/(TP_b t_b) differ by less than one row block of either part,
    and the limits give the pure modes."""
    for R, tc, nc, tb, nb, br in [(1000, 2.0, 3, 5.0, 1, 16), (65536, 1.0, 8, 1.0, 8, 16),
                                  (777, 3.0, 1, 0.5, 2, 4)]:
        r = L.eq1_boundary(R, tc, nc, tb, nb, br)
        assert r % br == 0 or r == R
        t_c, t_b = r / (tc * nc), (R - r) / (tb * nb)
        slack = br / (tc * nc) + br / (tb * nb)
        assert abs(t_c - t_b) <= slack
    assert L.eq1_boundary(100, 1.0, 4, 0.0, 0, 16) == 100
    assert L.eq1_boundary(100, 0.0, 0, 1.0, 4, 16) == 0
    assert L.eq1_boundary(64, 1.0, 1, 1.0, 1, 16) == 32


def test_quadratic_fit_recovers_exact_coefficients():
    """Pin: noise-free samples of a known quadratic are fitted exactly."""
    coef = np.array([3.0, 1.5, -0.25, -0.125, 0.0625])
    xs, ys = np.meshgrid(np.arange(0, 7), np.arange(0, 5))
    x, y = xs.ravel(), ys.ravel()
    perf = L.quad_eval(coef, x, y)
    fit = L.fit_quadratic_ref(x, y, perf)
    assert np.allclose(fit, coef, rtol=0, atol=1e-12)


def test_argmax_matches_concave_closed_form():
    """Pin: for a separable concave quadratic the unconstrained maximiser is
    x* = -a1/(2 a3), y* = -a2/(2 a4); with integer optima inside the
    feasible triangle the enumeration returns them."""
    coef = np.array([0.0, 6.0, 10.0, -1.0, -1.0])   # x* = 3, y* = 5
    assert L.argmax_ref(coef, 12) == (3, 5)
    # constraint active: x + y <= 4, maximise 6x - x^2 + 10y - y^2
    best = max(((x, y) for x in range(5) for y in range(5 - x) if x + y >= 1),
               key=lambda p: L.quad_eval(coef, *p))
    assert L.argmax_ref(coef, 4) == best == (1, 3)


def test_argmax_box_bounds():
    """Pin of the box-bounded form (x_min <= x <= x_max, y_min <= y <= y_max
    beside x + y <= T): for the separable concave quadratic with its free
    optimum (3, 5) outside the box [0, 2] x [0, 4] and T large enough that
    the triangle does not bind, each coordinate is maximised at its nearest
    box edge, the corner (2, 4); with lower bounds above the optimum the
    opposite corner (x_min, y_min) wins; and over random concave and convex
    quadratics, boxes and T the result equals an independent brute force
    that ranks candidates by value, then by (x, y)."""
    coef = np.array([0.0, 6.0, 10.0, -1.0, -1.0])   # free optimum (3, 5)
    assert L.argmax_ref(coef, 100, x_max=2, y_max=4) == (2, 4)
    assert L.argmax_ref(coef, 100, x_min=5, y_min=7, x_max=9, y_max=9) == (5, 7)
    # T binding inside the box: x + y <= 5 within [0, 2] x [0, 4]
    # maximise 6x - x^2 + 10y - y^2 on x + y <= 5: (1, 4) gives 5 + 24 = 29,
    # (2, 3) gives 8 + 21 = 29, the tie goes to the smaller x
    assert L.argmax_ref(coef, 5, x_max=2, y_max=4) == (1, 4)
    g = np.random.default_rng(17)
    for _ in range(200):
        c = g.normal(size=5) * np.array([1.0, 4.0, 4.0, 1.0, 1.0])
        T = int(g.integers(1, 12))
        x0, y0 = int(g.integers(0, 4)), int(g.integers(0, 4))
        x1, y1 = x0 + int(g.integers(0, 6)), y0 + int(g.integers(0, 6))
        cand = [(x, y) for x in range(x0, x1 + 1) for y in range(y0, y1 + 1) if 1 <= x + y <= T]
        want = None
        if cand:
            vals = [c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * y * y for x, y in cand]
            top = max(vals)
            want = min(p for p, v in zip(cand, vals) if v == top)
        assert L.argmax_ref(c, T, x_min=x0, y_min=y0, x_max=x1, y_max=y1) == want


# ---------------------------------------------------------------------------
# FP16 / BF16 rounding and per-row-block scaling
# ---------------------------------------------------------------------------
def _neighbours_check(x, q, grid_of):
    """q must be a nearest grid point of x, ties to the even code."""
    for xi, qi in zip(x, q):
        lo, hi, even = grid_of(xi)
        dl, dh = abs(xi - lo), abs(hi - xi)
        want = lo if dl < dh else hi if dh < dl else even
        assert qi == want, (xi, qi, lo, hi)


def _f16_grid(x):
    h = np.float16(x)
    a = np.nextafter(h, np.float16(-np.inf))
    b = np.nextafter(h, np.float16(np.inf))
    cands = sorted({float(a), float(h), float(b)})
    lo = max(c for c in cands if c <= x)
    hi = min(c for c in cands if c >= x)
    codes = {float(v): int(np.float16(v).view(np.uint16)) for v in cands}
    even = lo if codes[lo] % 2 == 0 else hi
    return lo, hi, even


def test_round_f16_nearest_even_brute_force():
    """Pin: every rounded value is a nearest FP16 neighbour, ties to even,
    across normal and subnormal magnitudes; and equals numpy's float16."""
    g = np.random.default_rng(0)
    x = np.concatenate([
        g.uniform(-2, 2, 2000),
        g.uniform(-1, 1, 500) * 2.0 ** -14,           # subnormal range
        g.uniform(-1, 1, 500) * 2.0 ** g.integers(-20, 15, 500),
        # exact ties between neighbouring codes
        (np.arange(1, 200) + 0.5) * 2.0 ** -10,
        (np.arange(1, 50) + 0.5) * 2.0 ** -24,
    ])
    q = L.round_rne_ref(x, "f16")
    _neighbours_check(x, q, _f16_grid)
    assert np.array_equal(q, x.astype(np.float16).astype(np.float64))
    assert np.isinf(L.round_rne_ref(np.array([65520.0]), "f16"))[0]
    assert L.round_rne_ref(np.array([65519.0]), "f16")[0] == 65504.0


def _bf16_grid(x):
    bits = int(np.float32(x).view(np.uint32)) & 0xFFFF0000
    cand = set()
    for d in (-2, -1, 0, 1, 2):
        b = (bits + (d << 16)) & 0xFFFFFFFF
        v = float(np.array([b], np.uint32).view(np.float32)[0])
        if math.isfinite(v):
            cand.add(v)
    lo = max(c for c in cand if c <= x)
    hi = min(c for c in cand if c >= x)
    code = lambda v: int(np.float32(v).view(np.uint32)) >> 16
    even = lo if code(lo) % 2 == 0 else hi
    return lo, hi, even


def test_round_bf16_nearest_even_brute_force():
    """Pin: brute-force nearest BF16 neighbour (from the FP32 bit grid),
    ties to even, straight from FP64 (no double rounding through FP32)."""
    g = np.random.default_rng(1)
    x = np.concatenate([
        g.uniform(-2, 2, 2000),
        g.uniform(-1, 1, 500) * 2.0 ** g.integers(-60, 60, 500),
        (np.arange(1, 300) + 0.5) * 2.0 ** -7,
    ])
    # a value just above a tie that FP32 rounding would turn into the tie
    x = np.append(x, 1.0 + 2.0 ** -8 + 2.0 ** -40)
    q = L.round_rne_ref(x, "bf16")
    _neighbours_check(x, q, _bf16_grid)
    assert q[-1] == 1.0 + 2.0 ** -7


def test_quantize_scales_are_exact_powers_of_two():
    """Pins: s = 2^floor(log2 max|a|) per row block; |a/s| in [0, 2);
    values of the form (integer < 2^10) * s_q are stored exactly."""
    a = gen.random_csr(2, 64, 64, 0.2)
    codes, s, deq = L.quantize_ref(a.m, a.row_ptr, a.vals, 16, "f16")
    for q in range(s.size):
        lo, hi = a.row_ptr[q * 16], a.row_ptr[q * 16 + 16]
        amax = np.max(np.abs(a.vals[lo:hi]))
        assert s[q] <= amax < 2 * s[q]
        assert math.frexp(s[q])[0] == 0.5
    se = s[a.rows() // 16]
    normal = np.abs(a.vals) / se >= 2.0 ** -14
    rel = np.abs(deq - a.vals)[normal] / np.abs(a.vals)[normal]
    assert rel.max() <= 2.0 ** -11          # half an ulp of an 11-bit significand
    # values (integer with fewer significant bits than the format) * 2^j
    g = np.random.default_rng(3)
    rows = a.rows()
    scale = 2.0 ** g.integers(-30, 30, (a.m + 15) // 16)
    for fmt, bits in (("f16", 11), ("bf16", 8)):
        ints = g.integers(-(2 ** bits - 1), 2 ** bits, a.nnz).astype(float)
        v = ints * scale[rows // 16]
        _, _, deq = L.quantize_ref(a.m, a.row_ptr, v, 16, fmt)
        assert np.array_equal(deq, v), fmt


def test_codes_round_trip():
    q = L.round_rne_ref(np.random.default_rng(4).uniform(-2, 2, 100), "bf16")
    c = L.codes_ref(q, "bf16")
    back = (c.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert np.array_equal(back, q)
    q16 = L.round_rne_ref(np.random.default_rng(5).uniform(-2, 2, 100), "f16")
    assert np.array_equal(L.codes_ref(q16, "f16").view(np.float16).astype(float), q16)
