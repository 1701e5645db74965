"""CPU restatement of the hybrid-format steps -- TEST INFRASTRUCTURE ONLY.

Written from the paper's description, step by step and slowly, so that the
arrays the device plan builds can be compared with these as exact integers:

* canonicalize_ref  -- the readings for ambiguous inputs: columns ascending
                       inside a row (a hash map has no order, Sec. 3.2.2) and
                       duplicate (row, col) entries summed (plain definition
                       of the product, Sec. 2.1).
* convert_ref       -- Alg. 1 (Sec. 3.2.2): the top r_boundary rows copied
                       into a CSR-part; the remaining rows cut into
                       B_r x 1 column tiles keyed by (i div B_r, j), tile
                       element (i mod B_r) holding the value.
* convert_assign_ref-- the same tiling where every B_r-row block is sent to
                       one part or the other independently (a contiguous
                       boundary is the special case).
* eq1_boundary      -- Eq. 1, read as balancing the two parts' predicted
                       times, rounded to a multiple of B_r.
* fit_quadratic_ref -- Eq. 2, least squares on [1, x, y, x^2, y^2].
* argmax_ref        -- Eq. 3, enumeration of x + y <= T.
* quantize_ref      -- FP16/BF16 storage of A with one power-of-two scale per
                       B_r-row block, round-to-nearest-even from FP64.
* transpose_ref     -- CSR of A^T, entries of a column kept in row order.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------
# canonical form
# ---------------------------------------------------------------------------
def canonicalize_ref(m, k, row_ptr, col_idx, vals):
    """Return (row_ptr, col, vals, canon_of_orig): columns ascending per row,
    duplicates summed in stored order; canon_of_orig[e] is the canonical
    position that original entry e went to."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    out_ptr = [0]
    out_col, out_val = [], []
    canon = np.empty(col_idx.shape[0], dtype=np.int64)
    for i in range(m):
        lo, hi = int(row_ptr[i]), int(row_ptr[i + 1])
        seen = {}
        for e in range(lo, hi):
            j = int(col_idx[e])
            seen.setdefault(j, []).append(e)
        for j in sorted(seen):
            total = 0.0
            for e in seen[j]:
                total += float(vals[e])
                canon[e] = len(out_col)
            out_col.append(j)
            out_val.append(total)
        out_ptr.append(len(out_col))
    return (np.array(out_ptr, dtype=np.int64), np.array(out_col, dtype=np.int64),
            np.array(out_val, dtype=np.float64), canon)


# ---------------------------------------------------------------------------
# Alg. 1
# ---------------------------------------------------------------------------
def convert_assign_ref(m, row_ptr, col_idx, vals, rb_is_bcsr, br):
    """Tile a canonical CSR matrix.  rb_is_bcsr[q] says whether row block q
    (rows q*br .. q*br+br-1) goes to the BCSR-part.

    Returns a dict with
      csr_rows, csr_ptr, csr_col, csr_val      CSR-part (rows ascending)
      bcsr_rb, blk_ptr, blk_col, blk_val       BCSR-part; blk_val is [nblk, br]
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    nrb = (m + br - 1) // br
    rb_is_bcsr = np.asarray(rb_is_bcsr, dtype=bool)
    assert rb_is_bcsr.shape == (nrb,)

    # Step 1: CSR-part, every row of a CSR row block copied as stored
    csr_rows, csr_ptr, csr_col, csr_val = [], [0], [], []
    for i in range(m):
        if rb_is_bcsr[i // br]:
            continue
        csr_rows.append(i)
        for e in range(row_ptr[i], row_ptr[i + 1]):
            csr_col.append(int(col_idx[e]))
            csr_val.append(float(vals[e]))
        csr_ptr.append(len(csr_col))

    # Step 2: BCSR-part, tiles keyed by (tile_r, tile_c) = (i div br, j)
    tile_map = {}
    for i in range(m):
        if not rb_is_bcsr[i // br]:
            continue
        for e in range(row_ptr[i], row_ptr[i + 1]):
            j = int(col_idx[e])
            key = (i // br, j)
            if key not in tile_map:
                tile_map[key] = np.zeros(br)
            tile_map[key][i % br] += float(vals[e])
    bcsr_rb = [q for q in range(nrb) if rb_is_bcsr[q]]
    blk_ptr, blk_col, blk_val = [0], [], []
    for q in bcsr_rb:
        cols = sorted(j for (r, j) in tile_map if r == q)
        for j in cols:
            blk_col.append(j)
            blk_val.append(tile_map[(q, j)])
        blk_ptr.append(len(blk_col))
    return {
        "csr_rows": np.array(csr_rows, dtype=np.int64),
        "csr_ptr": np.array(csr_ptr, dtype=np.int64),
        "csr_col": np.array(csr_col, dtype=np.int64),
        "csr_val": np.array(csr_val, dtype=np.float64),
        "bcsr_rb": np.array(bcsr_rb, dtype=np.int64),
        "blk_ptr": np.array(blk_ptr, dtype=np.int64),
        "blk_col": np.array(blk_col, dtype=np.int64),
        "blk_val": np.array(blk_val, dtype=np.float64).reshape(-1, br),
    }


def convert_ref(m, row_ptr, col_idx, vals, r_boundary, br):
    """Alg. 1 with a contiguous boundary: rows [0, r_boundary) form the
    CSR-part, rows [r_boundary, m) the BCSR-part.  r_boundary must be a
    multiple of br (or m) so that no tile straddles the two parts."""
    if not (r_boundary == m or r_boundary % br == 0):
        raise ValueError("r_boundary must be a multiple of the tile height")
    nrb = (m + br - 1) // br
    is_b = np.array([q * br >= r_boundary for q in range(nrb)], dtype=bool)
    return convert_assign_ref(m, row_ptr, col_idx, vals, is_b, br)


def rowblock_stats_ref(m, row_ptr, col_idx, br):
    """Per row block: stored entries and number of distinct columns (the
    number of non-empty br x 1 tiles)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    nrb = (m + br - 1) // br
    nnz = np.zeros(nrb, dtype=np.int64)
    nblk = np.zeros(nrb, dtype=np.int64)
    for q in range(nrb):
        lo, hi = row_ptr[q * br], row_ptr[min(m, q * br + br)]
        nnz[q] = hi - lo
        nblk[q] = np.unique(np.asarray(col_idx[lo:hi])).size
    return nnz, nblk


def to_coo_ref(m, fmt, br):
    """Expand a converted matrix back to sorted (row, col, val) triplets,
    dropping explicit zeros created by tile padding."""
    out = {}
    for r, i in enumerate(fmt["csr_rows"]):
        for e in range(fmt["csr_ptr"][r], fmt["csr_ptr"][r + 1]):
            key = (int(i), int(fmt["csr_col"][e]))
            out[key] = out.get(key, 0.0) + float(fmt["csr_val"][e])
    for t, q in enumerate(fmt["bcsr_rb"]):
        for b in range(fmt["blk_ptr"][t], fmt["blk_ptr"][t + 1]):
            for off in range(br):
                v = float(fmt["blk_val"][b, off])
                i = int(q) * br + off
                if v != 0.0 and i < m:
                    key = (i, int(fmt["blk_col"][b]))
                    out[key] = out.get(key, 0.0) + v
    keys = sorted(out)
    return [(i, j, out[(i, j)]) for (i, j) in keys]


# ---------------------------------------------------------------------------
# Eq. 1-3
# ---------------------------------------------------------------------------
def eq1_boundary(r_total, tp_csr, t_csr, tp_bcsr, t_bcsr, br):
    """Row boundary that equalises the predicted times of the two parts:
    r / (TP_c t_c) = (r_total - r) / (TP_b t_b), i.e.
    r = r_total TP_c t_c / (TP_c t_c + TP_b t_b), rounded to the nearest
    multiple of br and clamped to [0, r_total]."""
    wc = float(tp_csr) * float(t_csr)
    wb = float(tp_bcsr) * float(t_bcsr)
    if wc <= 0 and wb <= 0:
        raise ValueError("both parts have zero capacity")
    if wb <= 0:
        return int(r_total)
    if wc <= 0:
        return 0
    r = r_total * wc / (wc + wb)
    rb = int(math.floor(r / br + 0.5)) * br
    return int(min(max(rb, 0), r_total))


def fit_quadratic_ref(x, y, perf):
    """Least-squares coefficients (a0..a4) of perf = a0 + a1 x + a2 y +
    a3 x^2 + a4 y^2."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    A = np.stack([np.ones_like(x), x, y, x * x, y * y], axis=1)
    coef, *_ = np.linalg.lstsq(A, np.asarray(perf, dtype=np.float64), rcond=None)
    return coef


def quad_eval(coef, x, y):
    a0, a1, a2, a3, a4 = coef
    return a0 + a1 * x + a2 * y + a3 * x * x + a4 * y * y


def argmax_ref(coef, T, x_min=0, y_min=0, x_max=None, y_max=None):
    """argmax of the quadratic over integers x_min <= x <= x_max,
    y_min <= y <= y_max, 1 <= x + y <= T (bounds default to T); ties go to
    the first pair in (x, y) lexicographic order."""
    x_max = T if x_max is None else x_max
    y_max = T if y_max is None else y_max
    best, arg = -math.inf, None
    for x in range(x_min, min(T, x_max) + 1):
        for y in range(y_min, min(T - x, y_max) + 1):
            if x + y < 1:
                continue
            v = quad_eval(coef, x, y)
            if v > best:
                best, arg = v, (x, y)
    return arg


# ---------------------------------------------------------------------------
# FP16 / BF16 storage of A
# ---------------------------------------------------------------------------
_FMT = {
    # significant bits (incl. hidden), exponent of the smallest normal, largest finite
    "f16": (11, -14, 65504.0),
    "bf16": (8, -126, float.fromhex("0x1.fep127")),
}


def round_rne_ref(x, fmt):
    """Round float64 values to the nearest value of a binary format (f16 or
    bf16), ties to even, directly from float64 (no intermediate format).
    The quantum of x is 2^(e - p) with x = f 2^e, 0.5 <= |f| < 1, p the
    significant bits, floored at the subnormal quantum 2^(emin - p + 1)."""
    p, emin, maxf = _FMT[fmt]
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    f, e = np.frexp(x[nz])
    qexp = np.maximum(e.astype(np.int64) - p, emin - p + 1)
    scaled = np.ldexp(x[nz], -qexp)          # exact: power-of-two scaling
    r = np.rint(scaled)                        # ties to even
    out[nz] = np.ldexp(r, qexp)
    big = np.abs(out) > maxf
    out[big] = np.copysign(np.inf, out[big])
    return out


def codes_ref(q, fmt):
    """Bit patterns (uint16) of values already representable in fmt."""
    q = np.asarray(q, dtype=np.float64)
    if fmt == "f16":
        return q.astype(np.float16).view(np.uint16)
    return (q.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def rowblock_scales_ref(m, row_ptr, vals, br):
    """s_q = 2^floor(log2 max|a|) over the stored entries of row block q
    (1 for an all-zero or empty block)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    nrb = (m + br - 1) // br
    s = np.ones(nrb, dtype=np.float64)
    for q in range(nrb):
        lo, hi = row_ptr[q * br], row_ptr[min(m, q * br + br)]
        if hi > lo:
            amax = float(np.max(np.abs(vals[lo:hi])))
            if amax > 0:
                _, e = math.frexp(amax)      # amax = f 2^e, 0.5 <= f < 1
                s[q] = math.ldexp(1.0, e - 1)
    return s


def quantize_ref(m, row_ptr, vals, br, fmt):
    """Return (codes uint16 per entry, scales per row block, dequantised
    FP64 values q * s)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    s = rowblock_scales_ref(m, row_ptr, vals, br)
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    se = s[rows // br]
    q = round_rne_ref(vals / se, fmt)
    return codes_ref(q, fmt), s, q * se


# ---------------------------------------------------------------------------
# transpose
# ---------------------------------------------------------------------------
def transpose_ref(m, k, row_ptr, col_idx, vals=None):
    """CSR of A^T (k rows); entries of each column of A kept in row order.
    Returns (row_ptr_t, col_t, vals_t, perm) with perm[t] the index of the
    A entry that became entry t of A^T."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(row_ptr))
    buckets = [[] for _ in range(k)]
    for e in range(col_idx.shape[0]):
        buckets[int(col_idx[e])].append(e)
    perm = np.array([e for b in buckets for e in b], dtype=np.int64)
    ptr = np.zeros(k + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(b) for b in buckets])
    col_t = rows[perm] if perm.size else np.zeros(0, dtype=np.int64)
    vt = None if vals is None else np.asarray(vals, dtype=np.float64)[perm]
    return ptr, col_t, vt, perm
