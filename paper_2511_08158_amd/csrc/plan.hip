// Plan construction on the device: CSR validation, canonical form,
// row-block statistics, the cost-model split, Alg. 1 (CSR-part compaction
// and BCSR tiling with tiles in ascending column order), the transposed
// plan, and packing of the values in the compute dtype.
#include <algorithm>
#include <chrono>
#include <cstdlib>

#include "group.h"
#include "plan.h"
#include "prim.h"

namespace hspmm {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int threads = kThreads) {
    int64_t g = ceil_div(n, threads);
    if (g > 262144) g = 262144;
    if (g < 1) g = 1;
    return (unsigned)g;
}
inline unsigned grid_waves(int64_t nwaves) { return grid_for(nwaves * 64); }

#define GRID_STRIDE(i, n)                                                        \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)
#define WAVE_STRIDE(w, n)                                                                  \
    for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < (n); \
         w += ((int64_t)gridDim.x * blockDim.x) >> 6)

enum : int32_t { FLAG_ROWPTR = 1, FLAG_COL = 2, FLAG_NONCANON = 4 };

// ---------------------------------------------------------------------------
// validation and row expansion
// ---------------------------------------------------------------------------
__global__ void k_check_rowptr(const int32_t* __restrict__ rp, int64_t m, int64_t nnz, int32_t* flags) {
    GRID_STRIDE(i, m + 1) {
        const int32_t v = rp[i];
        bool bad = v < 0 || v > nnz;
        if (i == 0 && v != 0) bad = true;
        if (i == m && v != nnz) bad = true;
        if (i < m && rp[i + 1] < v) bad = true;
        if (bad) atomicOr(flags, FLAG_ROWPTR);
    }
}

__global__ void k_expand_rows(const int32_t* __restrict__ rp, int64_t m, int32_t* __restrict__ row_of) {
    const int lane = threadIdx.x & 63;
    WAVE_STRIDE(i, m) {
        const int32_t lo = rp[i], hi = rp[i + 1];
        for (int32_t e = lo + lane; e < hi; e += 64) row_of[e] = (int32_t)i;
    }
}

__global__ void k_check_cols(const int32_t* __restrict__ col, const int32_t* __restrict__ row_of, int64_t nnz,
                             int64_t k, int32_t* flags) {
    GRID_STRIDE(e, nnz) {
        const int32_t c = col[e];
        if (c < 0 || c >= k) {
            atomicOr(flags, FLAG_COL);
        } else if (e > 0 && row_of[e] == row_of[e - 1] && col[e - 1] >= c) {
            atomicOr(flags, FLAG_NONCANON);
        }
    }
}

// ---------------------------------------------------------------------------
// canonical form: entries sorted by (row, col), duplicates merged
// ---------------------------------------------------------------------------
__global__ void k_copy_u32_from_i32(uint32_t* dst, const int32_t* src, int64_t n) {
    GRID_STRIDE(i, n) dst[i] = (uint32_t)src[i];
}

__global__ void k_mark_heads(const int32_t* __restrict__ perm, const int32_t* __restrict__ row_of,
                             const int32_t* __restrict__ col, int64_t n, int32_t* __restrict__ head) {
    GRID_STRIDE(t, n) {
        int32_t h = 1;
        if (t > 0) {
            const int32_t a = perm[t], b = perm[t - 1];
            h = (row_of[a] != row_of[b] || col[a] != col[b]) ? 1 : 0;
        }
        head[t] = h;
    }
}

__global__ void k_canon_build(const int32_t* __restrict__ perm, const int32_t* __restrict__ head,
                              const int32_t* __restrict__ hx, const int32_t* __restrict__ row_of,
                              const int32_t* __restrict__ col, int64_t n, int32_t* __restrict__ canon_of_orig,
                              int32_t* __restrict__ seg, int32_t* __restrict__ ccol, int32_t* __restrict__ crow) {
    GRID_STRIDE(t, n) {
        const int32_t c = hx[t] + head[t] - 1;
        const int32_t e = perm[t];
        canon_of_orig[e] = c;
        if (head[t]) {
            seg[c] = (int32_t)t;
            ccol[c] = col[e];
            crow[c] = row_of[e];
        }
    }
}

__global__ void k_set_i32(int32_t* p, int32_t v) { *p = v; }

// Row pointer of a list sorted by row (key[0..n) ascending, rows < nrows):
// rp[r] = the first t with key[t] >= r (n if none), so rp[nrows] = n.  One
// thread per row finds it by binary search: a long stretch of empty rows
// costs no more than any other rows (writing the rows between consecutive
// keys from the key's thread would leave one thread all of them).
__global__ void k_row_starts(const int32_t* __restrict__ key, int64_t n, int64_t nrows, int32_t* __restrict__ rp) {
    GRID_STRIDE(r, nrows + 1) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (key[mid] < r) {
                lo = mid + 1;
            } else {
                hi = mid;
            }
        }
        rp[r] = (int32_t)lo;
    }
}

// ---------------------------------------------------------------------------
// row-block statistics and tiling (Alg. 1 step 2)
// ---------------------------------------------------------------------------
__global__ void k_gather_rb_key(uint32_t* __restrict__ key, const int32_t* __restrict__ row_of,
                                const int32_t* __restrict__ ord, int64_t n) {
    GRID_STRIDE(t, n) key[t] = (uint32_t)(row_of[ord[t]] >> 4);
}

__global__ void k_tile_heads(const int32_t* __restrict__ ord, const int32_t* __restrict__ row_of,
                             const int32_t* __restrict__ col, int64_t n, int32_t* __restrict__ hd) {
    GRID_STRIDE(t, n) {
        int32_t h = 1;
        if (t > 0) {
            const int32_t a = ord[t], b = ord[t - 1];
            h = ((row_of[a] >> 4) != (row_of[b] >> 4) || col[a] != col[b]) ? 1 : 0;
        }
        hd[t] = h;
    }
}

__global__ void k_rb_nblk(const int32_t* __restrict__ rp, const int32_t* __restrict__ hx, const int32_t* total,
                          int64_t m, int64_t nrb, int64_t n, int32_t* __restrict__ nblk) {
    GRID_STRIDE(q, nrb) {
        const int64_t r0 = q * 16, r1 = min(m, q * 16 + 16);
        const int32_t s = rp[r0], e = rp[r1];
        const int32_t hs = s < n ? hx[s] : *total;
        const int32_t he = e < n ? hx[e] : *total;
        nblk[q] = he - hs;
    }
}

__host__ __device__ inline int64_t pack_index(int64_t blk, int i, bool half) {
    // FP32/FP64: [tile][16]; FP16/BF16: per 32-tile step [tile/8 group][row][tile%8]
    if (!half) return blk * 16 + i;
    return (blk >> 5) * 512 + ((blk & 31) >> 3) * 128 + i * 8 + (blk & 7);
}

__global__ void k_build_csr(const int32_t* __restrict__ rows, const int32_t* __restrict__ cptr, int64_t nrows,
                            const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ src, int32_t* __restrict__ ccol,
                            int32_t* __restrict__ csrc) {
    const int lane = threadIdx.x & 63;
    WAVE_STRIDE(r, nrows) {
        const int32_t row = rows[r];
        const int32_t lo = rp[row], len = rp[row + 1] - lo, out = cptr[r];
        for (int32_t t = lane; t < len; t += 64) {
            ccol[out + t] = col[lo + t];
            csrc[out + t] = src ? src[lo + t] : lo + t;
        }
    }
}

__global__ void k_build_bcsr(const int32_t* __restrict__ ord, const int32_t* __restrict__ hd,
                             const int32_t* __restrict__ hx, const int32_t* __restrict__ row_of,
                             const int32_t* __restrict__ col, const int32_t* __restrict__ src,
                             const int32_t* __restrict__ rp, const int32_t* __restrict__ rb_slot,
                             const int32_t* __restrict__ blk_ptr, int64_t n, bool half,
                             int32_t* __restrict__ blk_col, int32_t* __restrict__ blk_src) {
    GRID_STRIDE(t, n) {
        const int32_t x = ord[t];
        const int32_t row = row_of[x];
        const int32_t q = row >> 4;
        const int32_t sl = rb_slot[q];
        if (sl < 0) continue;
        const int32_t gb0 = hx[rp[q * 16]];
        const int32_t local = hx[t] + hd[t] - 1 - gb0;
        const int64_t blk = (int64_t)blk_ptr[sl] + local;
        if (hd[t]) blk_col[blk] = col[x];
        blk_src[pack_index(blk, row & 15, half)] = src ? src[x] : x;
    }
}

// occupancy mask of every tile from its slot -> entry map
__global__ void k_build_mask(const int32_t* __restrict__ blk_src, int64_t nblk_pad, bool half,
                             uint16_t* __restrict__ blk_mask) {
    GRID_STRIDE(t, nblk_pad) {
        uint32_t mk = 0;
        for (int i = 0; i < 16; ++i) mk |= (blk_src[pack_index(t, i, half)] >= 0 ? 1u : 0u) << i;
        blk_mask[t] = (uint16_t)mk;
    }
}

// CSR-part work list, per row r of the sub-matrix: c[0] in the CSR-part,
// c[1] its entries, c[2] its virtual rows, c[3] long (cut into segments),
// c[4] its partial slots (all 0 outside the CSR-part); arrays of m each
__global__ void k_wl_counts(const int32_t* __restrict__ rp, const uint8_t* __restrict__ cls, int64_t m, int br,
                            int32_t seg, int32_t* __restrict__ c) {
    GRID_STRIDE(r, m) {
        const int32_t in = cls[r / br] ? 0 : 1;
        const int32_t len = rp[r + 1] - rp[r];
        const int32_t lng = in && len > seg ? 1 : 0;
        const int32_t ns = lng ? (len + seg - 1) / seg : in;
        c[r] = in;
        c[m + r] = in ? len : 0;
        c[2 * m + r] = ns;
        c[3 * m + r] = lng;
        c[4 * m + r] = lng ? ns : 0;
    }
}

// Fill the CSR-part's rows and row pointer, the virtual rows (a long row's
// segments in its place) and the long rows, from the counts' exclusive sums
// x (same layout as c)
__global__ void k_wl_fill(const int32_t* __restrict__ rp, const int32_t* __restrict__ c,
                          const int32_t* __restrict__ x, int64_t m, int32_t seg, int64_t nrows_c,
                          int32_t* __restrict__ rows, int32_t* __restrict__ cptr, int32_t* __restrict__ vs,
                          int32_t* __restrict__ ve, int32_t* __restrict__ vo, int32_t* __restrict__ vrow,
                          int32_t* __restrict__ lrow, int32_t* __restrict__ lfirst, int32_t* __restrict__ lcnt) {
    GRID_STRIDE(r, m) {
        if (!c[r]) continue;
        const int32_t ri = x[r], base = x[m + r], len = c[m + r], v0 = x[2 * m + r];
        rows[ri] = (int32_t)r;
        cptr[ri] = base;
        if (ri == nrows_c - 1) cptr[nrows_c] = base + len;
        if (c[3 * m + r]) {
            const int32_t li = x[3 * m + r], p0 = x[4 * m + r], ns = c[2 * m + r];
            lrow[li] = (int32_t)r;
            lfirst[li] = p0;
            lcnt[li] = ns;
            for (int32_t k = 0; k < ns; ++k) {
                vs[v0 + k] = base + k * seg;
                ve[v0 + k] = min(base + len, base + (k + 1) * seg);
                vo[v0 + k] = -(p0 + k + 1);
                vrow[v0 + k] = (int32_t)r;
            }
        } else {
            vs[v0] = base;
            ve[v0] = base + len;
            vo[v0] = (int32_t)r;
            vrow[v0] = (int32_t)r;
        }
    }
}

// sort key of virtual row v: its window, then 31 - floor(log2 len) (the
// longest first; lengths 0 and 1 are class 0)
__global__ void k_wl_keys(const int32_t* __restrict__ vs, const int32_t* __restrict__ ve, int64_t nv, int32_t window,
                          uint32_t* __restrict__ key) {
    GRID_STRIDE(v, nv) {
        const uint32_t len = (uint32_t)(ve[v] - vs[v]);
        const uint32_t cls = len > 1 ? 31u - (uint32_t)__clz((int)len) : 0u;
        key[v] = ((uint32_t)(v / window) << 5) | (31u - cls);
    }
}

__global__ void k_wl_gather(const int32_t* __restrict__ idx, int64_t nv, const int32_t* __restrict__ vs,
                            const int32_t* __restrict__ ve, const int32_t* __restrict__ vo,
                            const int32_t* __restrict__ vrow, int32_t* __restrict__ os, int32_t* __restrict__ oe,
                            int32_t* __restrict__ oo, int32_t* __restrict__ orow) {
    GRID_STRIDE(v, nv) {
        const int32_t i = idx[v];
        os[v] = vs[i];
        oe[v] = ve[i];
        oo[v] = vo[i];
        orow[v] = vrow[i];
    }
}

// fused-backward tables of A^T: which rows of each tile hold an entry, and
// the entry of the lowest such row (A's canonical index)
__global__ void k_tile_meta(const int32_t* __restrict__ blk_src, int64_t nblk_pad, int32_t* __restrict__ base,
                            uint16_t* __restrict__ mask) {
    GRID_STRIDE(t, nblk_pad) {
        uint32_t mk = 0;
        int32_t b = 0;
        for (int i = 15; i >= 0; --i) {
            const int32_t v = blk_src[t * 16 + i];
            if (v >= 0) {
                mk |= 1u << i;
                b = v;
            }
        }
        base[t] = b;
        mask[t] = (uint16_t)mk;
    }
}

// SDDMM chunk tables: one thread per (row block, row) walks the row block's
// chunks of 16 tiles in order, keeping the running canonical index of the
// row's next entry (tiles are sorted by column, as are a row's entries)
__global__ void k_build_chunk_meta(const int32_t* __restrict__ bcsr_rb, const int32_t* __restrict__ blk_ptr,
                                   const int32_t* __restrict__ blk_cnt, const uint16_t* __restrict__ blk_mask,
                                   const int32_t* __restrict__ chunk_ptr, const int32_t* __restrict__ canon_rp,
                                   int64_t m, int64_t n_rb, bool interleaved, int32_t* __restrict__ chunk_base,
                                   uint16_t* __restrict__ chunk_mask) {
    GRID_STRIDE(x, n_rb * 16) {
        const int64_t slot = x >> 4;
        const int R = (int)(x & 15);
        const int64_t row = (int64_t)bcsr_rb[slot] * 16 + R;
        const int b0 = blk_ptr[slot], cnt = blk_cnt[slot];
        const int64_t c0 = chunk_ptr[slot];
        // position of row R in the MFMA output: FP64 holds rows g + 4r in
        // lane group g, register r; the other types rows 4g + r
        const int pos = interleaved ? 4 * (R & 3) + (R >> 2) : R;
        int32_t run = row < m ? canon_rp[row] : 0;
        for (int c = 0; 16 * c < cnt; ++c) {
            uint32_t mk = 0;
            for (int t = 0; t < 16 && 16 * c + t < cnt; ++t) mk |= ((blk_mask[b0 + 16 * c + t] >> R) & 1u) << t;
            chunk_mask[(c0 + c) * 16 + pos] = (uint16_t)mk;
            chunk_base[(c0 + c) * 16 + pos] = run;
            run += __popc(mk);
        }
    }
}

// ---------------------------------------------------------------------------
// values
// ---------------------------------------------------------------------------
template <class T> __device__ inline double in_value(const void* v, int64_t i);
template <> __device__ inline double in_value<double>(const void* v, int64_t i) {
    return static_cast<const double*>(v)[i];
}
template <> __device__ inline double in_value<float>(const void* v, int64_t i) {
    return (double)static_cast<const float*>(v)[i];
}
template <> __device__ inline double in_value<half_t>(const void* v, int64_t i) {
    return (double)(float)static_cast<const half_t*>(v)[i];
}
template <> __device__ inline double in_value<bf16_t>(const void* v, int64_t i) {
    return (double)bf16_to_float(static_cast<const bf16_t*>(v)[i]);
}

// vb[c] = sum of the input values merged into canonical entry c, in input order
template <class T>
__global__ void k_base_values(const void* __restrict__ vals, const int32_t* __restrict__ perm,
                              const int32_t* __restrict__ seg, int64_t nc, double* __restrict__ vb) {
    GRID_STRIDE(c, nc) {
        if (!perm) {
            vb[c] = in_value<T>(vals, c);
        } else {
            double s = 0.0;
            for (int32_t t = seg[c]; t < seg[c + 1]; ++t) s += in_value<T>(vals, perm[t]);
            vb[c] = s;
        }
    }
}

// scale[q] = 2^floor(log2 max |a|) over row block q (1 if all zero)
__global__ void k_rb_scale(const int32_t* __restrict__ rp, const double* __restrict__ vb, int64_t m,
                           int64_t nrb, double* __restrict__ scale) {
    const int lane = threadIdx.x & 63;
    WAVE_STRIDE(q, nrb) {
        const int32_t lo = rp[q * 16], hi = rp[min(m, q * 16 + 16)];
        double mx = 0.0;
        for (int32_t e = lo + lane; e < hi; e += 64) mx = fmax(mx, fabs(vb[e]));
        for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) {
            double s = 1.0;
            if (mx > 0.0 && mx < INFINITY) {
                int ex;
                frexp(mx, &ex);          // mx = f 2^ex, 0.5 <= f < 1
                s = ldexp(1.0, ex - 1);
            }
            scale[q] = s;
        }
    }
}

__device__ inline float f16_code_to_float(uint16_t c) {
    half_t h;
    memcpy(&h, &c, 2);
    return (float)h;
}
__device__ inline float bf16_code_to_float(uint16_t c) {
    uint32_t u = (uint32_t)c << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// value of canonical A entry c as stored in A's parts, for the A^T parts
__device__ inline double eff_value(int act, const double* vb, int64_t c, const double* scale,
                                   const int32_t* row_of) {
    const double v = vb[c];
    switch (act) {
        case HSPMM_F32: return (double)(float)v;
        case HSPMM_F16: {
            const double s = scale[row_of[c] >> 4];
            return (double)f16_code_to_float(double_to_f16_code(v / s)) * s;
        }
        case HSPMM_BF16: {
            const double s = scale[row_of[c] >> 4];
            return (double)bf16_code_to_float(double_to_bf16_code(v / s)) * s;
        }
        default: return v;
    }
}

template <class TO> __device__ inline TO to_stored(double x);
template <> __device__ inline double to_stored<double>(double x) { return x; }
template <> __device__ inline float to_stored<float>(double x) { return (float)x; }
template <> __device__ inline half_t to_stored<half_t>(double x) {
    const uint16_t c = double_to_f16_code(x);
    half_t h;
    memcpy(&h, &c, 2);
    return h;
}
template <> __device__ inline bf16_t to_stored<bf16_t>(double x) {
    const uint16_t c = double_to_bf16_code(x);
    bf16_t h;
    memcpy(&h, &c, 2);
    return h;
}

// A's own parts: stored = value / scale[row block] in TO (scale null = 1).
// A^T parts (act >= 0): stored = the value A's parts hold, in TO.
template <class TO>
__global__ void k_pack_csr(const int32_t* __restrict__ rows, const int32_t* __restrict__ cptr, int64_t nrows,
                           const int32_t* __restrict__ csrc, const double* __restrict__ vb,
                           const double* __restrict__ scale, int act, const double* __restrict__ a_scale,
                           const int32_t* __restrict__ row_of, TO* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    WAVE_STRIDE(r, nrows) {
        const int32_t row = rows[r];
        const int32_t lo = cptr[r], hi = cptr[r + 1];
        const double s = scale ? scale[row >> 4] : 1.0;
        for (int32_t q = lo + lane; q < hi; q += 64) {
            const int32_t c = csrc[q];
            const double v = act >= 0 ? eff_value(act, vb, c, a_scale, row_of) : vb[c] / s;
            out[q] = to_stored<TO>(v);
        }
    }
}

template <class TO>
__global__ void k_pack_bcsr(const int32_t* __restrict__ rbl, const int32_t* __restrict__ bptr, int64_t nrb_b,
                            const int32_t* __restrict__ bsrc, const double* __restrict__ vb,
                            const double* __restrict__ scale, int act, const double* __restrict__ a_scale,
                            const int32_t* __restrict__ row_of, TO* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    WAVE_STRIDE(sl, nrb_b) {
        const int32_t q = rbl[sl];
        const int64_t lo = (int64_t)bptr[sl] * 16, hi = (int64_t)bptr[sl + 1] * 16;
        const double s = scale ? scale[q] : 1.0;
        for (int64_t i = lo + lane; i < hi; i += 64) {
            const int32_t c = bsrc[i];
            double v = 0.0;
            if (c >= 0) v = act >= 0 ? eff_value(act, vb, c, a_scale, row_of) : vb[c] / s;
            out[i] = to_stored<TO>(v);
        }
    }
}

__global__ void k_transpose_fill(const int32_t* __restrict__ ord, const int32_t* __restrict__ row_of,
                                 const int32_t* __restrict__ col, int64_t n, int32_t* __restrict__ tcol,
                                 int32_t* __restrict__ trow) {
    GRID_STRIDE(t, n) {
        const int32_t c = ord[t];
        tcol[t] = row_of[c];
        trow[t] = col[c];
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
template <class T>
int upload(Allocator& al, DevBuf& b, const std::vector<T>& h, hipStream_t s) {
    HSPMM_TRY(al.alloc(b, std::max<size_t>(1, h.size()) * sizeof(T)));
    if (!h.empty()) HIP_TRY(hipMemcpyAsync(b.ptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return HSPMM_OK;
}
template <class T>
int download(std::vector<T>& h, const void* d, size_t n, hipStream_t s) {
    h.resize(n);
    if (n) HIP_TRY(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HSPMM_OK;
}

int read_flag(const int32_t* d, int32_t* h, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(h, d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HSPMM_OK;
}

// Sort positions 0..n-1 of a canonical matrix by (row block, column), both
// stable: returns ord, the tile-head flags hd and their exclusive scan hx.
int tile_order(Plan& p, const int32_t* col, const int32_t* row_of, int64_t n, int64_t k, int64_t nrb,
               DevBuf& ord, DevBuf& hd, DevBuf& hx, DevBuf& total, hipStream_t s) {
    Allocator& al = p.al;
    DevBuf keys, ktmp, vtmp;
    HSPMM_TRY(al.alloc(ord, std::max<int64_t>(1, n) * 4));
    HSPMM_TRY(al.alloc(hd, std::max<int64_t>(1, n) * 4));
    HSPMM_TRY(al.alloc(hx, std::max<int64_t>(1, n) * 4));
    HSPMM_TRY(al.alloc(total, 4));
    HSPMM_TRY(al.alloc(keys, std::max<int64_t>(1, n) * 4));
    HSPMM_TRY(al.alloc(ktmp, std::max<int64_t>(1, n) * 4));
    HSPMM_TRY(al.alloc(vtmp, std::max<int64_t>(1, n) * 4));
    HSPMM_TRY(iota_i32(ord.as<int32_t>(), n, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_copy_u32_from_i32, dim3(grid_for(n)), dim3(kThreads), 0, s, keys.as<uint32_t>(),
                           col, n);
        HIP_LAUNCH_CHECK();
        HSPMM_TRY(radix_sort_pairs(keys.as<uint32_t>(), ord.as<int32_t>(), ktmp.as<uint32_t>(),
                                   vtmp.as<int32_t>(), n, bits_for(k - 1), al, s));
        hipLaunchKernelGGL(k_gather_rb_key, dim3(grid_for(n)), dim3(kThreads), 0, s, keys.as<uint32_t>(), row_of,
                           ord.as<int32_t>(), n);
        HIP_LAUNCH_CHECK();
        HSPMM_TRY(radix_sort_pairs(keys.as<uint32_t>(), ord.as<int32_t>(), ktmp.as<uint32_t>(),
                                   vtmp.as<int32_t>(), n, bits_for(nrb - 1), al, s));
        hipLaunchKernelGGL(k_tile_heads, dim3(grid_for(n)), dim3(kThreads), 0, s, ord.as<int32_t>(), row_of, col,
                           n, hd.as<int32_t>());
        HIP_LAUNCH_CHECK();
    }
    HSPMM_TRY(scan_exclusive_i32(hd.as<int32_t>(), hx.as<int32_t>(), n, total.as<int32_t>(), al, s));
    al.free(keys);
    al.free(ktmp);
    al.free(vtmp);
    return HSPMM_OK;
}

// Groups of row blocks sharing columns for the group kernels (FP32 / FP64
// BCSR-parts): built when staging is worth it -- at least 30 % of the tiles
// read a staged row and each staged row serves 1.5 tiles or more on
// average.  They are off by default (HSPMM_GROUPS unset or 0);
// HSPMM_GROUPS=-1 builds them when worth it, =1 keeps any grouping found;
// HSPMM_GROUP_UMAX / _GMAX override the stage size (rows) and the most row
// blocks per group.
int env_int(const char* name, int dflt) {
    const char* e = getenv(name);
    return (e && *e) ? atoi(e) : dflt;
}

int build_sub_groups(Plan& p, SubPlan& X, hipStream_t s) {
    Allocator& al = p.al;
    X.grouped = false;
    // off unless asked for: on the block stencil and the sweep's block-
    // diagonal matrices the staged kernel measured slower than the one-wave
    // walk it replaces (stencil FP32 forward 46.8 against 38.6 us)
    const int mode = env_int("HSPMM_GROUPS", 0);
    if (mode == 0 || X.rb_bcsr == 0) return HSPMM_OK;
    if (X.ct != HSPMM_F32 && X.ct != HSPMM_F64) return HSPMM_OK;
    std::vector<int32_t> h_col;
    HSPMM_TRY(download(h_col, X.blk_col.ptr, (size_t)X.nblk_pad, s));
    GroupParams prm;
    prm.u_max = env_int("HSPMM_GROUP_UMAX", kGroupStageRows);
    prm.g_max = env_int("HSPMM_GROUP_GMAX", kGroupMaxBlocks);
    if (prm.u_max < 1 || prm.u_max > kGroupStageRowsMax || prm.g_max < 1) return HSPMM_OK;
    // the group kernel reads every B operand from the stage: a row block
    // with more columns than a stage holds keeps the plan ungrouped
    if (X.max_rb_tiles > prm.u_max) return HSPMM_OK;
    prm.stage_all = true;
    Groups gr;
    build_groups(X.h_blk_ptr, X.h_blk_cnt, h_col, X.nblk_pad, X.k, prm, gr);
    int64_t urows = (int64_t)gr.ucol.size();
    // every tile reads the stage: worth it when the stage saves a third of
    // the row fetches (a staged row serves 1.5 tiles or more on average)
    const bool worth = gr.staged_tiles * 2 >= urows * 3;
    if (!(mode == 1 ? gr.staged_tiles > 0 : worth)) return HSPMM_OK;
    const int64_t ns = X.rb_bcsr;
    std::vector<int32_t> krb(ns), kptr(ns), kcnt(ns);
    for (int64_t i = 0; i < ns; ++i) {
        const int32_t o = gr.order[i];
        krb[i] = X.h_bcsr_rb[o];
        kptr[i] = X.h_blk_ptr[o];
        kcnt[i] = X.h_blk_cnt[o];
    }
    HSPMM_TRY(upload(al, X.kslot_rb, krb, s));
    HSPMM_TRY(upload(al, X.kslot_ptr, kptr, s));
    HSPMM_TRY(upload(al, X.kslot_cnt, kcnt, s));
    HSPMM_TRY(upload(al, X.grp_ptr, gr.grp_ptr, s));
    HSPMM_TRY(upload(al, X.grp_uptr, gr.u_ptr, s));
    HSPMM_TRY(upload(al, X.grp_ucol, gr.ucol, s));
    HSPMM_TRY(upload(al, X.blk_bsrc, gr.bsrc, s));
    HIP_TRY(hipStreamSynchronize(s));
    X.h_order = gr.order;
    X.ngroups = gr.ngroups();
    X.grp_max_u = gr.max_u;
    X.grp_staged = gr.staged_tiles;
    X.grp_union = urows;
    X.grouped = true;
    return HSPMM_OK;
}

// Build one sub-plan from a canonical CSR (device rp[m+1], col, row_of) whose
// entry x stands for A's canonical entry src[x] (src null = identity).
int build_sub(Plan& p, SubPlan& X, const int32_t* rp, const int32_t* col, const int32_t* row_of,
              const int32_t* src, hipStream_t s, int split_override = -1, int64_t r_override = -1) {
    Allocator& al = p.al;
    const int64_t m = X.m, n = X.nnz;
    const int br = X.br;
    X.nrb = ceil_div(m, br);
    const int64_t nrb = X.nrb;
    const bool half = X.ct == HSPMM_F16 || X.ct == HSPMM_BF16;

    std::vector<int32_t> h_rp;
    HSPMM_TRY(download(h_rp, rp, (size_t)m + 1, s));
    X.h_rb_nnz.assign(nrb, 0);
    for (int64_t q = 0; q < nrb; ++q) X.h_rb_nnz[q] = h_rp[std::min<int64_t>(m, q * br + br)] - h_rp[q * br];

    const int split = split_override >= 0 ? split_override : p.opts.split;
    const bool need_tiles = split != HSPMM_SPLIT_CSR_ONLY && n > 0;
    DevBuf ord, hd, hx, total;
    X.h_rb_nblk.assign(nrb, 0);
    if (need_tiles) {
        HSPMM_TRY(tile_order(p, col, row_of, n, X.k, nrb, ord, hd, hx, total, s));
        DevBuf dn;
        HSPMM_TRY(al.alloc(dn, std::max<int64_t>(1, nrb) * 4));
        hipLaunchKernelGGL(k_rb_nblk, dim3(grid_for(nrb)), dim3(kThreads), 0, s, rp, hx.as<int32_t>(),
                           total.as<int32_t>(), m, nrb, n, dn.as<int32_t>());
        HIP_LAUNCH_CHECK();
        HSPMM_TRY(download(X.h_rb_nblk, dn.ptr, (size_t)nrb, s));
        al.free(dn);
    }

    // ---- cost model: class of every row block ----
    const int sv = (int)dtype_size(X.ct), sb = sv;
    const int64_t nh = p.opts.n_hint > 0 ? p.opts.n_hint : 128;
    std::vector<uint8_t> auto_cls;
    double t_c = 0, t_b = 0;
    choose_auto(p.mm, X.h_rb_nnz, X.h_rb_nblk, nh, sv, sb, br, X.kc, auto_cls, t_c, t_b);
    X.h_cls.assign(nrb, 0);
    // the whole matrix in either part: the aggregate throughputs of Eq. 1
    X.pred_all_csr = X.pred_all_bcsr = 0;
    for (int64_t q = 0; q < nrb; ++q) {
        RowBlockCost c = rowblock_cost(p.mm, X.h_rb_nnz[q], X.h_rb_nblk[q], nh, sv, sb, br, X.kc);
        X.pred_all_csr += c.t_csr;
        X.pred_all_bcsr += c.t_bcsr;
    }
    if (split == HSPMM_SPLIT_AUTO) {
        X.h_cls = auto_cls;
    } else if (split == HSPMM_SPLIT_BCSR_ONLY) {
        X.h_cls.assign(nrb, 1);
    } else if (split == HSPMM_SPLIT_BOUNDARY) {
        int64_t rbd = r_override >= 0 ? r_override : p.opts.r_boundary;
        if (&X == &p.T || rbd < 0) {
            // Eq. 1: the aggregate throughput of each part is m / (its
            // predicted time for the whole matrix)
            const double tpc = X.pred_all_csr > 0 ? (double)m / X.pred_all_csr : 1.0;
            const double tpb = X.pred_all_bcsr > 0 ? (double)m / X.pred_all_bcsr : 1.0;
            rbd = eq1_boundary(m, tpc, 1.0, tpb, 1.0, br);
        }
        if (rbd > m) rbd = m;
        if (rbd % br != 0 && rbd != m) return fail(HSPMM_ERR_ARG, "r_boundary must be a multiple of block_rows");
        X.r_boundary = rbd;
        for (int64_t q = 0; q < nrb; ++q) X.h_cls[q] = (q * br >= rbd) ? 1 : 0;
    }
    if (!need_tiles) X.h_cls.assign(nrb, 0);
    // predicted times of the chosen split (reported in plan_info)
    X.pred_csr = X.pred_bcsr = 0;
    for (int64_t q = 0; q < nrb; ++q) {
        RowBlockCost c = rowblock_cost(p.mm, X.h_rb_nnz[q], X.h_rb_nblk[q], nh, sv, sb, br, X.kc);
        if (X.h_cls[q]) X.pred_bcsr += c.t_bcsr; else X.pred_csr += c.t_csr;
    }

    // ---- CSR-part lists ----
    // Counts on the host from the row pointer it holds; the lists themselves
    // are built on the device (no host arrays of the row count, no uploads).
    int64_t nrows_c = 0, nnz_c = 0;
    for (int64_t q = 0; q < nrb; ++q) {
        if (X.h_cls[q]) continue;
        const int64_t r1 = std::min<int64_t>(m, q * br + br);
        nrows_c += r1 - q * br;
        nnz_c += h_rp[r1] - h_rp[q * br];
    }
    X.rows_csr = nrows_c;
    X.nnz_csr = nnz_c;
    // virtual rows: rows longer than `seg` entries are cut into segments whose
    // partial rows are summed in order by a second kernel.  A lane group walks
    // its segment in dependent rounds of gathers, so a long segment is a long
    // critical path when the CSR-part has too little work to hide it: the
    // segment length shrinks (256 down to 32) until the CSR-part holds about
    // kSegTarget segments' worth of entries.
    constexpr int64_t kSegTarget = 16384;
    int32_t seg = X.seg;
    if (seg <= 0) {
        seg = 256;
        while (seg > 32 && X.nnz_csr < (int64_t)seg * kSegTarget) seg >>= 1;
    }
    X.seg = seg;
    int64_t nv = 0, nlong = 0, nparts = 0;
    int32_t maxlc = 0;
    for (int64_t q = 0; q < nrb; ++q) {
        if (X.h_cls[q]) continue;
        for (int64_t r = q * br; r < std::min<int64_t>(m, q * br + br); ++r) {
            const int32_t len = h_rp[r + 1] - h_rp[r];
            if (len > seg) {
                const int32_t ns = (len + seg - 1) / seg;
                nv += ns;
                nparts += ns;
                ++nlong;
                maxlc = std::max(maxlc, ns);
            } else {
                ++nv;
            }
        }
    }
    X.n_vrows = nv;
    X.n_long = nlong;
    X.n_partials = nparts;
    X.max_long_cnt = maxlc;
    HSPMM_TRY(al.alloc(X.csr_rows, std::max<int64_t>(1, nrows_c) * 4));
    HSPMM_TRY(al.alloc(X.csr_ptr, ((size_t)nrows_c + 1) * 4));
    HSPMM_TRY(al.alloc(X.vr_start, std::max<int64_t>(1, nv) * 4));
    HSPMM_TRY(al.alloc(X.vr_end, std::max<int64_t>(1, nv) * 4));
    HSPMM_TRY(al.alloc(X.vr_out, std::max<int64_t>(1, nv) * 4));
    HSPMM_TRY(al.alloc(X.vr_row, std::max<int64_t>(1, nv) * 4));
    HSPMM_TRY(al.alloc(X.long_row, std::max<int64_t>(1, nlong) * 4));
    HSPMM_TRY(al.alloc(X.long_first, std::max<int64_t>(1, nlong) * 4));
    HSPMM_TRY(al.alloc(X.long_cnt, std::max<int64_t>(1, nlong) * 4));
    HSPMM_TRY(fill_i32(X.csr_ptr.as<int32_t>(), 0, 1, s));
    if (nrows_c > 0) {
        // per row: in the CSR-part, its entries, virtual rows, long or not,
        // partial slots; their exclusive sums place every list entry.  One
        // list in row order, a long row's segments in its place: each XCD
        // takes a contiguous range of the list, so any cluster of long rows
        // (all of them first, say) would load one XCD with most of the work;
        // neighbouring rows also share gathered rows of B
        DevBuf d_cls, cnt, pre;
        std::vector<uint8_t> cls8(X.h_cls.begin(), X.h_cls.end());
        HSPMM_TRY(upload(al, d_cls, cls8, s));
        HSPMM_TRY(al.alloc(cnt, (size_t)5 * m * 4));
        HSPMM_TRY(al.alloc(pre, (size_t)5 * m * 4));
        int32_t* c = cnt.as<int32_t>();
        int32_t* x = pre.as<int32_t>();
        hipLaunchKernelGGL(k_wl_counts, dim3(grid_for(m)), dim3(kThreads), 0, s, rp,
                           static_cast<const uint8_t*>(d_cls.ptr), m, br, seg, c);
        HIP_LAUNCH_CHECK();
        for (int f = 0; f < 5; ++f) HSPMM_TRY(scan_exclusive_i32(c + f * m, x + f * m, m, nullptr, al, s));
        DevBuf vs, ve, vo, vrow;
        HSPMM_TRY(al.alloc(vs, std::max<int64_t>(1, nv) * 4));
        HSPMM_TRY(al.alloc(ve, std::max<int64_t>(1, nv) * 4));
        HSPMM_TRY(al.alloc(vo, std::max<int64_t>(1, nv) * 4));
        HSPMM_TRY(al.alloc(vrow, std::max<int64_t>(1, nv) * 4));
        hipLaunchKernelGGL(k_wl_fill, dim3(grid_for(m)), dim3(kThreads), 0, s, rp, c, x, m, seg, nrows_c,
                           X.csr_rows.as<int32_t>(), X.csr_ptr.as<int32_t>(), vs.as<int32_t>(), ve.as<int32_t>(),
                           vo.as<int32_t>(), vrow.as<int32_t>(), X.long_row.as<int32_t>(),
                           X.long_first.as<int32_t>(), X.long_cnt.as<int32_t>());
        HIP_LAUNCH_CHECK();
        // A lane group takes one virtual row and a wave as many as it has
        // lane groups, so a wave runs as long as its longest row.  Within
        // windows of consecutive virtual rows, order them by length class
        // floor(log2 len), longest first and stable: the rows of a wave then
        // have lengths within a factor of two, rows of one class keep their
        // order (and the B rows neighbouring rows share), and a window spans
        // at most 1/32 of the list so every XCD's contiguous range keeps its
        // share of long rows.  Measured: power law FP16 fwd+bwd 2.05 -> 3.6
        // TFLOP/s, GCN 4.1 -> 4.5, block stencil unchanged (one length
        // class); a sort over the whole list clusters the long rows on one
        // XCD (3x slower), exact lengths break the stencil's row order
        // (CSR-part 15 % slower).  One stable radix sort on the key
        // (window, 31 - class).
#ifndef HSPMM_SORT_WINDOW
#define HSPMM_SORT_WINDOW 8192
#endif
        int64_t window = HSPMM_SORT_WINDOW;
        while (window > 64 && window * 32 > nv) window >>= 1;
        DevBuf keys, idx, ktmp, itmp;
        HSPMM_TRY(al.alloc(keys, (size_t)nv * 4));
        HSPMM_TRY(al.alloc(idx, (size_t)nv * 4));
        HSPMM_TRY(al.alloc(ktmp, (size_t)nv * 4));
        HSPMM_TRY(al.alloc(itmp, (size_t)nv * 4));
        HSPMM_TRY(iota_i32(idx.as<int32_t>(), nv, s));
        hipLaunchKernelGGL(k_wl_keys, dim3(grid_for(nv)), dim3(kThreads), 0, s, vs.as<int32_t>(), ve.as<int32_t>(),
                           nv, (int32_t)window, keys.as<uint32_t>());
        HIP_LAUNCH_CHECK();
        HSPMM_TRY(radix_sort_pairs(keys.as<uint32_t>(), idx.as<int32_t>(), ktmp.as<uint32_t>(),
                                   itmp.as<int32_t>(), nv, bits_for((nv - 1) / window) + 5, al, s));
        hipLaunchKernelGGL(k_wl_gather, dim3(grid_for(nv)), dim3(kThreads), 0, s, idx.as<int32_t>(), nv,
                           vs.as<int32_t>(), ve.as<int32_t>(), vo.as<int32_t>(), vrow.as<int32_t>(),
                           X.vr_start.as<int32_t>(), X.vr_end.as<int32_t>(), X.vr_out.as<int32_t>(),
                           X.vr_row.as<int32_t>());
        HIP_LAUNCH_CHECK();
    }
    HSPMM_TRY(al.alloc(X.csr_col, std::max<int64_t>(1, X.nnz_csr) * 4));
    HSPMM_TRY(al.alloc(X.csr_src, std::max<int64_t>(1, X.nnz_csr) * 4));
    HSPMM_TRY(al.alloc(X.csr_val, std::max<int64_t>(1, X.nnz_csr) * dtype_size(X.ct)));
    if (X.rows_csr > 0) {
        hipLaunchKernelGGL(k_build_csr, dim3(grid_waves(X.rows_csr)), dim3(kThreads), 0, s,
                           X.csr_rows.as<int32_t>(), X.csr_ptr.as<int32_t>(), X.rows_csr, rp, col, src,
                           X.csr_col.as<int32_t>(), X.csr_src.as<int32_t>());
        HIP_LAUNCH_CHECK();
    }

    // ---- BCSR-part lists (host) ----
    X.h_bcsr_rb.clear();
    X.h_blk_cnt.clear();
    X.h_blk_ptr.assign(1, 0);
    std::vector<int32_t> rb_slot(nrb, -1);
    int64_t pad_acc = 0;
    X.nblk = 0;
    X.nchunks = 0;
    X.max_rb_tiles = 0;
    X.nnz_bcsr = 0;
    for (int64_t q = 0; q < nrb; ++q) {
        if (!X.h_cls[q]) continue;
        rb_slot[q] = (int32_t)X.h_bcsr_rb.size();
        X.h_bcsr_rb.push_back((int32_t)q);
        X.h_blk_cnt.push_back(X.h_rb_nblk[q]);
        X.max_rb_tiles = std::max<int64_t>(X.max_rb_tiles, X.h_rb_nblk[q]);
        X.nblk += X.h_rb_nblk[q];
        X.nnz_bcsr += X.h_rb_nnz[q];
        pad_acc += ceil_div(X.h_rb_nblk[q], X.kc) * X.kc;
        if (pad_acc * 16 >= (int64_t(1) << 31)) return fail(HSPMM_ERR_OVERFLOW, "padded tile slots exceed 2^31");
        X.h_blk_ptr.push_back((int32_t)pad_acc);
    }
    X.rb_bcsr = (int64_t)X.h_bcsr_rb.size();
    X.nblk_pad = pad_acc;
    HSPMM_TRY(upload(al, X.bcsr_rb, X.h_bcsr_rb, s));
    HSPMM_TRY(upload(al, X.blk_ptr, X.h_blk_ptr, s));
    HSPMM_TRY(upload(al, X.blk_cnt, X.h_blk_cnt, s));
    HSPMM_TRY(al.alloc(X.blk_col, std::max<int64_t>(1, X.nblk_pad) * 4));
    HSPMM_TRY(al.alloc(X.blk_src, std::max<int64_t>(1, X.nblk_pad * 16) * 4));
    HSPMM_TRY(al.alloc(X.blk_val, std::max<int64_t>(1, X.nblk_pad * 16) * dtype_size(X.ct)));
    if (X.rb_bcsr > 0) {
        DevBuf d_slot;
        HSPMM_TRY(upload(al, d_slot, rb_slot, s));
        HSPMM_TRY(fill_i32(X.blk_col.as<int32_t>(), 0, X.nblk_pad, s));
        HSPMM_TRY(fill_i32(X.blk_src.as<int32_t>(), -1, X.nblk_pad * 16, s));
        hipLaunchKernelGGL(k_build_bcsr, dim3(grid_for(n)), dim3(kThreads), 0, s, ord.as<int32_t>(),
                           hd.as<int32_t>(), hx.as<int32_t>(), row_of, col, src, rp, d_slot.as<int32_t>(),
                           X.blk_ptr.as<int32_t>(), n, half, X.blk_col.as<int32_t>(), X.blk_src.as<int32_t>());
        HIP_LAUNCH_CHECK();
        if (&X == &p.A) {
            DevBuf mask;
            HSPMM_TRY(al.alloc(mask, (size_t)X.nblk_pad * 2));
            hipLaunchKernelGGL(k_build_mask, dim3(grid_for(X.nblk_pad)), dim3(kThreads), 0, s,
                               X.blk_src.as<int32_t>(), X.nblk_pad, half, static_cast<uint16_t*>(mask.ptr));
            HIP_LAUNCH_CHECK();
            std::vector<int32_t> cptr(1, 0);
            for (int32_t c : X.h_blk_cnt) cptr.push_back(cptr.back() + (int32_t)ceil_div(c, 16));
            X.nchunks = cptr.back();
            HSPMM_TRY(upload(al, X.chunk_ptr, cptr, s));
            HSPMM_TRY(al.alloc(X.chunk_base, (size_t)X.nchunks * 16 * 4));
            HSPMM_TRY(al.alloc(X.chunk_mask, (size_t)X.nchunks * 16 * 2));
            hipLaunchKernelGGL(k_build_chunk_meta, dim3(grid_for(X.rb_bcsr * 16)), dim3(kThreads), 0, s,
                               X.bcsr_rb.as<int32_t>(), X.blk_ptr.as<int32_t>(), X.blk_cnt.as<int32_t>(),
                               static_cast<const uint16_t*>(mask.ptr), X.chunk_ptr.as<int32_t>(), rp, X.m,
                               X.rb_bcsr, X.ct == HSPMM_F64, X.chunk_base.as<int32_t>(),
                               static_cast<uint16_t*>(X.chunk_mask.ptr));
            HIP_LAUNCH_CHECK();
            HSPMM_TRY(sync_for_release(al, s));
            al.free(mask);
        }
        if (&X == &p.T && !half && X.nblk_pad > 0) {
            HSPMM_TRY(al.alloc(X.tile_base, (size_t)X.nblk_pad * 4));
            HSPMM_TRY(al.alloc(X.tile_mask, (size_t)X.nblk_pad * 2));
            hipLaunchKernelGGL(k_tile_meta, dim3(grid_for(X.nblk_pad)), dim3(kThreads), 0, s,
                               X.blk_src.as<int32_t>(), X.nblk_pad, X.tile_base.as<int32_t>(),
                               static_cast<uint16_t*>(X.tile_mask.ptr));
            HIP_LAUNCH_CHECK();
        }
        HSPMM_TRY(sync_for_release(al, s));
        al.free(d_slot);
        HSPMM_TRY(build_sub_groups(p, X, s));
    }
    // host vectors of this function were copied to the device: wait before
    // they go out of scope (also the buffers below, unless kept for reuse)
    HIP_TRY(hipStreamSynchronize(s));
    al.free(ord);
    al.free(hd);
    al.free(hx);
    al.free(total);
    return HSPMM_OK;
}

template <class TO>
int pack_sub(Plan& p, SubPlan& X, const double* vb, int act, hipStream_t s) {
    const double* scale = X.scaled ? X.scale.as<double>() : nullptr;
    const double* a_scale = p.A.scaled ? p.A.scale.as<double>() : nullptr;
    if (X.rows_csr > 0 && X.nnz_csr > 0) {
        hipLaunchKernelGGL(k_pack_csr<TO>, dim3(grid_waves(X.rows_csr)), dim3(kThreads), 0, s,
                           X.csr_rows.as<int32_t>(), X.csr_ptr.as<int32_t>(), X.rows_csr, X.csr_src.as<int32_t>(),
                           vb, scale, act, a_scale, p.row_of.as<int32_t>(), X.csr_val.as<TO>());
        HIP_LAUNCH_CHECK();
    }
    if (X.rb_bcsr > 0) {
        hipLaunchKernelGGL(k_pack_bcsr<TO>, dim3(grid_waves(X.rb_bcsr)), dim3(kThreads), 0, s,
                           X.bcsr_rb.as<int32_t>(), X.blk_ptr.as<int32_t>(), X.rb_bcsr, X.blk_src.as<int32_t>(),
                           vb, scale, act, a_scale, p.row_of.as<int32_t>(), X.blk_val.as<TO>());
        HIP_LAUNCH_CHECK();
    }
    return HSPMM_OK;
}

int pack_sub_any(Plan& p, SubPlan& X, const double* vb, int act, hipStream_t s) {
    switch (X.ct) {
        case HSPMM_F64: return pack_sub<double>(p, X, vb, act, s);
        case HSPMM_F32: return pack_sub<float>(p, X, vb, act, s);
        case HSPMM_F16: return pack_sub<half_t>(p, X, vb, act, s);
        case HSPMM_BF16: return pack_sub<bf16_t>(p, X, vb, act, s);
        default: return fail(HSPMM_ERR_DTYPE, "bad compute dtype");
    }
}

}  // namespace

// vb[c]: the canonical values of A in FP64 (duplicates summed in input order)
int canonical_values(Plan& p, const void* vals, int vals_dtype, DevBuf& vb, hipStream_t s) {
    HSPMM_TRY(p.al.alloc(vb, (size_t)p.nnz * 8));
    const int32_t* perm = p.canonical ? nullptr : p.perm.as<int32_t>();
    const int32_t* seg = p.canonical ? nullptr : p.seg.as<int32_t>();
    const unsigned g = grid_for(p.nnz);
    switch (vals_dtype) {
        case HSPMM_F64: hipLaunchKernelGGL(k_base_values<double>, dim3(g), dim3(kThreads), 0, s, vals, perm, seg, p.nnz, vb.as<double>()); break;
        case HSPMM_F32: hipLaunchKernelGGL(k_base_values<float>, dim3(g), dim3(kThreads), 0, s, vals, perm, seg, p.nnz, vb.as<double>()); break;
        case HSPMM_F16: hipLaunchKernelGGL(k_base_values<half_t>, dim3(g), dim3(kThreads), 0, s, vals, perm, seg, p.nnz, vb.as<double>()); break;
        case HSPMM_BF16: hipLaunchKernelGGL(k_base_values<bf16_t>, dim3(g), dim3(kThreads), 0, s, vals, perm, seg, p.nnz, vb.as<double>()); break;
        default: return fail(HSPMM_ERR_DTYPE, "bad vals dtype");
    }
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}

// the power-of-two scales (scaled sub-plans) and the packed values of one
// of A's sub-plans
int pack_a_like(Plan& p, SubPlan& X, const double* vb, hipStream_t s) {
    if (X.scaled) {
        hipLaunchKernelGGL(k_rb_scale, dim3(grid_waves(X.nrb)), dim3(kThreads), 0, s, p.canon_rp.as<int32_t>(), vb,
                           p.m, X.nrb, X.scale.as<double>());
        HIP_LAUNCH_CHECK();
    }
    return pack_sub_any(p, X, vb, -1, s);
}

int pack_values(Plan& p, const void* vals, int vals_dtype, hipStream_t s) {
    if (p.nnz == 0) return HSPMM_OK;
    DevBuf vb;
    HSPMM_TRY(canonical_values(p, vals, vals_dtype, vb, s));
    HSPMM_TRY(pack_a_like(p, p.A, vb.as<double>(), s));
    if (p.has_T) HSPMM_TRY(pack_sub_any(p, p.T, vb.as<double>(), p.compute, s));
    HSPMM_TRY(sync_for_release(p.al, s));
    p.al.free(vb);
    return HSPMM_OK;
}

// Seconds per forward product of the whole matrix in one part (CSR_ONLY or
// BCSR_ONLY) at width n_hint: a temporary sub-plan of A in that split,
// packed, run twice to warm up and timed over five launches on a zero B.
int time_whole_part(Plan& p, const SubPlan& like, int split, const int32_t* rp, const int32_t* col,
                    const double* vb, hipStream_t s, double* secs) {
    SubPlan X;
    X.ct = like.ct;
    X.m = like.m;
    X.k = like.k;
    X.nnz = like.nnz;
    X.br = like.br;
    X.kc = like.kc;
    X.scaled = like.scaled;
    HSPMM_TRY(build_sub(p, X, rp, col, p.row_of.as<int32_t>(), nullptr, s, split));
    if (X.scaled) HSPMM_TRY(p.al.alloc(X.scale, std::max<int64_t>(1, X.nrb) * 8));
    HSPMM_TRY(pack_a_like(p, X, vb, s));
    const int64_t n = std::max<int32_t>(1, p.opts.n_hint);
    const size_t eb = dtype_size(X.ct), ec = dtype_size(out_dtype(X.ct));
    DevBuf B, C;
    HSPMM_TRY(p.al.alloc(B, (size_t)std::max<int64_t>(1, X.k) * n * eb));
    HSPMM_TRY(p.al.alloc(C, (size_t)std::max<int64_t>(1, X.m) * n * ec));
    HSPMM_TRY(fill_i32(B.as<int32_t>(), 0, (int64_t)(B.bytes / 4), s));
    for (int i = 0; i < 2; ++i) HSPMM_TRY(launch_forward(p, X, n, B.ptr, n, C.ptr, n, s));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    constexpr int reps = 5;
    int rc = HSPMM_OK;
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps && rc == HSPMM_OK; ++i) rc = launch_forward(p, X, n, B.ptr, n, C.ptr, n, s);
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (rc == HSPMM_OK) {
        hipError_t e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) rc = hip_fail(e, "timing a part", __FILE__, __LINE__);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HSPMM_TRY(rc);
    HIP_TRY(hipStreamSynchronize(s));
    *secs = (double)ms * 1e-3 / reps;
    return HSPMM_OK;
}

int build_plan(Plan& p, const int32_t* row_ptr, const int32_t* col_idx, const void* vals, int vals_dtype,
               hipStream_t s) {
    Allocator& al = p.al;
    // the build's temporaries are reused in stream order, and freed at its
    // end (constructed before them, so destroyed after them)
    KeepBuffers keep(al);
    const int64_t m = p.m, nin = p.nnz_in;

    DevBuf flags;
    HSPMM_TRY(al.alloc(flags, 4));
    HIP_TRY(hipMemsetAsync(flags.ptr, 0, 4, s));
    hipLaunchKernelGGL(k_check_rowptr, dim3(grid_for(m + 1)), dim3(kThreads), 0, s, row_ptr, m, nin,
                       flags.as<int32_t>());
    HIP_LAUNCH_CHECK();
    int32_t hflag = 0;
    HSPMM_TRY(read_flag(flags.as<int32_t>(), &hflag, s));
    if (hflag & FLAG_ROWPTR) return fail(HSPMM_ERR_CSR, "row_ptr is not a monotone 0..nnz sequence");

    DevBuf row_in;  // row of every input entry
    HSPMM_TRY(al.alloc(row_in, std::max<int64_t>(1, nin) * 4));
    if (nin > 0) {
        hipLaunchKernelGGL(k_expand_rows, dim3(grid_waves(m)), dim3(kThreads), 0, s, row_ptr, m,
                           row_in.as<int32_t>());
        HIP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_check_cols, dim3(grid_for(nin)), dim3(kThreads), 0, s, col_idx, row_in.as<int32_t>(),
                           nin, p.k, flags.as<int32_t>());
        HIP_LAUNCH_CHECK();
    }
    HSPMM_TRY(read_flag(flags.as<int32_t>(), &hflag, s));
    if (hflag & FLAG_COL) return fail(HSPMM_ERR_CSR, "column index out of range");
    p.canonical = !(hflag & FLAG_NONCANON);

    DevBuf& crp = p.canon_rp;
    DevBuf ccol;
    HSPMM_TRY(al.alloc(crp, ((size_t)m + 1) * 4));
    if (p.canonical) {
        p.nnz = nin;
        HSPMM_TRY(al.alloc(ccol, std::max<int64_t>(1, nin) * 4));
        HIP_TRY(hipMemcpyAsync(crp.ptr, row_ptr, ((size_t)m + 1) * 4, hipMemcpyDeviceToDevice, s));
        if (nin) HIP_TRY(hipMemcpyAsync(ccol.ptr, col_idx, (size_t)nin * 4, hipMemcpyDeviceToDevice, s));
        p.row_of = std::move(row_in);
    } else {
        // stable sort by column, then stable sort by row: row-major order with
        // duplicates adjacent in input order
        DevBuf keys, ktmp, vtmp, head, hx, total;
        HSPMM_TRY(al.alloc(p.perm, nin * 4));
        HSPMM_TRY(al.alloc(keys, nin * 4));
        HSPMM_TRY(al.alloc(ktmp, nin * 4));
        HSPMM_TRY(al.alloc(vtmp, nin * 4));
        HSPMM_TRY(iota_i32(p.perm.as<int32_t>(), nin, s));
        hipLaunchKernelGGL(k_copy_u32_from_i32, dim3(grid_for(nin)), dim3(kThreads), 0, s, keys.as<uint32_t>(),
                           col_idx, nin);
        HIP_LAUNCH_CHECK();
        HSPMM_TRY(radix_sort_pairs(keys.as<uint32_t>(), p.perm.as<int32_t>(), ktmp.as<uint32_t>(),
                                   vtmp.as<int32_t>(), nin, bits_for(p.k - 1), al, s));
        HSPMM_TRY(gather_key_shift(keys.as<uint32_t>(), row_in.as<int32_t>(), p.perm.as<int32_t>(), 0, nin, s));
        HSPMM_TRY(radix_sort_pairs(keys.as<uint32_t>(), p.perm.as<int32_t>(), ktmp.as<uint32_t>(),
                                   vtmp.as<int32_t>(), nin, bits_for(m - 1), al, s));
        al.free(keys);
        al.free(ktmp);
        al.free(vtmp);
        HSPMM_TRY(al.alloc(head, nin * 4));
        HSPMM_TRY(al.alloc(hx, nin * 4));
        HSPMM_TRY(al.alloc(total, 4));
        hipLaunchKernelGGL(k_mark_heads, dim3(grid_for(nin)), dim3(kThreads), 0, s, p.perm.as<int32_t>(),
                           row_in.as<int32_t>(), col_idx, nin, head.as<int32_t>());
        HIP_LAUNCH_CHECK();
        HSPMM_TRY(scan_exclusive_i32(head.as<int32_t>(), hx.as<int32_t>(), nin, total.as<int32_t>(), al, s));
        int32_t nc = 0;
        HSPMM_TRY(read_flag(total.as<int32_t>(), &nc, s));
        p.nnz = nc;
        HSPMM_TRY(al.alloc(p.seg, ((size_t)nc + 1) * 4));
        HSPMM_TRY(al.alloc(p.canon_of_orig, nin * 4));
        HSPMM_TRY(al.alloc(ccol, std::max<int32_t>(1, nc) * 4));
        HSPMM_TRY(al.alloc(p.row_of, std::max<int32_t>(1, nc) * 4));
        hipLaunchKernelGGL(k_canon_build, dim3(grid_for(nin)), dim3(kThreads), 0, s, p.perm.as<int32_t>(),
                           head.as<int32_t>(), hx.as<int32_t>(), row_in.as<int32_t>(), col_idx, nin,
                           p.canon_of_orig.as<int32_t>(), p.seg.as<int32_t>(), ccol.as<int32_t>(),
                           p.row_of.as<int32_t>());
        HIP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, p.seg.as<int32_t>() + nc, (int32_t)nin);
        HIP_LAUNCH_CHECK();
        // canonical row pointer from the run starts of the (sorted) rows
        if (nc > 0) {
            hipLaunchKernelGGL(k_row_starts, dim3(grid_for(m + 1)), dim3(kThreads), 0, s, p.row_of.as<int32_t>(),
                               (int64_t)nc, m, crp.as<int32_t>());
            HIP_LAUNCH_CHECK();
        } else {
            HSPMM_TRY(fill_i32(crp.as<int32_t>(), 0, m + 1, s));
        }
        HSPMM_TRY(sync_for_release(al, s));
        al.free(head);
        al.free(hx);
        al.free(total);
        al.free(row_in);
    }

    // ---- A's sub-plan ----
    SubPlan& A = p.A;
    A.ct = p.compute;
    A.m = m;
    A.k = p.k;
    A.nnz = p.nnz;
    A.br = p.br;
    A.kc = (p.compute == HSPMM_F16 || p.compute == HSPMM_BF16) ? 32 : 4;
    A.scaled = (p.compute == HSPMM_F16 || p.compute == HSPMM_BF16);
    int64_t r_meas = -1;
    if (p.opts.split == HSPMM_SPLIT_BOUNDARY && p.opts.r_boundary == HSPMM_R_MEASURED && p.nnz > 0) {
        // Eq. 1 with throughputs measured on this matrix (the paper's
        // warm-up runs): TP of a part = m / (time of the whole matrix in it)
        DevBuf vb;
        HSPMM_TRY(canonical_values(p, vals, vals_dtype, vb, s));
        HSPMM_TRY(time_whole_part(p, A, HSPMM_SPLIT_CSR_ONLY, crp.as<int32_t>(), ccol.as<int32_t>(), vb.as<double>(),
                                  s, &p.meas_csr));
        HSPMM_TRY(time_whole_part(p, A, HSPMM_SPLIT_BCSR_ONLY, crp.as<int32_t>(), ccol.as<int32_t>(),
                                  vb.as<double>(), s, &p.meas_bcsr));
        r_meas = eq1_boundary(m, p.meas_csr > 0 ? (double)m / p.meas_csr : 1.0, 1.0,
                              p.meas_bcsr > 0 ? (double)m / p.meas_bcsr : 1.0, 1.0, p.br);
    }
    HSPMM_TRY(build_sub(p, A, crp.as<int32_t>(), ccol.as<int32_t>(), p.row_of.as<int32_t>(), nullptr, s, -1,
                        r_meas));
    if (A.scaled) HSPMM_TRY(al.alloc(A.scale, std::max<int64_t>(1, A.nrb) * 8));

    // ---- transposed sub-plan for dB = A^T dC ----
    if (p.opts.want_backward) {
        SubPlan& T = p.T;
        T.ct = p.compute == HSPMM_F64 ? HSPMM_F64 : HSPMM_F32;
        T.m = p.k;
        T.k = m;
        T.nnz = p.nnz;
        T.br = p.br;
        T.kc = 4;
        T.scaled = false;
        DevBuf ord, keys, ktmp, vtmp, tcol, trow, trp;
        const int64_t nc = p.nnz;
        HSPMM_TRY(al.alloc(ord, std::max<int64_t>(1, nc) * 4));
        HSPMM_TRY(al.alloc(keys, std::max<int64_t>(1, nc) * 4));
        HSPMM_TRY(al.alloc(ktmp, std::max<int64_t>(1, nc) * 4));
        HSPMM_TRY(al.alloc(vtmp, std::max<int64_t>(1, nc) * 4));
        HSPMM_TRY(iota_i32(ord.as<int32_t>(), nc, s));
        if (nc > 0) {
            hipLaunchKernelGGL(k_copy_u32_from_i32, dim3(grid_for(nc)), dim3(kThreads), 0, s, keys.as<uint32_t>(),
                               ccol.as<int32_t>(), nc);
            HIP_LAUNCH_CHECK();
            HSPMM_TRY(radix_sort_pairs(keys.as<uint32_t>(), ord.as<int32_t>(), ktmp.as<uint32_t>(),
                                       vtmp.as<int32_t>(), nc, bits_for(p.k - 1), al, s));
        }
        al.free(keys);
        al.free(ktmp);
        al.free(vtmp);
        HSPMM_TRY(al.alloc(tcol, std::max<int64_t>(1, nc) * 4));
        HSPMM_TRY(al.alloc(trow, std::max<int64_t>(1, nc) * 4));
        HSPMM_TRY(al.alloc(trp, ((size_t)p.k + 1) * 4));
        if (nc > 0) {
            hipLaunchKernelGGL(k_transpose_fill, dim3(grid_for(nc)), dim3(kThreads), 0, s, ord.as<int32_t>(),
                               p.row_of.as<int32_t>(), ccol.as<int32_t>(), nc, tcol.as<int32_t>(),
                               trow.as<int32_t>());
            HIP_LAUNCH_CHECK();
            // trow is sorted (the entries in column order): A^T's row
            // pointer from its run starts, not from per-row counters (the
            // atomics of a counter pass collide on every long row)
            hipLaunchKernelGGL(k_row_starts, dim3(grid_for(p.k + 1)), dim3(kThreads), 0, s, trow.as<int32_t>(), nc,
                               p.k, trp.as<int32_t>());
            HIP_LAUNCH_CHECK();
        } else {
            HSPMM_TRY(fill_i32(trp.as<int32_t>(), 0, p.k + 1, s));
        }
        HSPMM_TRY(build_sub(p, T, trp.as<int32_t>(), tcol.as<int32_t>(), trow.as<int32_t>(), ord.as<int32_t>(), s));
        HIP_TRY(hipStreamSynchronize(s));
        p.has_T = true;
    }
    al.free(ccol);

    HSPMM_TRY(pack_values(p, vals, vals_dtype, s));

    // scratch for split rows (sized for n up to max(n_hint, 256)) and, for
    // non-canonical inputs, the canonical dA buffer
    const int64_t nmax = std::max<int64_t>(256, p.opts.n_hint);
    const size_t acc_b = p.compute == HSPMM_F64 ? 8 : 4;
    size_t need = (size_t)std::max(p.A.n_partials, p.has_T ? p.T.n_partials : 0) * nmax * acc_b;
    if (!p.canonical) need = std::max(need, (size_t)p.nnz * acc_b);
    HSPMM_TRY(ensure_ws(p, need));
    HIP_TRY(hipStreamSynchronize(s));
    return HSPMM_OK;
}

int64_t SubPlan::bytes() const {
    return (int64_t)(csr_rows.bytes + csr_ptr.bytes + csr_col.bytes + csr_val.bytes + csr_src.bytes +
                     vr_start.bytes + vr_end.bytes + vr_out.bytes + vr_row.bytes + long_row.bytes + long_first.bytes +
                     long_cnt.bytes + bcsr_rb.bytes + blk_ptr.bytes + blk_cnt.bytes + blk_col.bytes +
                     blk_val.bytes + blk_src.bytes + tile_base.bytes + tile_mask.bytes + chunk_ptr.bytes + chunk_base.bytes + chunk_mask.bytes +
                     scale.bytes);
}

}  // namespace hspmm
