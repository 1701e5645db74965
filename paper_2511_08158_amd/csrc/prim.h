// Device primitives used while building a plan: exclusive scan, stable LSD
// radix sort of (key, index) pairs, and small fill/gather helpers.  All are
// deterministic (integer atomics only count; no floating-point atomics).
#pragma once

#include "common.h"

namespace hspmm {

// out[i] = sum_{j<i} in[i]; *total (device int32, may be null) = sum of all.
// n < 2^31; the caller guarantees the sum fits in int32.
int scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total,
                       Allocator& al, hipStream_t s);

// Stable sort of (keys, vals) by bits [0, nbits) of the keys.  On return the
// sorted pairs are back in keys/vals.  tmp buffers hold n elements each.
int radix_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_tmp, int32_t* vals_tmp,
                     int64_t n, int nbits, Allocator& al, hipStream_t s);

int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
int iota_i32(int32_t* p, int64_t n, hipStream_t s);
// dst[i] = src[idx[i]]
int gather_u32(uint32_t* dst, const uint32_t* src, const int32_t* idx, int64_t n, hipStream_t s);
// keys[i] = src[idx[i]] >> shift
int gather_key_shift(uint32_t* dst, const int32_t* src, const int32_t* idx, int shift, int64_t n,
                     hipStream_t s);

inline int bits_for(int64_t maxval) {  // bits needed to represent values in [0, maxval]
    int b = 0;
    while (b < 63 && (int64_t(1) << b) <= maxval) ++b;
    return b;
}

}  // namespace hspmm
