// dA = SDDMM(dC, B) on A's pattern: dA[e] = <dC[row(e),:], B[col(e),:]>.
//
// CSR-part: the work list of the forward CSR kernel; a lane group holds its
// row of dC in registers, fetches one B row segment per entry and reduces
// the dot product across the group.
// BCSR-part: per row block, the 16 x n slab of dC times the gathered B rows
// of 16 tiles at a time is one 16 x 16 MFMA product (K = the n columns);
// only the slots that hold an entry of A are written.
#include "plan.h"
#include "prim.h"

namespace hspmm {

namespace {

struct SddArgs {
    // CSR-part
    const int32_t* vr_start;
    const int32_t* vr_end;
    const int32_t* vr_row;
    const int32_t* col;
    const int32_t* dst;    // canonical entry of each CSR-part entry
    int64_t n_vrows;
    // BCSR-part
    const int32_t* rb;
    const int32_t* blk_ptr;
    const int32_t* blk_cnt;
    const int32_t* blk_col;
    const int32_t* chunk_ptr;    // first chunk of 16 tiles of each row block
    const int32_t* chunk_base;   // [chunk][16] canonical index of each row's first entry in the chunk
    const uint16_t* chunk_mask;  // [chunk][16] tiles of the chunk that hold an entry of each row
    int64_t n_rb;
    // dense operands
    const void* B;
    int64_t ldb;
    const void* dC;
    int64_t lddc;
    int64_t n;
    int64_t m;
    void* dA;
};

// N elements converted to the accumulation type, in loads of at most 16
// bytes (callers guarantee the alignment of each chunk)
template <class T, int N>
__device__ inline void load_as(const T* p, typename Elem<T>::acc_t (&out)[N]) {
    if constexpr (N == 1) {
        out[0] = Elem<T>::to_acc(*p);
    } else {
        constexpr int C = (N * (int)sizeof(T) > 16) ? 16 / (int)sizeof(T) : N;
        typedef T V __attribute__((ext_vector_type(C)));
#pragma unroll
        for (int k = 0; k < N; k += C) {
            const V v = *reinterpret_cast<const V*>(p + k);
#pragma unroll
            for (int i = 0; i < C; ++i) out[k + i] = Elem<T>::to_acc(v[i]);
        }
    }
}

// TB = storage type of B; TG = dC / dA type (= accumulation type).
// U entries are reduced across the LPR lanes of a group together: each
// butterfly stage halves the number of partial sums a lane holds (one
// shuffle per pair), so U dot products cost U - 1 + log2(LPR / U) shuffles
// instead of U log2(LPR); afterwards lane gl holds the sum of entry
// (gl / (LPR / U)) of the batch.
template <class TB, class TG, int VEC, int LPR>
__device__ void sdd_csr_wave(const SddArgs& a, int64_t wave) {
    constexpr int R = 64 / LPR;
    constexpr int U = LPR < 16 ? LPR : 16;
    constexpr int SPAN = LPR / U;  // lanes that end with the same entry
#ifndef HSPMM_SDD_CSR_UB
#define HSPMM_SDD_CSR_UB 8
#endif
    constexpr int UB = U < HSPMM_SDD_CSR_UB ? U : HSPMM_SDD_CSR_UB;
    const int lane = threadIdx.x & 63;
    const int g = lane / LPR, gl = lane % LPR;
    if (wave * R >= a.n_vrows) return;
    const int64_t vr = wave * R + g;
    const bool act = vr < a.n_vrows;
    const int start = act ? a.vr_start[vr] : 0;
    const int len = act ? a.vr_end[vr] - start : 0;
    const int row = act ? a.vr_row[vr] : 0;
    int maxlen = len;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, o, 64));
    const TB* __restrict__ B = static_cast<const TB*>(a.B);
    const TG* __restrict__ dC = static_cast<const TG*>(a.dC);
    TG* __restrict__ dA = static_cast<TG*>(a.dA);
    const bool one_panel = a.n <= (int64_t)LPR * VEC;
    const int64_t col0 = (int64_t)gl * VEC;
    TG g0[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) g0[v] = TG(0);
    if (one_panel && act && col0 < a.n) load_as<TG, VEC>(dC + (int64_t)row * a.lddc + col0, g0);

    for (int base = 0; base < maxlen; base += LPR) {
        const bool eok = base + gl < len;
        const int e = start + base + gl;
        const int my_col = eok ? a.col[e] : -1;
        const int my_dst = eok ? a.dst[e] : -1;
        const int cnt = min(LPR, maxlen - base);
        for (int u0 = 0; u0 < cnt; u0 += U) {
            TG part[U];
#pragma unroll
            for (int uu = 0; uu < U; ++uu) part[uu] = TG(0);
            if (one_panel) {
                // UB gathers in flight, branch-free: an absent entry or a
                // lane past n reads row 0 / column 0 and its product is
                // dropped by a select
#pragma unroll
                for (int ub = 0; ub < U; ub += UB) {
                    TG bv[UB][VEC];
                    bool ok[UB];
#pragma unroll
                    for (int k = 0; k < UB; ++k) {
                        const int c = __shfl(my_col, (u0 + ub + k) & (LPR - 1), LPR);
                        ok[k] = c >= 0 && u0 + ub + k < cnt && col0 < a.n;
                        load_as<TB, VEC>(B + (int64_t)(ok[k] ? c : 0) * a.ldb + (col0 < a.n ? col0 : 0), bv[k]);
                    }
#pragma unroll
                    for (int k = 0; k < UB; ++k) {
                        TG dot = TG(0);
#pragma unroll
                        for (int v = 0; v < VEC; ++v) dot += g0[v] * bv[k][v];
                        part[ub + k] = ok[k] ? dot : TG(0);
                    }
                }
            } else {
                // several panels of LPR * VEC columns: every lane takes the
                // same number of panels (the shuffles need every lane of the
                // group active), a lane past n reads column 0 and its
                // products are dropped
                for (int64_t cb = 0; cb < a.n; cb += (int64_t)LPR * VEC) {
                    const int64_t c0 = cb + col0;
                    const bool cok = c0 < a.n;
                    TG gv[VEC];
                    load_as<TG, VEC>(dC + (int64_t)row * a.lddc + (cok ? c0 : 0), gv);
#pragma unroll
                    for (int ub = 0; ub < U; ub += UB) {
                        TG bv[UB][VEC];
                        bool ok[UB];
#pragma unroll
                        for (int k = 0; k < UB; ++k) {
                            const int c = __shfl(my_col, (u0 + ub + k) & (LPR - 1), LPR);
                            ok[k] = c >= 0 && u0 + ub + k < cnt && cok;
                            load_as<TB, VEC>(B + (int64_t)(ok[k] ? c : 0) * a.ldb + (cok ? c0 : 0), bv[k]);
                        }
#pragma unroll
                        for (int k = 0; k < UB; ++k) {
                            TG dot = TG(0);
#pragma unroll
                            for (int v = 0; v < VEC; ++v) dot += gv[v] * bv[k][v];
                            part[ub + k] += ok[k] ? dot : TG(0);
                        }
                    }
                }
            }
            // halving butterfly over the offsets LPR/2 .. SPAN
#pragma unroll
            for (int nv = U, o = LPR / 2; nv > 1; nv >>= 1, o >>= 1) {
                const bool up = (gl & o) != 0;
#pragma unroll
                for (int i = 0; i < nv / 2; ++i) {
                    const TG keep = up ? part[i + nv / 2] : part[i];
                    const TG send = up ? part[i] : part[i + nv / 2];
                    part[i] = keep + __shfl_xor(send, o, LPR);
                }
            }
#pragma unroll
            for (int o = SPAN / 2; o >= 1; o >>= 1) part[0] += __shfl_xor(part[0], o, LPR);
            const int idx = u0 + gl / SPAN;
            const int d = __shfl(my_dst, idx & (LPR - 1), LPR);
            const int c = __shfl(my_col, idx & (LPR - 1), LPR);
            if ((gl % SPAN) == 0 && idx < cnt && c >= 0) dA[d] = part[0];
        }
    }
}

__device__ inline f4_t mfma4(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline d4_t mfma4(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <class T> struct AccOf;
template <> struct AccOf<float> { typedef f4_t type; };
template <> struct AccOf<double> { typedef d4_t type; };
template <class T> __host__ __device__ constexpr int out_row(int g, int r) { return 4 * g + r; }
template <> __host__ __device__ constexpr int out_row<double>(int g, int r) { return g + 4 * r; }

// One workgroup per row block.  K of the MFMA runs over the n columns:
// lane (i, q) supplies columns kbase + q*VEC + v of dC row i and of B row j,
// so each of the VEC MFMAs of a step consumes one component.  When n fits in
// NKR steps the 16 x n slab of dC is staged once in LDS and read from there
// by all four waves at each step (holding it in registers instead costs
// NKR*VEC registers and with them occupancy); the row block's chunks of 16
// tiles are dealt to the waves round-robin (independent outputs, no
// reduction needed).
template <class TB, class TG, int VEC, int NKR>
__device__ void sdd_bcsr_wg(const SddArgs& a, int64_t slot, TG* lds) {
    typedef typename AccOf<TG>::type acc_v;
    if (slot >= a.n_rb) return;  // uniform over the workgroup
    const int lane = threadIdx.x & 63, w = wave_id(), j = lane & 15, q = lane >> 4;
    const int rb = a.rb[slot];
    const int b0 = a.blk_ptr[slot];
    const int cnt = a.blk_cnt[slot];
    const TB* __restrict__ B = static_cast<const TB*>(a.B);
    const TG* __restrict__ dC = static_cast<const TG*>(a.dC);
    TG* __restrict__ dA = static_cast<TG*>(a.dA);
    constexpr int STEP = 4 * VEC;
    constexpr int NMAX = NKR * STEP;
    constexpr int LDR = NMAX + 4;  // padded LDS row
    const int64_t arow = (int64_t)rb * 16 + j;
    const bool arow_ok = arow < a.m;
    const int nsteps = (int)ceil_div(a.n, STEP);
    const bool cached = nsteps <= NKR;
    if (cached) {
        // 16-byte chunks (the launcher's vector path guarantees 16-byte
        // aligned rows of dC and n a multiple of the chunk; LDS rows of
        // NMAX + 4 elements stay 16-byte aligned)
        constexpr int SV = VEC > 1 ? 16 / (int)sizeof(TG) : 1;
        for (int idx = threadIdx.x * SV; idx < 16 * NMAX; idx += 256 * SV) {
            const int i = idx / NMAX, c = idx - i * NMAX;
            const int64_t row = (int64_t)rb * 16 + i;
            TG v[SV];
            if (row < a.m && c < a.n) {
                load_as<TG, SV>(dC + row * a.lddc + c, v);
            } else {
#pragma unroll
                for (int e = 0; e < SV; ++e) v[e] = TG(0);
            }
#pragma unroll
            for (int e = 0; e < SV; ++e) lds[i * LDR + c + e] = v[e];
        }
        __syncthreads();
    }
    const TG* __restrict__ gl_row = lds + j * LDR + q * VEC;
#ifndef HSPMM_SDD_GATHER
#define HSPMM_SDD_GATHER 8
#endif
    // steps whose gathers are in flight together: 8 (a lane's 8 x 16-byte
    // gathers, every step of n = 128 FP32) at 52-56 registers; on the block
    // stencil 2-5 % faster than 4 (FP32 37.1 against 37.6 us, FP16 34.9
    // against 35.7) and 2 slower again.  With per-call destination ballots
    // the kernel needed 68 registers and 4 won by 9-17 %.
    constexpr int GB = (HSPMM_SDD_GATHER > 0 && HSPMM_SDD_GATHER < NKR) ? HSPMM_SDD_GATHER : NKR;
    static_assert(NKR % GB == 0, "gather batch must divide the cached steps");
    // this lane's rows out_row(q, r) sit at positions 4q + r of the chunk tables
    const int64_t chunk0 = a.chunk_ptr[slot];
    const uint32_t below = (1u << j) - 1u;
    for (int it0 = 0; 16 * w + 64 * it0 < cnt; it0 += 4) {
        // tile columns of this wave's next four chunks: lane l -> chunk it0 + l/16
        const int pre = 16 * w + 64 * (it0 + (lane >> 4)) + j;
        const int colreg = pre < cnt ? a.blk_col[b0 + pre] : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int it = it0 + k;
            const int c0 = 16 * w + 64 * it;
            if (c0 >= cnt) break;
            const int bc = __shfl(colreg, (16 * k + j) & 63, 64);
            const bool bok = c0 + j < cnt;
            // destinations: the first canonical index of each of the lane's
            // four rows in this chunk, and which tiles of the chunk hold them
            const int64_t ci = chunk0 + (c0 >> 4);
            const int4 cb = *reinterpret_cast<const int4*>(a.chunk_base + ci * 16 + 4 * q);
            const uint2 cm = *reinterpret_cast<const uint2*>(a.chunk_mask + ci * 16 + 4 * q);
            acc_v acc = acc_v{0, 0, 0, 0};
            if (cached) {
                // the gathers of GB steps first, then their products.  The
                // gathers are unconditional: a tile past the row block's end
                // reads row 0 of B (its results have no destination), and a
                // column past n reads column 0 against the zero padding of
                // the dC slab in LDS
                for (int s0 = 0; s0 < nsteps; s0 += GB) {
                    TG bv[GB][VEC];
#pragma unroll
                    for (int t = 0; t < GB; ++t) {
                        const int64_t c = (int64_t)(s0 + t) * STEP + q * VEC;
                        load_as<TB, VEC>(B + (int64_t)bc * a.ldb + (c < a.n ? c : 0), bv[t]);
                    }
#pragma unroll
                    for (int t = 0; t < GB; ++t) {
                        TG gv[VEC];
#pragma unroll
                        for (int v = 0; v < VEC; ++v) gv[v] = gl_row[(s0 + t) * STEP + v];
#pragma unroll
                        for (int v = 0; v < VEC; ++v) acc = mfma4(gv[v], bv[t][v], acc);
                    }
                }
            } else {
                for (int s = 0; s < nsteps; ++s) {
                    const int64_t c = (int64_t)s * STEP + q * VEC;
                    TG gv[VEC], bv[VEC];
                    if (arow_ok && c < a.n) {
                        load_as<TG, VEC>(dC + arow * a.lddc + c, gv);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v) gv[v] = TG(0);
                    }
                    if (bok && c < a.n) {
                        load_as<TB, VEC>(B + (int64_t)bc * a.ldb + c, bv);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v) bv[v] = TG(0);
                    }
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc = mfma4(gv[v], bv[v], acc);
                }
            }
            // lane (j, q) holds rows out_row(q, r) of tile c0 + j; the row's
            // entries in the chunk are consecutive in canonical order
            const int32_t base[4] = {cb.x, cb.y, cb.z, cb.w};
            const uint32_t bits[4] = {cm.x & 0xffffu, cm.x >> 16, cm.y & 0xffffu, cm.y >> 16};
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if ((bits[r] >> j) & 1u) dA[base[r] + __popc(bits[r] & below)] = acc[r];
        }
    }
}

// FP16 / BF16 row blocks on 16x16x32 MFMAs (K = 32 columns of n per step).
// The 16 x n slab of dC is staged in LDS in the compute type after an exact
// power-of-two scale s that puts its largest magnitude in [2^14, 2^15) (no
// FP16 overflow, and the FP16 normal range below it is kept), so the only
// change to dC is one rounding per element, as for B; products accumulate
// in FP32 and the results are multiplied back by s.  Lane (i, q) supplies
// dC row i and B row j of the step's columns 8q .. 8q + 7: one 16-byte LDS
// read and one 16-byte gather per step.  The launcher guarantees
// n <= 32 NKH, n a multiple of 8, 16-byte aligned rows of B and dC.
template <class T> struct Mfma32;
template <> struct Mfma32<half_t> {
    typedef h8_t v8;
    typedef _Float16 v4 __attribute__((ext_vector_type(4)));
    static __device__ f4_t run(v8 a, v8 b, f4_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <> struct Mfma32<bf16_t> {
    typedef b8_t v8;
    typedef __bf16 v4 __attribute__((ext_vector_type(4)));
    static __device__ f4_t run(v8 a, v8 b, f4_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <class TB, int NKH>
__device__ void sdd_bcsr_wg_h(const SddArgs& a, int64_t slot, unsigned char* smem) {
    typedef typename Mfma32<TB>::v8 v8;
    typedef typename Mfma32<TB>::v4 v4;
    if (slot >= a.n_rb) return;  // uniform over the workgroup
    constexpr int NMAX = 32 * NKH;
    constexpr int LDR = NMAX + 8;  // halfs per LDS row: rows stay 16-byte aligned
    constexpr int NV = NMAX / 64;  // float4 of the slab per thread
    TB* lds = reinterpret_cast<TB*>(smem);
    float* red = reinterpret_cast<float*>(smem + 16 * LDR * sizeof(TB));
    const int lane = threadIdx.x & 63, w = wave_id(), j = lane & 15, q = lane >> 4;
    const int rb = a.rb[slot];
    const int b0 = a.blk_ptr[slot];
    const int cnt = a.blk_cnt[slot];
    const TB* __restrict__ B = static_cast<const TB*>(a.B);
    const float* __restrict__ dC = static_cast<const float*>(a.dC);
    float* __restrict__ dA = static_cast<float*>(a.dA);
    f4_t x[NV];
    float mx = 0.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int idx = (threadIdx.x + 256 * v) * 4;
        const int i = idx / NMAX, c = idx - i * NMAX;
        const int64_t row = (int64_t)rb * 16 + i;
        x[v] = (row < a.m && c < a.n) ? *reinterpret_cast<const f4_t*>(dC + row * a.lddc + c) : f4_t{0.f, 0.f, 0.f, 0.f};
        mx = fmaxf(mx, fmaxf(fmaxf(fabsf(x[v][0]), fabsf(x[v][1])), fmaxf(fabsf(x[v][2]), fabsf(x[v][3]))));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) red[w] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    // mx in [2^(e-1), 2^e); a zero or non-finite slab is left unscaled.
    // e is held at -111 or above so that both 2^(15 - e) and 2^(e - 15)
    // are finite normal FP32 numbers: a slab below 2^-112 is scaled by
    // 2^126 only (its largest magnitude then stays below 2^14)
    int e = 0;
    (void)frexpf(mx, &e);
    e = e < -111 ? -111 : e;
    const bool scl = mx > 0.f && mx <= 3.4e38f;
    const float s = scl ? ldexpf(1.f, e - 15) : 1.f;
    const float inv = scl ? ldexpf(1.f, 15 - e) : 1.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int idx = (threadIdx.x + 256 * v) * 4;
        const int i = idx / NMAX, c = idx - i * NMAX;
        v4 hv;
#pragma unroll
        for (int t = 0; t < 4; ++t) hv[t] = (TB)(x[v][t] * inv);
        *reinterpret_cast<v4*>(lds + i * LDR + c) = hv;
    }
    __syncthreads();
    const TB* __restrict__ arow = lds + j * LDR + q * 8;
    const int64_t chunk0 = a.chunk_ptr[slot];
    const uint32_t below = (1u << j) - 1u;
    for (int it0 = 0; 16 * w + 64 * it0 < cnt; it0 += 4) {
        // tile columns of this wave's next four chunks: lane l -> chunk it0 + l/16
        const int pre = 16 * w + 64 * (it0 + (lane >> 4)) + j;
        const int colreg = pre < cnt ? a.blk_col[b0 + pre] : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c0 = 16 * w + 64 * (it0 + k);
            if (c0 >= cnt) break;
            const int bc = __shfl(colreg, (16 * k + j) & 63, 64);
            const int64_t ci = chunk0 + (c0 >> 4);
            const int4 cb = *reinterpret_cast<const int4*>(a.chunk_base + ci * 16 + 4 * q);
            const uint2 cm = *reinterpret_cast<const uint2*>(a.chunk_mask + ci * 16 + 4 * q);
            // unconditional gathers: a tile past the row block's end reads
            // row 0 of B, a step past n reads column 0 against zeros in LDS
            v8 bv[NKH];
#pragma unroll
            for (int t = 0; t < NKH; ++t) {
                const int64_t c = (int64_t)t * 32 + q * 8;
                bv[t] = *reinterpret_cast<const v8*>(B + (int64_t)bc * a.ldb + (c < a.n ? c : 0));
            }
            f4_t acc = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < NKH; ++t) {
                const v8 av = *reinterpret_cast<const v8*>(arow + t * 32);
                acc = Mfma32<TB>::run(av, bv[t], acc);
            }
            const int32_t base[4] = {cb.x, cb.y, cb.z, cb.w};
            const uint32_t bits[4] = {cm.x & 0xffffu, cm.x >> 16, cm.y & 0xffffu, cm.y >> 16};
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if ((bits[r] >> j) & 1u) dA[base[r] + __popc(bits[r] & below)] = acc[r] * s;
        }
    }
}

// DO_CSR / DO_BCSR compile out a part the plan does not have (register
// footprint of a one-part launch).
template <class TB, class TG, int VEC, int LPR, int BVEC, int NKR, bool DO_CSR, bool DO_BCSR>
__global__ __launch_bounds__(256) void k_sddmm(SddArgs a, uint32_t g_bcsr, uint32_t g_csr, int remap) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint32_t bid = blockIdx.x;
    const int w = wave_id();
    if (bid < g_bcsr) {
        if constexpr (DO_BCSR) {
            // BVEC 8: the FP16 / BF16 MFMA form, NKR steps of 32 columns
            if constexpr (BVEC == 8)
                sdd_bcsr_wg_h<TB, NKR>(a, (int64_t)xcd_remap(bid, g_bcsr, remap), lds_raw);
            else
                sdd_bcsr_wg<TB, TG, BVEC, NKR>(a, (int64_t)xcd_remap(bid, g_bcsr, remap),
                                               reinterpret_cast<TG*>(lds_raw));
        }
    } else {
        if constexpr (DO_CSR)
            sdd_csr_wave<TB, TG, VEC, LPR>(a, (int64_t)xcd_remap(bid - g_bcsr, g_csr, remap) * 4 + w);
    }
}

template <class TG>
__global__ void k_gather_dA(const TG* __restrict__ canon, const int32_t* __restrict__ idx, int64_t n,
                            TG* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = canon[idx[i]];
}

inline uint32_t pad8(int64_t g) { return (uint32_t)(ceil_div(g, 8) * 8); }

inline int lpr_for(int64_t n, int vec) {
    int64_t need = ceil_div(n, vec);
    int l = 4;
    while (l < 64 && l < need) l <<= 1;
    return l;
}

template <class TB, class TG, int VEC, int LPR, int BVEC, int NKR>
int launch_sdd(const SubPlan& X, SddArgs a, hipStream_t s, bool last) {
    constexpr int R = 64 / LPR;
    const int64_t csr_waves = ceil_div(X.n_vrows, R);
    const uint32_t g_csr = csr_waves ? pad8(ceil_div(csr_waves, 4)) : 0;
    const uint32_t g_bcsr = X.rb_bcsr ? pad8(X.rb_bcsr) : 0;
    if (g_csr + g_bcsr == 0) return HSPMM_OK;
    const size_t lds = !g_bcsr ? 0
                       : BVEC == 8 ? (size_t)16 * (NKR * 32 + 8) * 2 + 4 * sizeof(float)
                                   : (size_t)16 * (NKR * 4 * BVEC + 4) * sizeof(TG);
    const dim3 grid(g_bcsr + g_csr), block(256);
    const int rm = xcd_remap_mode();
    if (g_bcsr && g_csr && hybrid_launch_mode() == 2) {
        HSPMM_LAUNCH((k_sddmm<TB, TG, VEC, LPR, BVEC, NKR, false, true>), dim3(g_bcsr), block, lds, s, true, false, a,
                     g_bcsr, 0u, rm);
        HIP_LAUNCH_CHECK();
        HSPMM_LAUNCH((k_sddmm<TB, TG, VEC, LPR, BVEC, NKR, true, false>), dim3(g_csr), block, 0, s, false, last, a, 0u,
                     g_csr, rm);
    } else if (g_bcsr && g_csr) {
        HSPMM_LAUNCH((k_sddmm<TB, TG, VEC, LPR, BVEC, NKR, true, true>), grid, block, lds, s, true, last, a, g_bcsr,
                     g_csr, rm);
    } else if (g_csr) {
        HSPMM_LAUNCH((k_sddmm<TB, TG, VEC, LPR, BVEC, NKR, true, false>), grid, block, 0, s, true, last, a, g_bcsr,
                     g_csr, rm);
    } else {
        HSPMM_LAUNCH((k_sddmm<TB, TG, VEC, LPR, BVEC, NKR, false, true>), grid, block, lds, s, true, last, a, g_bcsr,
                     g_csr, rm);
    }
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}

#define HSPMM_LPR_SWITCH(LPRV, ...)                               \
    switch (LPRV) {                                               \
        case 4: { constexpr int LPR = 4; __VA_ARGS__; } break;   \
        case 8: { constexpr int LPR = 8; __VA_ARGS__; } break;   \
        case 16: { constexpr int LPR = 16; __VA_ARGS__; } break; \
        case 32: { constexpr int LPR = 32; __VA_ARGS__; } break; \
        default: { constexpr int LPR = 64; __VA_ARGS__; } break; \
    }

inline bool aligned(const void* p, size_t al) { return ((uintptr_t)p % al) == 0; }

// columns per lane of the FP16/BF16 SDDMM's CSR-part when rows of B allow
// 16-byte loads: 8 (16 bytes of B, 32 of dC per lane and entry).  Power
// law FP16 n = 64: dA 371 us against 415 at 4 columns
#ifndef HSPMM_SDD_H_VEC
#define HSPMM_SDD_H_VEC 8
#endif

}  // namespace

namespace {
// dA from canonical order to the input order of a non-canonical plan
int gather_dA(Plan& p, const DevBuf& ws, void* dA, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(p.nnz_in, 256), 65536);
    if (p.compute == HSPMM_F64) {
        HSPMM_LAUNCH(k_gather_dA<double>, dim3(g), dim3(256), 0, s, false, true, ws.as<double>(),
                     p.canon_of_orig.as<int32_t>(), p.nnz_in, static_cast<double*>(dA));
    } else {
        HSPMM_LAUNCH(k_gather_dA<float>, dim3(g), dim3(256), 0, s, false, true, ws.as<float>(),
                     p.canon_of_orig.as<int32_t>(), p.nnz_in, static_cast<float*>(dA));
    }
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}
}  // namespace

int launch_backward_fused(Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc, void* dB,
                          int64_t lddb, void* dA, hipStream_t s) {
    const size_t go = p.compute == HSPMM_F64 ? 8 : 4;
    void* target = dA;
    // (the plan's first scratch buffer may hold A^T's split-row partials)
    if (!p.canonical) {
        HSPMM_TRY(grow_buf(p, p.ws2, (size_t)p.nnz * go));
        target = p.ws2.ptr;
    }
    HSPMM_TRY(launch_bwd_fused_kernel(p, n, B, ldb, dC, lddc, dB, lddb, target, s, p.canonical));
    if (!p.canonical) HSPMM_TRY(gather_dA(p, p.ws2, dA, s));
    return HSPMM_OK;
}

int launch_sddmm(Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc, void* dA,
                 hipStream_t s, DevBuf* wsb) {
    SubPlan& X = p.A;
    if (p.nnz == 0) return HSPMM_OK;
    const size_t go = p.compute == HSPMM_F64 ? 8 : 4;
    void* target = dA;
    DevBuf& ws = wsb ? *wsb : p.ws;
    if (!p.canonical) {
        HSPMM_TRY(grow_buf(p, ws, (size_t)p.nnz * go));
        target = ws.ptr;
    }
    if (n == 0) {
        // a fill kernel rather than a memset node (callers may capture the
        // backward in a graph); 0.0 is the all-zero bit pattern in FP32/FP64
        HSPMM_TRY(fill_i32(static_cast<int32_t*>(target), 0, p.nnz * (int64_t)(go / 4), s));
    } else {
        SddArgs a{X.vr_start.as<int32_t>(), X.vr_end.as<int32_t>(), X.vr_row.as<int32_t>(), X.csr_col.as<int32_t>(),
                  X.csr_src.as<int32_t>(), X.n_vrows, X.bcsr_rb.as<int32_t>(), X.blk_ptr.as<int32_t>(),
                  X.blk_cnt.as<int32_t>(), X.blk_col.as<int32_t>(), X.chunk_ptr.as<int32_t>(),
                  X.chunk_base.as<int32_t>(), static_cast<const uint16_t*>(X.chunk_mask.ptr), X.rb_bcsr, B, ldb, dC, lddc, n, X.m, target};
        const size_t eb = dtype_size(X.ct);
        const bool last = p.canonical;  // else the gather to input order follows
        const int rc = [&]() -> int {
            switch (X.ct) {
                case HSPMM_F32: {
                    const bool v = n % 4 == 0 && ldb % 4 == 0 && lddc % 4 == 0 && aligned(B, 16) && aligned(dC, 16);
                    if (!v) return launch_sdd<float, float, 1, 64, 1, 32>(X, a, s, last);
                    HSPMM_LPR_SWITCH(lpr_for(n, 4), return (launch_sdd<float, float, 4, LPR, 4, 8>(X, a, s, last)));
                }
                case HSPMM_F64: {
                    const bool v = n % 2 == 0 && ldb % 2 == 0 && lddc % 2 == 0 && aligned(B, 16) && aligned(dC, 16);
                    if (!v) return launch_sdd<double, double, 1, 64, 1, 32>(X, a, s, last);
                    HSPMM_LPR_SWITCH(lpr_for(n, 2), return (launch_sdd<double, double, 2, LPR, 2, 16>(X, a, s, last)));
                }
                case HSPMM_F16: {
                    const bool v = n % 4 == 0 && ldb % 4 == 0 && lddc % 4 == 0 && aligned(B, 8) && aligned(dC, 16);
                    if (!v) return launch_sdd<half_t, float, 1, 64, 1, 32>(X, a, s, last);
                    // the FP16 MFMA form: n a multiple of 8 up to 256, 16-byte rows of B
                    if (n % 8 == 0 && n <= 256 && ldb % 8 == 0 && aligned(B, 16)) {
                        if (n <= 128)
                            HSPMM_LPR_SWITCH(lpr_for(n, HSPMM_SDD_H_VEC),
                                             return (launch_sdd<half_t, float, HSPMM_SDD_H_VEC, LPR, 8, 4>(X, a, s, last)));
                        HSPMM_LPR_SWITCH(lpr_for(n, HSPMM_SDD_H_VEC),
                                         return (launch_sdd<half_t, float, HSPMM_SDD_H_VEC, LPR, 8, 8>(X, a, s, last)));
                    }
                    HSPMM_LPR_SWITCH(lpr_for(n, 4), return (launch_sdd<half_t, float, 4, LPR, 4, 8>(X, a, s, last)));
                }
                case HSPMM_BF16: {
                    const bool v = n % 4 == 0 && ldb % 4 == 0 && lddc % 4 == 0 && aligned(B, 8) && aligned(dC, 16);
                    if (!v) return launch_sdd<bf16_t, float, 1, 64, 1, 32>(X, a, s, last);
                    // the BF16 MFMA form: n a multiple of 8 up to 256, 16-byte rows of B
                    if (n % 8 == 0 && n <= 256 && ldb % 8 == 0 && aligned(B, 16)) {
                        if (n <= 128)
                            HSPMM_LPR_SWITCH(lpr_for(n, HSPMM_SDD_H_VEC),
                                             return (launch_sdd<bf16_t, float, HSPMM_SDD_H_VEC, LPR, 8, 4>(X, a, s, last)));
                        HSPMM_LPR_SWITCH(lpr_for(n, HSPMM_SDD_H_VEC),
                                         return (launch_sdd<bf16_t, float, HSPMM_SDD_H_VEC, LPR, 8, 8>(X, a, s, last)));
                    }
                    if (n % 8 == 0 && ldb % 8 == 0 && aligned(B, 16))
                        HSPMM_LPR_SWITCH(lpr_for(n, HSPMM_SDD_H_VEC),
                                         return (launch_sdd<bf16_t, float, HSPMM_SDD_H_VEC, LPR, 4, 8>(X, a, s, last)));
                    HSPMM_LPR_SWITCH(lpr_for(n, 4), return (launch_sdd<bf16_t, float, 4, LPR, 4, 8>(X, a, s, last)));
                }
                default: return fail(HSPMM_ERR_DTYPE, "bad compute dtype");
            }
            return HSPMM_OK;
        }();
        (void)eb;
        HSPMM_TRY(rc);
    }
    if (!p.canonical) HSPMM_TRY(gather_dA(p, ws, dA, s));
    return HSPMM_OK;
}

}  // namespace hspmm
