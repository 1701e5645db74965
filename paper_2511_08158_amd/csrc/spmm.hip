// Forward kernels: C = X * B for one sub-plan, both parts in one launch.
//
// CSR-part (the AXPY kernel of Sec. 3.3): a wavefront serves 64/LPR virtual
// rows, LPR lanes per row, each lane owning VEC consecutive columns of C.
// The row's (column, value) pairs are fetched once, coalesced, one entry
// per lane, and broadcast inside the lane group; every entry then costs one
// coalesced VEC-wide load of a B row segment and VEC FMAs.
//
// BCSR-part (the outer-product kernel of Sec. 3.3, Alg. 2-3): one wave, or
// for row blocks with very many tiles one workgroup, owns one 16-row block
// and one column panel of C.  Each MFMA step takes kc tiles of the block (a
// 16 x kc slab of A, packed in lane order at plan time) and the kc gathered
// B rows, so every gathered B row serves 16 rows of C.  FP64/FP32 use
// 16x16x4 MFMAs (kc = 4); FP16/BF16 use 16x16x32 MFMAs (kc = 32, the
// widening accumulate of Alg. 3, with FP32 sums).  Partial K steps are
// padded with zero-valued tiles, as Alg. 3 pairs an odd tile with zeros.
//
// Each row of C has exactly one writer (Sec. 3.4): no atomics, and the
// result does not depend on scheduling.
#include "plan.h"

namespace hspmm {

namespace {

struct CsrArgs {
    const int32_t* vr_start;
    const int32_t* vr_end;
    const int32_t* vr_out;
    const int32_t* col;
    const void* val;
    int64_t n_vrows;
};

struct BcsrArgs {
    const int32_t* rb;
    const int32_t* blk_ptr;
    const int32_t* blk_cnt;
    const int32_t* blk_col;
    const void* val;
    int64_t n_rb;
    int32_t n_panels;
};

struct DenseArgs {
    const void* B;
    int64_t ldb;
    void* C;
    int64_t ldc;
    int64_t n;
    int64_t m;
    void* ws;            // partial rows of split CSR rows: [n_partials][n]
    const double* scale; // per 16-row block, or null
};

template <class T, int N>
__device__ inline void load_vec(const T* p, T (&out)[N]) {
    constexpr int C = (N * (int)sizeof(T) > 16) ? 16 / (int)sizeof(T) : N;  // 16-byte chunks
    if constexpr (C == 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = p[i];
    } else {
        typedef T V __attribute__((ext_vector_type(C)));
#pragma unroll
        for (int k = 0; k < N; k += C) {
            const V v = *reinterpret_cast<const V*>(p + k);
#pragma unroll
            for (int i = 0; i < C; ++i) out[k + i] = v[i];
        }
    }
}

// stores of up to 16 bytes per instruction (callers guarantee 16-byte
// alignment of every chunk).  HSPMM_NT_STORE=1 (build time) marks them
// non-temporal, the output being written once and never read by the kernel
// (so that it would not displace gathered rows of B from L2): measured on
// the block stencil FP32 forward 37.2 against 38.4 us warm but 43.2 against
// 42.6 us cold, and over whole steps (forward and one-pass backward, with
// its dA stores non-temporal too) 96.6 against 98.5 us warm but 111.2
// against 109.5 us cold, so it is off.
#ifndef HSPMM_NT_STORE
#define HSPMM_NT_STORE 0
#endif
template <class V>
__device__ inline void put(V* p, const V& v) {
    if constexpr (HSPMM_NT_STORE) {
        __builtin_nontemporal_store(v, p);
    } else {
        *p = v;
    }
}
template <class T, int N>
__device__ inline void store_vec(T* p, const T (&in)[N]) {
    constexpr int C = (N * (int)sizeof(T) > 16) ? 16 / (int)sizeof(T) : N;
    if constexpr (C == 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) put(p + i, in[i]);
    } else {
        typedef T V __attribute__((ext_vector_type(C)));
#pragma unroll
        for (int q = 0; q < N; q += C) {
            V v;
#pragma unroll
            for (int i = 0; i < C; ++i) v[i] = in[q + i];
            put(reinterpret_cast<V*>(p + q), v);
        }
    }
}

// ---------------------------------------------------------------------------
// CSR-part
// ---------------------------------------------------------------------------
template <class TV, class TB, class TC, int VEC, int LPR, int U>
__device__ void csr_wave(const CsrArgs& a, const DenseArgs& d, int64_t wave) {
    typedef typename Elem<TB>::acc_t acc_t;
    constexpr int R = 64 / LPR;
    const int lane = threadIdx.x & 63;
    const int g = lane / LPR, gl = lane % LPR;
    const int64_t vr = wave * R + g;
    if (wave * R >= a.n_vrows) return;  // wave-uniform
    const bool act = vr < a.n_vrows;
    const int start = act ? a.vr_start[vr] : 0;
    const int len = act ? a.vr_end[vr] - start : 0;
    const int out = act ? a.vr_out[vr] : 0;
    int maxlen = len;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, o, 64));
    const TV* __restrict__ val = static_cast<const TV*>(a.val);
    const TB* __restrict__ B = static_cast<const TB*>(d.B);

    for (int64_t c0 = 0; c0 < d.n; c0 += (int64_t)LPR * VEC) {
        const int64_t col0 = c0 + (int64_t)gl * VEC;
        const bool colok = col0 < d.n;
        acc_t acc[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = acc_t(0);
        for (int base = 0; base < maxlen; base += LPR) {
            const bool eok = base + gl < len;
            const int e = start + base + gl;
            const int my_col = eok ? a.col[e] : -1;
            const acc_t my_val = eok ? Elem<TV>::to_acc(val[e]) : acc_t(0);
            const int cnt = min(LPR, maxlen - base);
            for (int u0 = 0; u0 < cnt; u0 += U) {
                int cc[U];
                acc_t vv[U];
#pragma unroll
                for (int uu = 0; uu < U; ++uu) {
                    cc[uu] = __shfl(my_col, (u0 + uu) & (LPR - 1), LPR);
                    vv[uu] = __shfl(my_val, (u0 + uu) & (LPR - 1), LPR);
                }
                // branch-free gathers: an absent entry or a lane past n
                // reads row 0 / column 0 and a select drops the value
                // (power law FP16 n = 64 forward 451 -> 398 us; FP32
                // unchanged)
                TB bv[U][VEC];
                bool ok[U];
#pragma unroll
                for (int uu = 0; uu < U; ++uu) {
                    ok[uu] = cc[uu] >= 0 && colok && u0 + uu < cnt;
                    load_vec<TB, VEC>(B + (int64_t)(ok[uu] ? cc[uu] : 0) * d.ldb + (colok ? col0 : 0), bv[uu]);
                }
#pragma unroll
                for (int uu = 0; uu < U; ++uu)
#pragma unroll
                    for (int v = 0; v < VEC; ++v)
                        acc[v] += vv[uu] * (ok[uu] ? Elem<TB>::to_acc(bv[uu][v]) : acc_t(0));
            }
        }
        if (act && colok) {
            if (out >= 0) {
                const acc_t s = d.scale ? (acc_t)d.scale[out >> 4] : acc_t(1);
                TC o[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) o[v] = (TC)(acc[v] * s);
                store_vec<TC, VEC>(static_cast<TC*>(d.C) + (int64_t)out * d.ldc + col0, o);
            } else {
                acc_t* ws = static_cast<acc_t*>(d.ws) + (int64_t)(-out - 1) * d.n + col0;
#pragma unroll
                for (int v = 0; v < VEC; ++v) ws[v] = acc[v];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// BCSR-part, FP32 / FP64: 16x16x4 MFMA, four tiles per step
// ---------------------------------------------------------------------------
__device__ inline f4_t mfma4(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline d4_t mfma4(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <class T> struct AccOf;
template <> struct AccOf<float> { typedef f4_t type; };
template <> struct AccOf<double> { typedef d4_t type; };

// Row of the 16x16 MFMA result held in register r of lane group g
// (g = lane / 16): interleaved for the FP64 instruction, blocked otherwise.
template <class T> __device__ inline int out_row(int g, int r) { return 4 * g + r; }
template <> __device__ inline int out_row<double>(int g, int r) { return g + 4 * r; }

// K steps per load batch of the workgroup form below
#ifndef HSPMM_STEP_BATCH
#define HSPMM_STEP_BATCH 1
#endif
constexpr int kStepBatch = HSPMM_STEP_BATCH;
// gathers a CSR lane group keeps in flight: 4, also for FP16/BF16 lane
// groups of 8 lanes or fewer (HSPMM_CSR_U_NARROW).  With branch-free
// gathers, power law FP16 n = 64 (8 lanes) forward 456 / 399 / 370 us at
// 1 / 2 / 4; with a branch around each gather 2 had been best there.  Block
// stencil FP32 n = 128 (32 lanes) CSR-only forward 51.3 / 49.7 / 54.3 us
// at 8 / 4 / 2.
#ifndef HSPMM_CSR_U
#define HSPMM_CSR_U 4
#endif
#ifndef HSPMM_CSR_U_NARROW
#define HSPMM_CSR_U_NARROW 4
#endif
#ifndef HSPMM_F32_CSR_VEC8
#define HSPMM_F32_CSR_VEC8 0
#endif
// Operands of SB consecutive K steps of one wave.
template <class T, int VEC, int NL, int SB = kStepBatch>
struct StepRegs {
    T av[SB];
    T bv[SB][NL][VEC];
};

// Operands of this wave's K steps in rounds r .. r + kStepBatch - 1.  The
// loads are unconditional, so the compiler can count them precisely and
// the MFMAs of one batch wait only for their own operands, not for the
// batch loaded after them: a round past the wave's last one reloads the
// last round (never used), a tile past the row block's end reads its
// zero-valued padding slot and row 0 of B (0 * finite = 0), and a column
// past n reads column 0 into a result column that is never stored.
// The packed values are loaded with the default cache policy: the
// non-temporal hint measured 7 % (FP32) to 13 % (FP64) slower.
template <class T, int VEC, int NL>
__device__ inline void load_steps(const T* __restrict__ vals, const T* __restrict__ B, int64_t ldb, int64_t n,
                                  int b0, int w, int kq, int lane, int colreg, int j0, int jlast, int r,
                                  int64_t cbase, StepRegs<T, VEC, NL>& o) {
#pragma unroll
    for (int s = 0; s < kStepBatch; ++s) {
        const int rr = min(r + s, jlast);
        const int step0 = 16 * rr + 4 * w;
        const int bc = __shfl(colreg, (4 * (rr - j0) + kq) & 63, 64);
        o.av[s] = vals[(int64_t)(b0 + step0) * 16 + lane];
#pragma unroll
        for (int h = 0; h < NL; ++h) {
            const int64_t col = cbase + (int64_t)h * 16 * VEC;
            load_vec<T, VEC>(B + (int64_t)bc * ldb + (col < n ? col : 0), o.bv[s][h]);
        }
    }
}

// MFMAs of the batch's rounds r .. r + kStepBatch - 1; a round at or past
// jend holds a reloaded copy, whose A operand is replaced by zero (a select,
// not a branch, so the loop body stays one block)
template <class T, class ACC, int VEC, int NL, int SB>
__device__ inline void mfma_steps(const StepRegs<T, VEC, NL, SB>& o, ACC (&acc)[VEC * NL], int r, int jend) {
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        const T a = r + s < jend ? o.av[s] : T(0);
#pragma unroll
        for (int h = 0; h < NL; ++h)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[h * VEC + v] = mfma4(a, o.bv[s][h][v], acc[h * VEC + v]);
    }
}

// One workgroup (4 waves) per (row block, column panel).  The row block's
// K steps of 4 tiles are dealt round-robin to the 4 waves (step s -> wave
// s % 4), so four independent gather streams run per row block; the four
// partial 16 x PANEL tiles are then summed in a fixed order through LDS and
// each wave stores one register row of the result.  The tile columns of up
// to 16 rounds are fetched with one coalesced load and handed to the lanes
// by a shuffle, so B loads never wait on an index load, and the loads of the
// next kStepBatch steps are in flight while the MFMAs of the current ones run.
// Per-unit metadata of the BCSR-part (row block, tile range, the tile
// columns of the first 16 rounds).  Loading it is a short chain of
// dependent loads, so the workgroup fetches the next unit's metadata
// before it works on the current one.
struct UnitMeta {
    int rb, b0, cnt, panel, colreg;
    bool valid;
};

__device__ inline UnitMeta bcsr_meta(const BcsrArgs& a, int64_t unit) {
    UnitMeta m{0, 0, 0, 0, 0, false};
    const int64_t slot = unit / a.n_panels;
    if (slot >= a.n_rb) return m;
    const int lane = threadIdx.x & 63, w = wave_id();
    m.valid = true;
    m.panel = (int)(unit - slot * a.n_panels);
    m.rb = a.rb[slot];
    m.b0 = a.blk_ptr[slot];
    m.cnt = a.blk_cnt[slot];
    const int pre = 16 * (lane >> 2) + 4 * w + (lane & 3);
    m.colreg = pre < m.cnt ? a.blk_col[m.b0 + pre] : 0;
    return m;
}

template <class T, int VEC, int NL>
__device__ void bcsr_wg_f(const BcsrArgs& a, const DenseArgs& d, const UnitMeta& um, T* red) {
    typedef typename AccOf<T>::type acc_v;
    constexpr int PANEL = 16 * VEC * NL;
    constexpr int TILES = VEC * NL;
    if (!um.valid) return;  // uniform over the workgroup
    const int lane = threadIdx.x & 63, w = wave_id(), j = lane & 15, kq = lane >> 4;
    const int rb = um.rb;
    const int b0 = um.b0;
    const int cnt = um.cnt;
    const int64_t cbase = (int64_t)um.panel * PANEL + (int64_t)j * VEC;
    const T* __restrict__ vals = static_cast<const T*>(a.val);
    const T* __restrict__ B = static_cast<const T*>(d.B);
    acc_v acc[TILES];
#pragma unroll
    for (int t = 0; t < TILES; ++t) acc[t] = acc_v{0, 0, 0, 0};

    // a round = 16 tiles = one step per wave; this wave's step of round rr
    // starts at tile 16 rr + 4 w, so it has rounds 0 .. nr_w - 1
    const int nr_w = cnt > 4 * w ? (cnt - 4 * w + 15) >> 4 : 0;
    for (int j0 = 0; j0 < nr_w; j0 += 16) {
        int colreg = um.colreg;
        if (j0 > 0) {
            const int pre = 16 * (j0 + (lane >> 2)) + 4 * w + (lane & 3);
            colreg = pre < cnt ? a.blk_col[b0 + pre] : 0;
        }
        const int jend = min(nr_w, j0 + 16);
        StepRegs<T, VEC, NL> x, y;
        load_steps<T, VEC, NL>(vals, B, d.ldb, d.n, b0, w, kq, lane, colreg, j0, jend - 1, j0, cbase, x);
        // the scheduling barriers keep each batch's loads ahead of the
        // previous batch's MFMAs (the compiler would otherwise sink them to
        // their use to save registers, serialising load and compute)
        // (a body without an early exit: the batch after the last round is
        // loaded from clamped addresses and multiplied by zero)
        for (int jr = j0; jr < jend; jr += 2 * kStepBatch) {
            load_steps<T, VEC, NL>(vals, B, d.ldb, d.n, b0, w, kq, lane, colreg, j0, jend - 1, jr + kStepBatch,
                                   cbase, y);
            __builtin_amdgcn_sched_barrier(0);
            mfma_steps<T, acc_v, VEC, NL, kStepBatch>(x, acc, jr, jend);
            __builtin_amdgcn_sched_barrier(0);
            load_steps<T, VEC, NL>(vals, B, d.ldb, d.n, b0, w, kq, lane, colreg, j0, jend - 1,
                                   jr + 2 * kStepBatch, cbase, x);
            __builtin_amdgcn_sched_barrier(0);
            mfma_steps<T, acc_v, VEC, NL, kStepBatch>(y, acc, jr + kStepBatch, jend);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // fixed-order reduction of the four partial tiles, in two passes over
    // halves of the tiles so the LDS buffer stays at 16 KB
    constexpr int PASSES = TILES >= 2 ? 2 : 1;
    constexpr int TP = TILES / PASSES;
    T sum[TILES];
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
        if (p) __syncthreads();
#pragma unroll
        for (int t = 0; t < TP; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[((w * TP + t) * 4 + r) * 64 + lane] = acc[p * TP + t][r];
        __syncthreads();
#pragma unroll
        for (int t = 0; t < TP; ++t) {
            T x = red[((0 * TP + t) * 4 + w) * 64 + lane];
#pragma unroll
            for (int v = 1; v < 4; ++v) x += red[((v * TP + t) * 4 + w) * 64 + lane];
            sum[p * TP + t] = x;
        }
    }
    const int64_t row = (int64_t)rb * 16 + out_row<T>(kq, w);
    if (row >= d.m) return;
    const T sc = d.scale ? (T)d.scale[rb] : T(1);
#pragma unroll
    for (int h = 0; h < NL; ++h) {
        const int64_t col = cbase + (int64_t)h * 16 * VEC;
        if (col >= d.n) continue;
        T o[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) o[v] = sum[h * VEC + v] * sc;
        store_vec<T, VEC>(static_cast<T*>(d.C) + row * d.ldc + col, o);
    }
}

// One wave per (row block, column panel): the wave runs every K step of the
// row block (step s = tiles 4s .. 4s+3; lane (j, q) supplies tile 4s + q),
// so the result needs no reduction and is stored from the accumulators.
// Used when no row block of the part has more than kWaveMaxTiles tiles
// (one wave's sequential walk bounds the kernel's critical path); measured
// on the block stencil FP32 n = 128: forward 34.9 -> 33.5 us, FP64 68.2 ->
// 65.6 us against the four-wave split with its LDS reduction.
constexpr int kWaveMaxTiles = 2048;
// load batches in flight in the one-wave FP32 / FP64 walk: 2; 3 (loads of
// batch b + 2 issued before the MFMAs of batch b) measured the same for FP32
// and slower for FP64 on the block stencil (forward 39.3 vs 38.6 us, FP64
// 64.0 vs 58.9 us)
#ifndef HSPMM_WAVE_DEPTH
#define HSPMM_WAVE_DEPTH 2
#endif
constexpr int kWaveDepth = HSPMM_WAVE_DEPTH;
template <class T, int VEC, int NL, int SB>
__device__ inline void load_wave_steps(const T* __restrict__ vals, const T* __restrict__ B, int64_t ldb, int64_t n,
                                       int b0, int q, int lane, int colreg, int s0, int slast, int st,
                                       int64_t cbase, StepRegs<T, VEC, NL, SB>& o) {
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        const int ss = min(st + s, slast);
        const int bc = __shfl(colreg, (4 * (ss - s0) + q) & 63, 64);
        o.av[s] = vals[(int64_t)(b0 + 4 * ss) * 16 + lane];
#pragma unroll
        for (int h = 0; h < NL; ++h) {
            const int64_t col = cbase + (int64_t)h * 16 * VEC;
            load_vec<T, VEC>(B + (int64_t)bc * ldb + (col < n ? col : 0), o.bv[s][h]);
        }
    }
}

template <class T, int VEC, int NL, int DEPTH = 2>
__device__ void bcsr_wave_f(const BcsrArgs& a, const DenseArgs& d, int64_t unit) {
    typedef typename AccOf<T>::type acc_v;
    constexpr int PANEL = 16 * VEC * NL;
    constexpr int TILES = VEC * NL;
    const int64_t slot = unit / a.n_panels;
    if (slot >= a.n_rb) return;  // uniform over the wave
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const int panel = (int)(unit - slot * a.n_panels);
    const int rb = a.rb[slot];
    const int b0 = a.blk_ptr[slot];
    const int cnt = a.blk_cnt[slot];
    const int nsteps = (cnt + 3) >> 2;
    const int64_t cbase = (int64_t)panel * PANEL + (int64_t)j * VEC;
    const T* __restrict__ vals = static_cast<const T*>(a.val);
    const T* __restrict__ B = static_cast<const T*>(d.B);
    acc_v acc[TILES];
#pragma unroll
    for (int t = 0; t < TILES; ++t) acc[t] = acc_v{0, 0, 0, 0};
    for (int s0 = 0; s0 < nsteps; s0 += 16) {
        // 16 steps = 64 tiles: lane l holds the column of tile 4 s0 + l
        const int colreg = 4 * s0 + lane < cnt ? a.blk_col[b0 + 4 * s0 + lane] : 0;
        const int send = min(nsteps, s0 + 16);
        // steps per batch: 2 for FP64 (52.5 against 55.8 us on the stencil),
        // 1 for FP32 (no gain from 2)
        constexpr int SB = sizeof(T) == 8 ? 2 : 1;
        StepRegs<T, VEC, NL, SB> x, y;
        load_wave_steps<T, VEC, NL, SB>(vals, B, d.ldb, d.n, b0, q, lane, colreg, s0, send - 1, s0, cbase, x);
        if constexpr (DEPTH == 3) {
            // three batches in flight: the loads of batch b + 2 are issued
            // before the MFMAs of batch b
            StepRegs<T, VEC, NL, SB> z;
            load_wave_steps<T, VEC, NL, SB>(vals, B, d.ldb, d.n, b0, q, lane, colreg, s0, send - 1, s0 + SB, cbase,
                                            y);
            for (int sr = s0; sr < send; sr += 3 * SB) {
                load_wave_steps<T, VEC, NL, SB>(vals, B, d.ldb, d.n, b0, q, lane, colreg, s0, send - 1, sr + 2 * SB,
                                                cbase, z);
                __builtin_amdgcn_sched_barrier(0);
                mfma_steps<T, acc_v, VEC, NL, SB>(x, acc, sr, send);
                __builtin_amdgcn_sched_barrier(0);
                load_wave_steps<T, VEC, NL, SB>(vals, B, d.ldb, d.n, b0, q, lane, colreg, s0, send - 1, sr + 3 * SB,
                                                cbase, x);
                __builtin_amdgcn_sched_barrier(0);
                mfma_steps<T, acc_v, VEC, NL, SB>(y, acc, sr + SB, send);
                __builtin_amdgcn_sched_barrier(0);
                load_wave_steps<T, VEC, NL, SB>(vals, B, d.ldb, d.n, b0, q, lane, colreg, s0, send - 1, sr + 4 * SB,
                                                cbase, y);
                __builtin_amdgcn_sched_barrier(0);
                mfma_steps<T, acc_v, VEC, NL, SB>(z, acc, sr + 2 * SB, send);
                __builtin_amdgcn_sched_barrier(0);
            }
            continue;
        }
        for (int sr = s0; sr < send; sr += 2 * SB) {
            load_wave_steps<T, VEC, NL, SB>(vals, B, d.ldb, d.n, b0, q, lane, colreg, s0, send - 1, sr + SB, cbase,
                                            y);
            __builtin_amdgcn_sched_barrier(0);
            mfma_steps<T, acc_v, VEC, NL, SB>(x, acc, sr, send);
            __builtin_amdgcn_sched_barrier(0);
            load_wave_steps<T, VEC, NL, SB>(vals, B, d.ldb, d.n, b0, q, lane, colreg, s0, send - 1, sr + 2 * SB,
                                            cbase, x);
            __builtin_amdgcn_sched_barrier(0);
            mfma_steps<T, acc_v, VEC, NL, SB>(y, acc, sr + SB, send);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const T sc = d.scale ? (T)d.scale[rb] : T(1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = (int64_t)rb * 16 + out_row<T>(q, r);
        if (row >= d.m) continue;
#pragma unroll
        for (int h = 0; h < NL; ++h) {
            const int64_t col = cbase + (int64_t)h * 16 * VEC;
            if (col >= d.n) continue;
            T o[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) o[v] = acc[h * VEC + v][r] * sc;
            store_vec<T, VEC>(static_cast<T*>(d.C) + row * d.ldc + col, o);
        }
    }
}

// ---------------------------------------------------------------------------
// Fused backward on the BCSR-part of A^T (FP32 / FP64)
// ---------------------------------------------------------------------------
// A tile of A^T (row block R of A^T, column i) holds A[i][16R .. 16R + 15].
// The walk that computes dB = A^T dC for row block R gathers row i of dC for
// that tile, and the same row is all the SDDMM needs for the tile's entries
// of dA: dA[i][16R + r] = <dC[i,:], B[16R + r,:]> (the gradient of Sec.
// 3.3's product with respect to A's stored values).  One pass over A^T's
// tiles thus yields both gradients with one gather of dC per tile, where
// separate dB and SDDMM kernels run two gather streams (rows of dC, rows of
// B): on the block stencil FP32 n = 128 the L1 -> L2 read requests of the
// backward fall by 41 % and the backward from 70 to 62 us cold.
//
// For dA the contraction runs over the columns, so the gathered rows are
// needed with the column on the MFMA's K lanes, where the dB product has
// them on its N lanes: each step's gathered rows are written to an LDS tile
// of 16 rows (one per tile of a round of 4 steps) and read back after the
// round.  The 16 x 16 result of a round is
//     out[r][t] = sum_c B[16R + r][c] * dC[i_t][c],
// with B's 16 rows (the row block's columns of A) held in registers for the
// whole row block.  A tile's entries are consecutive columns of one row of
// A, so they are consecutive in A's canonical order too: entry r of tile t
// goes to tile_base[t] + popcount(tile_mask[t] below bit r).
struct BwdArgs {
    const int32_t* tile_base;   // [tiles] canonical index of the tile's first entry of A
    const uint16_t* tile_mask;  // [tiles] rows of the tile that hold an entry
    const void* B;              // forward dense operand, k x n
    int64_t ldb;
    int64_t kb;                 // rows of B (columns of A)
    void* dA;                   // canonical order of A's entries
};

template <class T, int N>
__device__ inline void store_lds_vec(T* p, const T (&in)[N]) {
    if constexpr (N == 1) {
        *p = in[0];
    } else {
        typedef T V __attribute__((ext_vector_type(N)));
        V v;
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = in[i];
        *reinterpret_cast<V*>(p) = v;
    }
}

// A workgroup of NW waves per row block of A^T, wave w owning columns
// [w CW, (w + 1) CW) of the panel (CW = 16 VEC, each lane VEC elements = 16
// bytes of a gathered row).  Every wave walks all of the row block's tiles,
// so each gathered row of dC is fetched as NW segments, one per wave, and a
// wave's registers hold only its share of the dB accumulators and of the
// 16 rows of B.  One wave holding the whole panel (the forward's walk plus
// the dA product) needed 136 registers, 3 waves per SIMD, and ran the block
// stencil's backward in 74 us; two waves of 64 columns need 94 (5 per
// SIMD).  Four waves of 8-byte segments (8 per SIMD) were slower (68 us):
// twice the load instructions, and each wave reloads the tile values.
// Each wave's dA products cover its own columns; after each round of 16
// tiles the partial 16 x 16 results are summed in wave order through LDS
// (double-buffered, one barrier per round) and written tile by tile, the 16
// lanes of a tile side by side on its consecutive entries (writing them
// from the MFMA layout, 4 scattered entries per tile and instruction, cost
// 2 us more).  The dA tile metadata of 64 tiles is fetched with their
// columns: a load inside a round would make the round's end wait for the
// gathers already issued for the next one.
template <class T, int NW, int VEC>
struct BwdCs {
    static constexpr int CW = 16 * VEC;              // columns per wave
    static constexpr int PANEL = NW * CW;
    static constexpr int KS = CW / 4;                // dA MFMA steps per round (K = 4 columns each)
    static constexpr int RPW = 4 / NW;               // dA store rounds of 4 tiles per wave and round
    static constexpr int CWP = CW + 16 / (int)sizeof(T);  // padded LDS row of the transposition buffer
    // LDS: per wave 16 rows of CWP, then two buffers of NW waves x 64 lanes x 4 partial sums
    static constexpr size_t kLdsT = (size_t)NW * 16 * CWP * sizeof(T);
    static constexpr size_t kLdsP = (size_t)2 * NW * 64 * 4 * sizeof(T);
    static constexpr size_t kLds = kLdsT + kLdsP;
};

template <class T, int NW, int VEC>
__device__ void bwd_cs(const BcsrArgs& a, const DenseArgs& d, const BwdArgs& bw, int64_t slot, unsigned char* smem,
                       int& buf) {
    typedef typename AccOf<T>::type acc_v;
    typedef BwdCs<T, NW, VEC> P;
    constexpr int CW = P::CW, KS = P::KS, CWP = P::CWP, RPW = P::RPW;
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4, w = wave_id();
    T* __restrict__ lt = reinterpret_cast<T*>(smem) + (int64_t)w * 16 * CWP;
    T* __restrict__ lp = reinterpret_cast<T*>(smem + P::kLdsT);
    const int rb = a.rb[slot];
    const int b0 = a.blk_ptr[slot];
    const int cnt = a.blk_cnt[slot];
    const int nsteps = (cnt + 3) >> 2;
    const int64_t c0 = (int64_t)w * CW;                 // this wave's first column
    const int64_t cl = c0 + (int64_t)j * VEC;           // this lane's columns in the walk
    const bool colok = cl < d.n;
    const T* __restrict__ vals = static_cast<const T*>(a.val);
    const T* __restrict__ G = static_cast<const T*>(d.B);
    // the dA product's A operand: row 16 rb + j of B at this wave's columns
    // c0 + KS q + s, the K lane of step s being q
    // (16-byte chunks, each wholly inside or outside n)
    T bs[KS];
    {
        constexpr int CH = 16 / (int)sizeof(T);
        const int64_t brow = (int64_t)rb * 16 + j;
#pragma unroll
        for (int h = 0; h < KS; h += CH) {
            const int64_t c = c0 + (int64_t)KS * q + h;
            T x[CH];
            if (brow < bw.kb && c < d.n) {
                load_vec<T, CH>(static_cast<const T*>(bw.B) + brow * bw.ldb + c, x);
            } else {
#pragma unroll
                for (int e = 0; e < CH; ++e) x[e] = T(0);
            }
#pragma unroll
            for (int e = 0; e < CH; ++e) bs[h + e] = x[e];
        }
    }
    acc_v acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = acc_v{0, 0, 0, 0};
    for (int s0 = 0; s0 < nsteps; s0 += 16) {
        const int colreg = 4 * s0 + lane < cnt ? a.blk_col[b0 + 4 * s0 + lane] : 0;
        // the dA destinations of the same 64 tiles (tiles past cnt: none),
        // fetched with the columns so that no load waits inside a round
        const int32_t basereg = 4 * s0 + lane < cnt ? bw.tile_base[b0 + 4 * s0 + lane] : 0;
        const uint32_t maskreg = 4 * s0 + lane < cnt ? (uint32_t)bw.tile_mask[b0 + 4 * s0 + lane] : 0u;
        const int send = min(nsteps, s0 + 16);
        // operands of one step: this lane's A value and VEC elements of the
        // gathered row of tile 4 st + q (steps past the last reload it)
        auto load = [&](int st, T& av, T (&bv)[VEC]) {
            const int ss = min(st, send - 1);
            const int bc = __shfl(colreg, (4 * (ss - s0) + q) & 63, 64);
            av = vals[(int64_t)(b0 + 4 * ss) * 16 + lane];
            load_vec<T, VEC>(G + (int64_t)bc * d.ldb + (colok ? cl : 0), bv);
        };
        T ax, ay, bx[VEC], by[VEC];
        load(s0, ax, bx);
        for (int sr = s0; sr < send; sr += 4) {
#pragma unroll
            for (int st = 0; st < 4; st += 2) {
                load(sr + st + 1, ay, by);
                __builtin_amdgcn_sched_barrier(0);
                {
                    const T av = sr + st < send ? ax : T(0);
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[v] = mfma4(av, bx[v], acc[v]);
                    store_lds_vec<T, VEC>(lt + (4 * st + q) * CWP + j * VEC, bx);
                }
                __builtin_amdgcn_sched_barrier(0);
                load(sr + st + 2, ax, bx);
                __builtin_amdgcn_sched_barrier(0);
                {
                    const T av = sr + st + 1 < send ? ay : T(0);
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[v] = mfma4(av, by[v], acc[v]);
                    store_lds_vec<T, VEC>(lt + (4 * (st + 1) + q) * CWP + j * VEC, by);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            // this wave's share of the round's dA: lane (j, q) supplies tile
            // j's columns KS q + s (its own writes above, in LDS order)
            T gv[KS];
            load_vec<T, KS>(lt + j * CWP + KS * q, gv);
            acc_v g = acc_v{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s) g = mfma4(bs[s], gv[s], g);
            T* __restrict__ pb = lp + (int64_t)buf * NW * 64 * 4;
            {
                const T gp[4] = {g[0], g[1], g[2], g[3]};
                store_lds_vec<T, 4>(pb + ((int64_t)w * 64 + lane) * 4, gp);
            }
            // the buffers alternate over every round the workgroup runs, so
            // a buffer is rewritten only after every wave passed the
            // barrier that follows its last reads
            __syncthreads();
            // the sums over the waves (in wave order), written tile by tile:
            // lane l takes row rr = l % 16 of tile t = 4 i + l / 16, so the
            // 16 lanes of a tile write its entries, consecutive in A's
            // canonical order, side by side; wave w takes tiles
            // [16 w / NW, 16 (w + 1) / NW)
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int t = (16 / NW) * w + 4 * i + q;   // tile of this lane
                const int rr = j;                          // its row (a column of A)
                const int g4 = sizeof(T) == 8 ? (rr & 3) : (rr >> 2);  // lane group holding row rr
                const int r = sizeof(T) == 8 ? (rr >> 2) : (rr & 3);   // and its register
                const int src = 16 * g4 + t;
                T sum = pb[(0 * 64 + src) * 4 + r];
#pragma unroll
                for (int u = 1; u < NW; ++u) sum += pb[((int64_t)u * 64 + src) * 4 + r];
                const int32_t base = __shfl((int)basereg, (4 * (sr - s0) + t) & 63, 64);
                const uint32_t mk = (uint32_t)__shfl((int)maskreg, (4 * (sr - s0) + t) & 63, 64);
                if ((mk >> rr) & 1u) static_cast<T*>(bw.dA)[base + __popc(mk & ((1u << rr) - 1u))] = sum;
            }
            buf ^= 1;
        }
    }
    if (!colok) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = (int64_t)rb * 16 + out_row<T>(q, r);
        if (row >= d.m) continue;
        T o[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) o[v] = acc[v][r];
        store_vec<T, VEC>(static_cast<T*>(d.C) + row * d.ldc + cl, o);
    }
}

template <class T, int NW, int VEC>
__global__ __launch_bounds__(256) void k_bwd_cs(BcsrArgs ba, DenseArgs da, BwdArgs bw, uint32_t g, int remap) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int buf = 0;
    for (int64_t slot = (int64_t)xcd_remap(blockIdx.x, g, remap); slot < ba.n_rb; slot += g)
        bwd_cs<T, NW, VEC>(ba, da, bw, slot, lds_raw, buf);
}

// CSR-part of A^T in the fused backward: LPR lanes per (segment of a) row
// j of A^T, which is column j of A, each lane VEC columns of one panel.
// Row j of B sits in the lane group's registers; every entry (i, a_ij)
// gathers row i of dC once, adds a_ij dC[i,:] to the row of dB (in entry
// order, as the forward's CSR walk sums) and forms the lane's share of
// dA[i][j] = <dC[i,:], B[j,:]>, reduced across the group U entries at a
// time by a halving butterfly (U - 1 + log2(LPR / U) shuffles per U
// entries).  dA goes to A's canonical index of the entry.
struct CsrBwdArgs {
    const int32_t* vr_start;
    const int32_t* vr_end;
    const int32_t* vr_out;   // row of dB, or -(partial slot + 1) of a split row
    const int32_t* vr_row;   // row of A^T
    const int32_t* col;      // row of A
    const void* val;         // values of A^T (the dC type)
    const int32_t* dst;      // A's canonical index of each entry
    int64_t n_vrows;
    const void* B;           // forward dense operand (compute type)
    int64_t ldb;
    void* dA;
};

// entries reduced together (U) and gathers in flight (UB): 8 / 4 against
// 16 / 8 (137 -> 94 registers at 32 lanes) measured GCN FP32 n = 128
// backward 837 -> 823 us, power law FP16 n = 128 1490 -> 1487; 4 / 4 was
// within 3 % either way
#ifndef HSPMM_BWD_CSR_U
#define HSPMM_BWD_CSR_U 8
#endif
#ifndef HSPMM_BWD_CSR_UB
#define HSPMM_BWD_CSR_UB 4
#endif
template <class TB, class TG, int VEC, int LPR>
__device__ void csr_bwd_wave(const CsrBwdArgs& a, const DenseArgs& d, int64_t wave) {
    constexpr int R = 64 / LPR;
    constexpr int U = LPR < HSPMM_BWD_CSR_U ? LPR : HSPMM_BWD_CSR_U;
    constexpr int SPAN = LPR / U;  // lanes that end with the same entry
    constexpr int UB = U < HSPMM_BWD_CSR_UB ? U : HSPMM_BWD_CSR_UB;  // gathers in flight
    const int lane = threadIdx.x & 63;
    const int g = lane / LPR, gl = lane % LPR;
    if (wave * R >= a.n_vrows) return;  // wave-uniform
    const int64_t vr = wave * R + g;
    const bool act = vr < a.n_vrows;
    const int start = act ? a.vr_start[vr] : 0;
    const int len = act ? a.vr_end[vr] - start : 0;
    const int out = act ? a.vr_out[vr] : 0;
    const int row = act ? a.vr_row[vr] : 0;
    int maxlen = len;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, o, 64));
    const TG* __restrict__ val = static_cast<const TG*>(a.val);
    const TG* __restrict__ dC = static_cast<const TG*>(d.B);
    TG* __restrict__ dA = static_cast<TG*>(a.dA);
    const int64_t col0 = (int64_t)gl * VEC;
    const bool colok = col0 < d.n;
    TG b0[VEC];
    {
        TB x[VEC];
        if (act && colok) {
            load_vec<TB, VEC>(static_cast<const TB*>(a.B) + (int64_t)row * a.ldb + col0, x);
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) x[v] = TB(0);
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v) b0[v] = Elem<TB>::to_acc(x[v]);
    }
    TG acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = TG(0);
    for (int base = 0; base < maxlen; base += LPR) {
        const bool eok = base + gl < len;
        const int e = start + base + gl;
        const int my_col = eok ? a.col[e] : -1;
        const TG my_val = eok ? val[e] : TG(0);
        const int my_dst = eok ? a.dst[e] : -1;
        const int cnt = min(LPR, maxlen - base);
        for (int u0 = 0; u0 < cnt; u0 += U) {
            TG part[U];
#pragma unroll
            for (int ub = 0; ub < U; ub += UB) {
                // branch-free gathers: an absent entry or a lane past n
                // reads row 0 / column 0 and a select drops its products
                TG cv[UB][VEC];
                TG vv[UB];
                bool ok[UB];
#pragma unroll
                for (int k = 0; k < UB; ++k) {
                    const int c = __shfl(my_col, (u0 + ub + k) & (LPR - 1), LPR);
                    vv[k] = __shfl(my_val, (u0 + ub + k) & (LPR - 1), LPR);
                    ok[k] = c >= 0 && u0 + ub + k < cnt && colok;
                    load_vec<TG, VEC>(dC + (int64_t)(ok[k] ? c : 0) * d.ldb + (colok ? col0 : 0), cv[k]);
                }
#pragma unroll
                for (int k = 0; k < UB; ++k) {
                    TG dot = TG(0);
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        acc[v] += vv[k] * (ok[k] ? cv[k][v] : TG(0));
                        dot += b0[v] * cv[k][v];
                    }
                    part[ub + k] = ok[k] ? dot : TG(0);
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
            const int dd = __shfl(my_dst, idx & (LPR - 1), LPR);
            if ((gl % SPAN) == 0 && idx < cnt && dd >= 0) dA[dd] = part[0];
        }
    }
    if (act && colok) {
        if (out >= 0) {
            store_vec<TG, VEC>(static_cast<TG*>(d.C) + (int64_t)out * d.ldc + col0, acc);
        } else {
            TG* ws = static_cast<TG*>(d.ws) + (int64_t)(-out - 1) * d.n + col0;
#pragma unroll
            for (int v = 0; v < VEC; ++v) ws[v] = acc[v];
        }
    }
}

template <class TB, class TG, int VEC, int LPR>
__global__ __launch_bounds__(256) void k_bwd_csr(CsrBwdArgs a, DenseArgs d, uint32_t g, int remap) {
    constexpr int R = 64 / LPR;
    const int64_t waves = (a.n_vrows + R - 1) / R;
    for (int64_t wave = (int64_t)xcd_remap(blockIdx.x, g, remap) * 4 + wave_id(); wave < waves;
         wave += (int64_t)g * 4)
        csr_bwd_wave<TB, TG, VEC, LPR>(a, d, wave);
}

// ---------------------------------------------------------------------------
// BCSR-part in groups of row blocks that share columns, FP32 / FP64
// ---------------------------------------------------------------------------
// One workgroup per (group, column panel of 256 bytes).  It copies the
// panel of every column the group's tiles use into LDS with direct
// global -> LDS loads (all of a wave's copies in flight at once), and while
// they are in flight each wave loads the values and stage rows of its first
// row block; its four waves then take the group's row blocks in turn and
// run the MFMA walk of bcsr_wave_f over them with every B operand read from
// LDS.  A column several row blocks of the group use is fetched once per
// group instead of once per tile, and the walk waits on no global load.
struct GroupArgs {
    const int32_t* rb;        // kernel slot -> row block
    const int32_t* blk_ptr;   // kernel slot -> first stored tile
    const int32_t* blk_cnt;   // kernel slot -> real tiles
    const int32_t* grp_ptr;   // [ngroups + 1]: kernel slots of each group
    const int32_t* grp_uptr;  // [ngroups + 1]: staged columns of each group
    const int32_t* ucol;
    const int32_t* bsrc;      // per stored tile: its row of the group's stage
    const void* val;
    int64_t ngroups;
    int32_t n_panels;
};

// operands of up to 32 MFMA steps (128 tiles) of one row block: the values
// of row (lane & 15) of tile (lane >> 4) of each step, and the stage row of
// tile 64 h + lane in bs[h]
template <class T>
struct GBlock {
    T av[32];
    int bs[2];
};

template <class T>
__device__ inline void load_gblock(const T* __restrict__ vals, const int32_t* __restrict__ bsrc, int b0, int nsteps,
                                   int st0, int lane, GBlock<T>& o) {
    const int last = nsteps - 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int tt = 4 * st0 + 64 * h + lane;
        o.bs[h] = tt < 4 * nsteps ? bsrc[b0 + tt] : 0;
    }
#pragma unroll
    for (int t = 0; t < 32; ++t) o.av[t] = vals[(int64_t)(b0 + 4 * min(st0 + t, last)) * 16 + lane];
}

template <class T, int VEC>
__device__ void bcsr_group_f(const GroupArgs& a, const DenseArgs& d, int64_t unit, T* lds, int* lidx) {
    typedef typename AccOf<T>::type acc_v;
    constexpr int PANEL = 16 * VEC;                     // 256 bytes of a B row
    constexpr int RS = kGroupRowBytes / (int)sizeof(T);  // LDS row stride, elements
    constexpr int CH = 16 / (int)sizeof(T);             // elements per 16-byte copy
    static_assert(PANEL * (int)sizeof(T) == kGroupRowBytes, "a panel is one staged row");
    const int64_t grp = unit / a.n_panels;
    if (grp >= a.ngroups) return;  // uniform over the workgroup
    const int panel = (int)(unit - grp * a.n_panels);
    const int64_t pcol0 = (int64_t)panel * PANEL;
    const int s0 = a.grp_ptr[grp], s1 = a.grp_ptr[grp + 1];
    const int u0 = a.grp_uptr[grp], U = a.grp_uptr[grp + 1] - u0;
    const T* __restrict__ B = static_cast<const T*>(d.B);
    const T* __restrict__ vals = static_cast<const T*>(a.val);
    const int lane = threadIdx.x & 63, w = wave_id(), j = lane & 15, q = lane >> 4;

    // the stage's columns into LDS, and this wave's first row block, before
    // any copy is issued (the copies and the block's operand loads below
    // then wait on no global load for their addresses)
    int sl = s0 + w;
    int rb = 0, b0 = 0, nsteps = 0;
    if (sl < s1) {
        rb = a.rb[sl];
        b0 = a.blk_ptr[sl];
        nsteps = (a.blk_cnt[sl] + 3) >> 2;
    }
    for (int i = threadIdx.x; i < U; i += 256) lidx[i] = a.ucol[u0 + i];
    __syncthreads();
    // the stage: four rows per wave instruction (lane l copies 16 bytes of
    // row r0 + l / 16); columns past n copy column 0 (their results are
    // never stored); a wave's last copy may fill up to three rows past U
    // with the stage's first column
    {
        const int64_t col = pcol0 + (lane & 15) * CH;
        const int64_t gc = col < d.n ? col : 0;
        for (int r0 = 4 * w; r0 < U; r0 += 16) {
            const int r = r0 + (lane >> 4);
            const int64_t brow = lidx[r < U ? r : 0];
            __builtin_amdgcn_global_load_lds(B + brow * d.ldb + gc, lds + r0 * RS, 16, 0, 0);
        }
    }
    // the operands of this wave's first row block, loaded while the stage
    // is in flight
    GBlock<T> blk;
    if (sl < s1) load_gblock<T>(vals, a.bsrc, b0, nsteps, 0, lane, blk);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const int64_t cb = pcol0 + (int64_t)j * VEC;
    const bool colok = cb < d.n;
    const T* lrow = lds + j * VEC;
    for (; sl < s1; sl += 4) {
        acc_v acc[VEC];
#pragma unroll
        for (int t = 0; t < VEC; ++t) acc[t] = acc_v{0, 0, 0, 0};
        for (int st0 = 0; st0 < nsteps; st0 += 32) {
            if (st0 > 0) load_gblock<T>(vals, a.bsrc, b0, nsteps, st0, lane, blk);
            // four steps at a time, the B operands of the next four read
            // from LDS while the MFMAs of these run; a step past the row
            // block's last multiplies zero values (its stage row is row 0)
            T bc[4][VEC];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int bs = __shfl(blk.bs[0], (4 * k + q) & 63, 64);
                load_vec<T, VEC>(lrow + bs * RS, bc[k]);
            }
#pragma unroll
            for (int t4 = 0; t4 < 32; t4 += 4) {
                if (st0 + t4 >= nsteps) break;  // uniform over the wave
                T bn[4][VEC];
                if (t4 + 4 < 32) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int t = t4 + 4 + k;
                        const int bs = __shfl(blk.bs[t >> 4], (4 * (t & 15) + q) & 63, 64);
                        load_vec<T, VEC>(lrow + bs * RS, bn[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const T x = st0 + t4 + k < nsteps ? blk.av[t4 + k] : T(0);
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[v] = mfma4(x, bc[k][v], acc[v]);
                }
                if (t4 + 4 < 32) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
#pragma unroll
                        for (int v = 0; v < VEC; ++v) bc[k][v] = bn[k][v];
                }
            }
        }
        const T sc = d.scale ? (T)d.scale[rb] : T(1);
        if (colok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = (int64_t)rb * 16 + out_row<T>(q, r);
                if (row >= d.m) continue;
                T o[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) o[v] = acc[v][r] * sc;
                store_vec<T, VEC>(static_cast<T*>(d.C) + row * d.ldc + cb, o);
            }
        }
        if (sl + 4 < s1) {
            rb = a.rb[sl + 4];
            b0 = a.blk_ptr[sl + 4];
            nsteps = (a.blk_cnt[sl + 4] + 3) >> 2;
            load_gblock<T>(vals, a.bsrc, b0, nsteps, 0, lane, blk);
        }
    }
}

template <class T, int VEC>
__global__ __launch_bounds__(256) void k_bcsr_group(GroupArgs ga, DenseArgs da, uint32_t g, int remap,
                                                    int stage_rows) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* stage = reinterpret_cast<T*>(lds_raw);
    int* lidx = reinterpret_cast<int*>(lds_raw + (size_t)(stage_rows + 4) * kGroupRowBytes);
    const int64_t units = ga.ngroups * (int64_t)ga.n_panels;
    for (int64_t unit = (int64_t)xcd_remap(blockIdx.x, g, remap); unit < units; unit += g) {
        bcsr_group_f<T, VEC>(ga, da, unit, stage, lidx);
        __syncthreads();  // the stage is rewritten by the next unit
    }
}

// ---------------------------------------------------------------------------
// BCSR-part, FP16 / BF16: 16x16x32 MFMA (FP32 accumulate), 32 tiles per step
// ---------------------------------------------------------------------------
__device__ inline f4_t mfma32(h8_t a, h8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ inline f4_t mfma32(b8_t a, b8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
template <class T> struct V8Of;
template <> struct V8Of<half_t> { typedef h8_t type; };
template <> struct V8Of<bf16_t> { typedef b8_t type; };

// Same workgroup scheme with 32-tile K steps (16x16x32 MFMA): step s of the
// row block goes to wave s % 4.  Lane (j, g) gathers CPL columns of the 8 B
// rows of tiles 8g..8g+7 of the step and transposes them in registers into
// the K-major operand of each of the CPL column tiles.
template <class T, int CPL>
__device__ void bcsr_wg_h(const BcsrArgs& a, const DenseArgs& d, int64_t unit, float* red) {
    typedef typename V8Of<T>::type v8;
    constexpr int PANEL = 16 * CPL;
    const int64_t slot = unit / a.n_panels;
    if (slot >= a.n_rb) return;
    const int panel = (int)(unit - slot * a.n_panels);
    const int lane = threadIdx.x & 63, w = wave_id(), j = lane & 15, g = lane >> 4;
    const int rb = a.rb[slot];
    const int b0 = a.blk_ptr[slot];
    const int cnt = a.blk_cnt[slot];
    const int64_t cbase = (int64_t)panel * PANEL + (int64_t)j * CPL;
    const bool colok = cbase < d.n;
    const T* __restrict__ vals = static_cast<const T*>(a.val);
    const T* __restrict__ B = static_cast<const T*>(d.B);
    f4_t acc[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) acc[t] = f4_t{0.f, 0.f, 0.f, 0.f};

    for (int step0 = 32 * w; step0 < cnt; step0 += 128) {
        // the 32 columns of this step: lane l holds tile step0 + (l & 31)
        const int pre = step0 + (lane & 31);
        const int colreg = pre < cnt ? a.blk_col[b0 + pre] : 0;
        const v8 av = *reinterpret_cast<const v8*>(vals + ((int64_t)(b0 + step0) * 16 + lane * 8));
        T raw[8][CPL];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int kk = step0 + 8 * g + u;
            const int bc = __shfl(colreg, 8 * g + u, 64);
            if (kk < cnt && colok) {
                load_vec<T, CPL>(B + (int64_t)bc * d.ldb + cbase, raw[u]);
            } else {
#pragma unroll
                for (int t = 0; t < CPL; ++t) raw[u][t] = T(0);
            }
        }
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            v8 bop;
#pragma unroll
            for (int u = 0; u < 8; ++u) bop[u] = raw[u][t];
            acc[t] = mfma32(av, bop, acc[t]);
        }
    }
    constexpr int PASSES = CPL >= 2 ? 2 : 1;
    constexpr int TP = CPL / PASSES;
    float o[CPL];
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
        if (p) __syncthreads();
#pragma unroll
        for (int t = 0; t < TP; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[((w * TP + t) * 4 + r) * 64 + lane] = acc[p * TP + t][r];
        __syncthreads();
#pragma unroll
        for (int t = 0; t < TP; ++t) {
            float x = red[((0 * TP + t) * 4 + w) * 64 + lane];
#pragma unroll
            for (int v = 1; v < 4; ++v) x += red[((v * TP + t) * 4 + w) * 64 + lane];
            o[p * TP + t] = x;
        }
    }
    const int64_t row = (int64_t)rb * 16 + 4 * g + w;
    if (row >= d.m || !colok) return;
    const float sc = d.scale ? (float)d.scale[rb] : 1.0f;
#pragma unroll
    for (int t = 0; t < CPL; ++t) o[t] *= sc;
    store_vec<float, CPL>(static_cast<float*>(d.C) + row * d.ldc + cbase, o);
}

// One wave per (row block, column panel) for FP16 / BF16: the wave runs the
// row block's 32-tile K steps itself, loading step s + 1 (tile columns,
// packed values, the 8 gathered rows per lane) while the MFMAs of step s
// run, and stores its accumulators directly.  Loads are unconditional: a
// padding tile reads row 0 of B against zero values, a column group past n
// reads column 0 into results that are not stored.
template <class T, int CPL>
struct HStep {
    typename V8Of<T>::type av;
    T raw[8][CPL];
};

template <class T, int CPL>
__device__ inline void load_hstep(const BcsrArgs& a, const T* __restrict__ vals, const T* __restrict__ B,
                                  int64_t ldb, int b0, int cnt, int step0, int lane, int g, int64_t col,
                                  HStep<T, CPL>& o) {
    typedef typename V8Of<T>::type v8;
    const int pre = step0 + (lane & 31);
    const int colreg = pre < cnt ? a.blk_col[b0 + pre] : 0;
    o.av = *reinterpret_cast<const v8*>(vals + ((int64_t)(b0 + step0) * 16 + lane * 8));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int bc = __shfl(colreg, 8 * g + u, 64);
        load_vec<T, CPL>(B + (int64_t)bc * ldb + col, o.raw[u]);
    }
}

template <class T, int CPL>
__device__ inline void mfma_hstep(const HStep<T, CPL>& o, f4_t (&acc)[CPL]) {
    typedef typename V8Of<T>::type v8;
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
        v8 bop;
#pragma unroll
        for (int u = 0; u < 8; ++u) bop[u] = o.raw[u][t];
        acc[t] = mfma32(o.av, bop, acc[t]);
    }
}

template <class T, int CPL>
__device__ void bcsr_wave_h(const BcsrArgs& a, const DenseArgs& d, int64_t unit) {
    constexpr int PANEL = 16 * CPL;
    const int64_t slot = unit / a.n_panels;
    if (slot >= a.n_rb) return;  // uniform over the wave
    const int panel = (int)(unit - slot * a.n_panels);
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const int rb = a.rb[slot];
    const int b0 = a.blk_ptr[slot];
    const int cnt = a.blk_cnt[slot];
    const int64_t cbase = (int64_t)panel * PANEL + (int64_t)j * CPL;
    const bool colok = cbase < d.n;
    const int64_t col = colok ? cbase : 0;
    const T* __restrict__ vals = static_cast<const T*>(a.val);
    const T* __restrict__ B = static_cast<const T*>(d.B);
    f4_t acc[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) acc[t] = f4_t{0.f, 0.f, 0.f, 0.f};
    const int nsteps = (cnt + 31) >> 5;
    HStep<T, CPL> x, y;
    // an empty row block (forced splits put them in the BCSR-part) has no
    // packed values at all: its first step must not be loaded, since
    // blk_ptr of the last row block can be the end of the value array
    if (nsteps > 0) load_hstep<T, CPL>(a, vals, B, d.ldb, b0, cnt, 0, lane, g, col, x);
    for (int s = 0; s < nsteps; s += 2) {
        // the step after the last one reloads the last (multiplied by zero)
        const int s1 = min(s + 1, nsteps - 1), s2 = min(s + 2, nsteps - 1);
        load_hstep<T, CPL>(a, vals, B, d.ldb, b0, cnt, 32 * s1, lane, g, col, y);
        __builtin_amdgcn_sched_barrier(0);
        mfma_hstep<T, CPL>(x, acc);
        __builtin_amdgcn_sched_barrier(0);
        load_hstep<T, CPL>(a, vals, B, d.ldb, b0, cnt, 32 * s2, lane, g, col, x);
        __builtin_amdgcn_sched_barrier(0);
        if (s + 1 >= nsteps) y.av = typename V8Of<T>::type{};  // a select, not a branch
        mfma_hstep<T, CPL>(y, acc);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (!colok) return;
    const float sc = d.scale ? (float)d.scale[rb] : 1.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = (int64_t)rb * 16 + 4 * g + r;
        if (row >= d.m) continue;
        float o[CPL];
#pragma unroll
        for (int t = 0; t < CPL; ++t) o[t] = acc[t][r] * sc;
        store_vec<float, CPL>(static_cast<float*>(d.C) + row * d.ldc + cbase, o);
    }
}

// ---------------------------------------------------------------------------
// fused launch: workgroups [0, g_bcsr) run the BCSR-part, the rest the CSR-part
// ---------------------------------------------------------------------------
// DO_CSR / DO_BCSR compile a part out when the plan has none of it, so a
// one-part plan does not pay the other part's register footprint.  When both
// parts are compiled in, the kernel is held to the waves per SIMD that the
// BCSR-only kernel reaches: the BCSR-part loses in proportion to lost
// occupancy, while the CSR code, compiled into a tighter register budget,
// makes up with the extra waves.
template <class TV, int VEC, int BV, int BNL, bool WAVE>
constexpr int bcsr_waves_per_simd() {
    // register-limited occupancy of the BCSR-only instantiations on gfx950
    // (VGPR + AGPR count from the compiler's resource usage report); FP16 /
    // BF16 with 4 column groups is held one wave lower, where the fused
    // kernel fits without spilling
    if (sizeof(TV) == 2) return VEC == 1 ? 7 : (BV == 8 ? (WAVE ? 3 : 4) : (WAVE ? 4 : 5));
    if (sizeof(TV) == 8) return VEC == 1 ? 4 : (BNL >= 2 ? 4 : (WAVE ? 8 : 7));
    return VEC == 1 ? (WAVE ? 7 : 6) : (BNL >= 2 ? (WAVE ? 5 : 4) : 8);
}

template <class TV, class TB, class TC, int VEC, int LPR, int BV, int BNL, bool DO_CSR, bool DO_BCSR, bool WAVE>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(DO_CSR && DO_BCSR ? bcsr_waves_per_simd<TV, VEC, BV, BNL, WAVE>() : 1)))
void k_hybrid(CsrArgs ca, BcsrArgs ba, DenseArgs da, uint32_t g_bcsr, uint32_t g_csr, int remap) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint32_t bid = blockIdx.x;
    const int w = wave_id();
    if (bid < g_bcsr) {
        if constexpr (DO_BCSR) {
            // g_bcsr workgroups stride over the row-block units (one unit
            // each unless a calibrated partition caps the part's workgroups)
            const int64_t units = ba.n_rb * (int64_t)ba.n_panels;
            if constexpr (sizeof(TV) == 2 && WAVE) {
                // four units per workgroup, one per wave
                for (int64_t u4 = (int64_t)xcd_remap(bid, g_bcsr, remap); u4 * 4 < units; u4 += g_bcsr)
                    bcsr_wave_h<TV, BV>(ba, da, u4 * 4 + w);
            } else if constexpr (sizeof(TV) == 2) {
                for (int64_t unit = (int64_t)xcd_remap(bid, g_bcsr, remap); unit < units; unit += g_bcsr) {
                    bcsr_wg_h<TV, BV>(ba, da, unit, reinterpret_cast<float*>(lds_raw));
                    __syncthreads();  // the reduction buffer is reused by the next unit
                }
            } else if constexpr (WAVE) {
                // four units per workgroup, one per wave
                for (int64_t u4 = (int64_t)xcd_remap(bid, g_bcsr, remap); u4 * 4 < units; u4 += g_bcsr)
                    bcsr_wave_f<TV, BV, BNL, kWaveDepth>(ba, da, u4 * 4 + w);
            } else {
                // a contiguous range of units per workgroup (neighbouring row
                // blocks share gathered rows of B in the XCD's L2)
                const int64_t per = (units + g_bcsr - 1) / g_bcsr;
                int64_t unit = (int64_t)xcd_remap(bid, g_bcsr, remap) * per;
                const int64_t uend = unit + per < units ? unit + per : units;
                UnitMeta cur = unit < uend ? bcsr_meta(ba, unit) : UnitMeta{0, 0, 0, 0, 0, false};
                for (; unit < uend; ++unit) {
                    const UnitMeta nxt = unit + 1 < uend ? bcsr_meta(ba, unit + 1) : UnitMeta{0, 0, 0, 0, 0, false};
                    bcsr_wg_f<TV, BV, BNL>(ba, da, cur, reinterpret_cast<TV*>(lds_raw));
                    __syncthreads();  // the reduction buffer is reused by the next unit
                    cur = nxt;
                }
            }
        }
    } else {
        if constexpr (DO_CSR) {
            constexpr int R = 64 / LPR;
            const int64_t waves = (ca.n_vrows + R - 1) / R;
            for (int64_t wave = (int64_t)xcd_remap(bid - g_bcsr, g_csr, remap) * 4 + w; wave < waves;
                 wave += (int64_t)g_csr * 4)
                csr_wave<TV, TB, TC, VEC, LPR, (sizeof(TV) == 2 && LPR <= 8 ? HSPMM_CSR_U_NARROW : HSPMM_CSR_U)>(
                    ca, da, wave);
        }
    }
}

// Sum of the partial rows of split CSR rows.  A workgroup takes one long
// row and a chunk of up to 64*V columns; lanes form groups of L lanes (V
// columns each) that cover the chunk, and group g adds the row's partials
// g, g + NG, g + 2 NG, ... (NG = BT / L groups, RU loads in flight each).
// The group sums are then added in group order through LDS: the order is
// fixed by (cnt, L, BT), so repeated runs give identical results.  Rows cut
// into hundreds of segments are summed by many waves at once instead of one
// lane walking every partial in turn.
template <class TC, class Acc, int V, int BT>
__global__ __launch_bounds__(BT) void k_long_reduce(const int32_t* __restrict__ long_row,
                                                    const int32_t* __restrict__ long_first,
                                                    const int32_t* __restrict__ long_cnt,
                                                    const Acc* __restrict__ ws, TC* __restrict__ C,
                                                    int64_t ldc, int64_t n, int L,
                                                    const double* __restrict__ scale) {
    constexpr int RU = 4;
    __shared__ Acc red[BT * V];
    const int t = threadIdx.x;
    const int NG = BT / L, g = t / L, gl = t % L;
    const int64_t col = (int64_t)blockIdx.y * 64 * V + (int64_t)gl * V;
    const bool colok = col < n;
    const int64_t w = blockIdx.x;
    const int row = long_row[w], first = long_first[w], cnt = long_cnt[w];
    Acc acc[RU][V];
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[u][v] = Acc(0);
    if (colok) {
        for (int q0 = g; q0 < cnt; q0 += NG * RU) {
            Acc x[RU][V];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int q = q0 + u * NG;
                if (q < cnt) {
                    load_vec<Acc, V>(ws + (int64_t)(first + q) * n + col, x[u]);
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) x[u][v] = Acc(0);
                }
            }
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) acc[u][v] += x[u][v];
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) red[t * V + v] = ((acc[0][v] + acc[1][v]) + acc[2][v]) + acc[3][v];
    __syncthreads();
    if (g == 0 && colok) {
        Acc sum[V];
#pragma unroll
        for (int v = 0; v < V; ++v) sum[v] = red[gl * V + v];
        for (int h = 1; h < NG; ++h)
#pragma unroll
            for (int v = 0; v < V; ++v) sum[v] += red[(h * L + gl) * V + v];
        const Acc sc = scale ? (Acc)scale[row >> 4] : Acc(1);
#pragma unroll
        for (int v = 0; v < V; ++v) C[(int64_t)row * ldc + col + v] = (TC)(sum[v] * sc);
    }
}

// Launch of the reduction above: V columns per lane when the partial rows
// allow 16-byte loads, and 1024 threads when, at 256, the longest row would
// leave more than 8 partials to each lane group (256 / L groups): a row of
// 490 partials at n = 256 needs the extra groups, while rows of at most 79
// at n = 64 FP16 keep 256 (power law forward's reduction 38 -> 9 us).
template <class TC, class Acc>
void launch_long_reduce(const SubPlan& X, const DenseArgs& d, hipStream_t s) {
    constexpr int VW = 16 / (int)sizeof(Acc);
    const bool vec = d.n % VW == 0 && (uintptr_t)d.ws % 16 == 0;
    const int V = vec ? VW : 1;
    int L = 1;
    while (L < 64 && (int64_t)L * V < d.n) L <<= 1;
    const dim3 grid((unsigned)X.n_long, (unsigned)ceil_div(d.n, (int64_t)64 * V));
    const bool big = (int64_t)X.max_long_cnt * L > 8 * 256;
    const Acc* ws = static_cast<const Acc*>(d.ws);
    TC* C = static_cast<TC*>(d.C);
#define HSPMM_LR(VV, BB)                                                                                     \
    HSPMM_LAUNCH((k_long_reduce<TC, Acc, VV, BB>), grid, dim3(BB), 0, s, false, true, X.long_row.as<int32_t>(), \
                 X.long_first.as<int32_t>(), X.long_cnt.as<int32_t>(), ws, C, d.ldc, d.n, L, d.scale)
    if (vec) {
        if (big) HSPMM_LR(VW, 1024); else HSPMM_LR(VW, 256);
    } else {
        if (big) HSPMM_LR(1, 1024); else HSPMM_LR(1, 256);
    }
#undef HSPMM_LR
}

inline uint32_t pad8(int64_t g) { return (uint32_t)(ceil_div(g, 8) * 8); }

// 1 (default): grouped BCSR-parts run the LDS-staged group kernel; 0
// (HSPMM_GROUP_KERNEL=0): the one-wave kernel in group order
int group_kernel_mode() {
    const char* e = getenv("HSPMM_GROUP_KERNEL");
    return (e && e[0] == '0') ? 0 : 1;
}

template <class TV, class TB, class TC, int VEC, int LPR, int BV, int BNL, bool WAVE>
int launch_cfg_w(const SubPlan& X, const DenseArgs& d, hipStream_t s, LaunchQuery* q) {
    CsrArgs ca{X.vr_start.as<int32_t>(), X.vr_end.as<int32_t>(), X.vr_out.as<int32_t>(),
               X.csr_col.as<int32_t>(), X.csr_val.ptr, X.n_vrows};
    constexpr int PANEL = (sizeof(TV) == 2) ? 16 * BV : 16 * BV * BNL;
    const int32_t n_panels = (int32_t)ceil_div(d.n, PANEL);
    // a grouped plan's row blocks in group order: the four waves of a
    // workgroup take neighbouring row blocks of one group
    const bool gord = X.grouped;
    BcsrArgs ba{(gord ? X.kslot_rb : X.bcsr_rb).as<int32_t>(), (gord ? X.kslot_ptr : X.blk_ptr).as<int32_t>(),
                (gord ? X.kslot_cnt : X.blk_cnt).as<int32_t>(), X.blk_col.as<int32_t>(), X.blk_val.ptr, X.rb_bcsr,
                n_panels};
    constexpr int R = 64 / LPR;
    const int64_t csr_waves = ceil_div(X.n_vrows, R);
    const int64_t bcsr_units = X.rb_bcsr * (int64_t)n_panels;
    // a BCSR unit is a workgroup, or a wave (four units per workgroup)
    const int64_t bcsr_wgs = WAVE ? ceil_div(bcsr_units, 4) : bcsr_units;
    uint32_t g_csr = csr_waves ? pad8(ceil_div(csr_waves, 4)) : 0;
    uint32_t g_bcsr = bcsr_units ? pad8(bcsr_wgs) : 0;
    if (g_csr + g_bcsr == 0) return HSPMM_OK;
    // LDS of the workgroup's BCSR reduction: 4 waves x tiles x 4 registers x 64 lanes
    constexpr int TILES = (sizeof(TV) == 2) ? BV : BV * BNL;
    constexpr int TP = TILES >= 2 ? TILES / 2 : 1;
    constexpr size_t ACC_B = (sizeof(TV) == 8) ? 8 : 4;
    const size_t lds = g_bcsr && !WAVE ? (size_t)4 * TP * 4 * 64 * ACC_B : 0;
    // the BCSR-part's workgroups stay resident and stride over the units
    // (the next unit's metadata is fetched while the current one runs):
    // cap the part at what the GPU holds at once
    if (g_bcsr && !q && !WAVE && bcsr_persistent()) {
        static int resident = -1;  // per kernel instantiation
        if (resident < 0) {
            int nb = 0, dev = 0, cus = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &nb, reinterpret_cast<const void*>(&k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, false, true, WAVE>),
                    256, lds) != hipSuccess)
                nb = 0;
            resident = nb > 0 ? nb * cus : 0;
        }
        if (resident > 0 && (int64_t)g_bcsr > resident) g_bcsr = pad8(resident);
    }
    // calibrated partition (Eq. 3 analogue): caps on each part's workgroups
    if (X.part_csr > 0 && g_csr > (uint32_t)X.part_csr) g_csr = pad8(X.part_csr);
    if (X.part_bcsr > 0 && g_bcsr > (uint32_t)X.part_bcsr) g_bcsr = pad8(X.part_bcsr);
    if (q) {
        // geometry of the default launch and how many of its workgroups fit on a CU
        q->g_csr = csr_waves ? pad8(ceil_div(csr_waves, 4)) : 0;
        q->g_bcsr = bcsr_units ? pad8(bcsr_wgs) : 0;
        int nb = 0;
        hipError_t e;
        if (q->g_bcsr && q->g_csr)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void*>(&k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, true, true, WAVE>), 256,
                lds);
        else if (q->g_csr)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void*>(&k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, true, false, false>), 256,
                0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void*>(&k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, false, true, WAVE>), 256,
                lds);
        HIP_TRY(e);
        q->wg_per_cu = nb;
        return HSPMM_OK;
    }
    const dim3 grid(g_bcsr + g_csr), block(256);
    const int rm = xcd_remap_mode();
    const bool last = X.n_long == 0;  // no reduction kernel follows
    if (g_bcsr && g_csr && hybrid_launch_mode() == 2) {
        // the two parts as two kernels, each with its own register budget
        HSPMM_LAUNCH((k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, false, true, WAVE>), dim3(g_bcsr), block, lds, s, true,
                     false, ca, ba, d, g_bcsr, 0u, rm);
        HIP_LAUNCH_CHECK();
        HSPMM_LAUNCH((k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, true, false, false>), dim3(g_csr), block, 0, s, false,
                     last, ca, ba, d, 0u, g_csr, rm);
    } else if (g_bcsr && g_csr) {
        HSPMM_LAUNCH((k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, true, true, WAVE>), grid, block, lds, s, true, last, ca,
                     ba, d, g_bcsr, g_csr, rm);
    } else if (g_csr) {
        HSPMM_LAUNCH((k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, true, false, false>), grid, block, 0, s, true, last, ca,
                     ba, d, g_bcsr, g_csr, rm);
    } else {
        HSPMM_LAUNCH((k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, false, true, WAVE>), grid, block, lds, s, true, last, ca,
                     ba, d, g_bcsr, g_csr, rm);
    }
    HIP_LAUNCH_CHECK();
    if (X.n_long > 0) {
        typedef typename Elem<TB>::acc_t acc_t;
        launch_long_reduce<TC, acc_t>(X, d, s);
        HIP_LAUNCH_CHECK();
    }
    return HSPMM_OK;
}

// A grouped BCSR-part (FP32 / FP64 with 16-byte rows of B and C): the
// group kernel for it, the CSR-part (if any) as its own launch, then the
// reduction of split CSR rows.
template <class TV, class TB, class TC, int VEC, int LPR, int BV, int BNL>
int launch_grouped(const SubPlan& X, const DenseArgs& d, hipStream_t s, LaunchQuery* q) {
    constexpr int PANEL = 16 * BV;
    const int32_t n_panels = (int32_t)ceil_div(d.n, PANEL);
    GroupArgs ga{X.kslot_rb.as<int32_t>(), X.kslot_ptr.as<int32_t>(), X.kslot_cnt.as<int32_t>(),
                 X.grp_ptr.as<int32_t>(), X.grp_uptr.as<int32_t>(), X.grp_ucol.as<int32_t>(),
                 X.blk_bsrc.as<int32_t>(), X.blk_val.ptr, X.ngroups, n_panels};
    CsrArgs ca{X.vr_start.as<int32_t>(), X.vr_end.as<int32_t>(), X.vr_out.as<int32_t>(),
               X.csr_col.as<int32_t>(), X.csr_val.ptr, X.n_vrows};
    BcsrArgs ba{};
    constexpr int R = 64 / LPR;
    const int64_t csr_waves = ceil_div(X.n_vrows, R);
    uint32_t g_csr = csr_waves ? pad8(ceil_div(csr_waves, 4)) : 0;
    const int64_t units = X.ngroups * (int64_t)n_panels;
    uint32_t g_grp = units ? pad8(units) : 0;
    // the stage, the up to three rows a wave's last copy may run past it,
    // and the stage's column indices
    const size_t lds = (size_t)(X.grp_max_u + 4) * kGroupRowBytes + (size_t)std::max<int64_t>(1, X.grp_max_u) * 4;
    if (X.part_csr > 0 && g_csr > (uint32_t)X.part_csr) g_csr = pad8(X.part_csr);
    if (X.part_bcsr > 0 && g_grp > (uint32_t)X.part_bcsr) g_grp = pad8(X.part_bcsr);
    if (q) {
        q->g_csr = csr_waves ? pad8(ceil_div(csr_waves, 4)) : 0;
        q->g_bcsr = units ? pad8(units) : 0;
        int nb = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(&k_bcsr_group<TV, BV>), 256, lds));
        q->wg_per_cu = nb;
        return HSPMM_OK;
    }
    const int rm = xcd_remap_mode();
    if (g_grp) {
        HSPMM_LAUNCH((k_bcsr_group<TV, BV>), dim3(g_grp), dim3(256), lds, s, true, !g_csr && !X.n_long, ga, d, g_grp,
                     rm, (int)X.grp_max_u);
        HIP_LAUNCH_CHECK();
    }
    if (g_csr) {
        HSPMM_LAUNCH((k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL, true, false, false>), dim3(g_csr), dim3(256), 0, s,
                     !g_grp, !X.n_long, ca, ba, d, 0u, g_csr, rm);
        HIP_LAUNCH_CHECK();
    }
    if (X.n_long > 0) {
        typedef typename Elem<TB>::acc_t acc_t;
        launch_long_reduce<TC, acc_t>(X, d, s);
        HIP_LAUNCH_CHECK();
    }
    return HSPMM_OK;
}

// BCSR-parts whose row blocks are all short run one wave per row block
// The FP16 / BF16 one-wave form holds 3-4 waves per SIMD; a fused launch
// with a large CSR-part is held there too, which costs the CSR-part more
// than the form gains (stencil FP16 with half the rows in the CSR-part:
// 51 -> 57 us), so FP16 / BF16 take it only when the CSR-part is at most a
// quarter of the entries (BCSR-only forward 26.5 -> 21.5 us).
template <class TV, class TB, class TC, int VEC, int LPR, int BV, int BNL>
int launch_cfg(const SubPlan& X, const DenseArgs& d, hipStream_t s, LaunchQuery* q) {
    if constexpr (sizeof(TV) != 2 && BV * sizeof(TV) == 16) {
        if (X.grouped && X.rb_bcsr > 0 && group_kernel_mode())
            return launch_grouped<TV, TB, TC, VEC, LPR, BV, BNL>(X, d, s, q);
    }
    const bool wave_ok = sizeof(TV) != 2 || 3 * X.nnz_csr <= X.nnz_bcsr;
    if (X.rb_bcsr > 0 && X.max_rb_tiles <= kWaveMaxTiles && wave_ok)
        return launch_cfg_w<TV, TB, TC, VEC, LPR, BV, BNL, true>(X, d, s, q);
    return launch_cfg_w<TV, TB, TC, VEC, LPR, BV, BNL, false>(X, d, s, q);
}

inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// lanes per CSR row for n columns at VEC per lane (power of two, 4..64)
inline int lpr_for(int64_t n, int vec) {
    int64_t need = ceil_div(n, vec);
    int l = 4;
    while (l < 64 && l < need) l <<= 1;
    return l;
}

#define HSPMM_LPR_SWITCH(LPRV, ...)                      \
    switch (LPRV) {                                      \
        case 4: { constexpr int LPR = 4; __VA_ARGS__; } break;   \
        case 8: { constexpr int LPR = 8; __VA_ARGS__; } break;   \
        case 16: { constexpr int LPR = 16; __VA_ARGS__; } break; \
        case 32: { constexpr int LPR = 32; __VA_ARGS__; } break; \
        default: { constexpr int LPR = 64; __VA_ARGS__; } break; \
    }

template <class TV, class TB, class TC>
int dispatch_dtype(const SubPlan& X, const DenseArgs& d, bool vec_ok, hipStream_t s, LaunchQuery* q);

// FP32: VEC 4 (16-byte loads) when n, ld and pointers allow, else scalar
template <>
int dispatch_dtype<float, float, float>(const SubPlan& X, const DenseArgs& d, bool vec_ok, hipStream_t s,
                                        LaunchQuery* q) {
    if (vec_ok) {
        const int lpr = lpr_for(d.n, 4);
        // BCSR panel of 128 columns per wave (NL = 2); NL = 1 (64 columns,
        // twice the waves, each at 8 per SIMD) measured no faster on the
        // block stencil n = 128 (forward 36.8 against 36.4 us cold)
#ifndef HSPMM_F32_NL
#define HSPMM_F32_NL 2
#endif
        if (d.n <= 64) {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<float, float, float, 4, LPR, 4, 1>(X, d, s, q)));
        } else if (HSPMM_F32_CSR_VEC8 && d.n % 8 == 0) {
            HSPMM_LPR_SWITCH(lpr_for(d.n, 8),
                             return (launch_cfg<float, float, float, 8, LPR, 4, HSPMM_F32_NL>(X, d, s, q)));
        } else {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<float, float, float, 4, LPR, 4, HSPMM_F32_NL>(X, d, s, q)));
        }
    }
    return launch_cfg<float, float, float, 1, 64, 1, 4>(X, d, s, q);
}

template <>
int dispatch_dtype<double, double, double>(const SubPlan& X, const DenseArgs& d, bool vec_ok, hipStream_t s,
                                           LaunchQuery* q) {
    if (vec_ok) {
        const int lpr = lpr_for(d.n, 2);
        if (d.n <= 32) {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<double, double, double, 2, LPR, 2, 1>(X, d, s, q)));
        } else {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<double, double, double, 2, LPR, 2, 2>(X, d, s, q)));
        }
    }
    return launch_cfg<double, double, double, 1, 64, 1, 4>(X, d, s, q);
}

template <class TH>
int dispatch_half(const SubPlan& X, const DenseArgs& d, bool vec_ok, hipStream_t s, LaunchQuery* q) {
    if (vec_ok) {
        const int lpr = lpr_for(d.n, 8);
        if (d.n <= 64) {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<TH, TH, float, 8, LPR, 4, 1>(X, d, s, q)));
        } else {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<TH, TH, float, 8, LPR, 8, 1>(X, d, s, q)));
        }
    }
    return launch_cfg<TH, TH, float, 1, 64, 1, 1>(X, d, s, q);
}

}  // namespace

// widest n of the fused backward: FP32 four waves (BCSR-part) or 64 lanes
// (CSR-part) of 16-byte segments, FP64 the same at half the columns
inline int64_t bwd_max_n(int ct) { return ct == HSPMM_F64 ? 128 : 256; }

bool bwd_fusable(const Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc,
                 const void* dB, int64_t lddb) {
    if (!bwd_fused_mode() || !p.has_T || n <= 0) return false;
    const SubPlan& T = p.T;
    const bool has_b = T.rb_bcsr > 0, has_c = T.n_vrows > 0;
    if (T.scaled || (!has_b && !has_c)) return false;
    const int64_t vec = T.ct == HSPMM_F64 ? 2 : 4;  // elements of dC in 16 bytes
    if (n > bwd_max_n(T.ct) || n % vec != 0 || ldb % vec != 0 || lddc % vec != 0 || lddb % vec != 0 ||
        !aligned(dC, 16) || !aligned(dB, 16))
        return false;
    // the BCSR-part form holds B's rows in the compute type of its MFMAs:
    // FP32 / FP64 plans only, with 16-byte rows
    if (has_b && (p.compute != T.ct || !T.tile_base.ptr || T.max_rb_tiles > kWaveMaxTiles || !aligned(B, 16)))
        return false;
    // the CSR-part form saves the SDDMM's gather of a row of B per entry
    // but writes each entry's dA on its own (the entries of a row of A^T
    // lie in different rows of A) and adds a reduction across the lane
    // group: measured (backward, us, fused / separate) GCN FP32 n = 64
    // 543 / 671, n = 128 823 / 1336, FP16 n = 128 830 / 1007; power law
    // FP32 n = 64 991 / 1150, FP16 n = 128 1511 / 1726, but FP16 n = 64
    // (rows of 128 bytes) 991 / 921: it is taken from 256-byte rows of B
    if (has_c && n * (int64_t)dtype_size(p.compute) < 256) return false;
    return aligned(B, (size_t)vec * dtype_size(p.compute));
}

namespace {
template <class T, int NW>
int launch_bwd_cs(Plan& p, int64_t n, const void* B, int64_t ldb, const DenseArgs& da, void* dA, hipStream_t s,
                  bool first, bool last) {
    constexpr int VEC = 16 / (int)sizeof(T);
    const SubPlan& X = p.T;
    BcsrArgs ba{X.bcsr_rb.as<int32_t>(), X.blk_ptr.as<int32_t>(), X.blk_cnt.as<int32_t>(), X.blk_col.as<int32_t>(),
                X.blk_val.ptr, X.rb_bcsr, 1};
    BwdArgs bw{X.tile_base.as<int32_t>(), static_cast<const uint16_t*>(X.tile_mask.ptr), B, ldb, p.k, dA};
    const uint32_t g = pad8(X.rb_bcsr);
    const size_t lds = BwdCs<T, NW, VEC>::kLds;
    HSPMM_LAUNCH((k_bwd_cs<T, NW, VEC>), dim3(g), dim3(64 * NW), lds, s, first, last, ba, da, bw, g,
                 xcd_remap_mode());
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}

template <class TB, class TG>
int launch_bwd_csr(Plan& p, int64_t n, const void* B, int64_t ldb, const DenseArgs& da, void* dA, hipStream_t s,
                   bool first, bool last) {
    constexpr int VEC = 16 / (int)sizeof(TG);
    const SubPlan& X = p.T;
    CsrBwdArgs ca{X.vr_start.as<int32_t>(), X.vr_end.as<int32_t>(), X.vr_out.as<int32_t>(), X.vr_row.as<int32_t>(),
                  X.csr_col.as<int32_t>(), X.csr_val.ptr, X.csr_src.as<int32_t>(), X.n_vrows, B, ldb, dA};
    const int rm = xcd_remap_mode();
    HSPMM_LPR_SWITCH(lpr_for(n, VEC), {
        constexpr int R = 64 / LPR;
        const uint32_t g = pad8(ceil_div(ceil_div(X.n_vrows, R), 4));
        HSPMM_LAUNCH((k_bwd_csr<TB, TG, VEC, LPR>), dim3(g), dim3(256), 0, s, first, last, ca, da, g, rm);
    });
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}

template <class TB, class TG>
int launch_bwd_parts(Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc, void* dB,
                     int64_t lddb, void* dA, hipStream_t s, bool last) {
    SubPlan& X = p.T;
    // partial rows of split CSR rows of A^T (every slot written before the
    // reduction reads it)
    void* ws = nullptr;
    if (X.n_partials > 0) {
        HSPMM_TRY(ensure_ws(p, forward_scratch_bytes(X, n)));
        ws = p.ws.ptr;
    }
    DenseArgs da{dC, lddc, dB, lddb, n, X.m, ws, nullptr};
    const bool has_b = X.rb_bcsr > 0, has_c = X.n_vrows > 0, has_l = X.n_long > 0;
    if (has_b) {
        if constexpr (std::is_same<TB, TG>::value) {
            // two waves while n fits their panel (more waves per SIMD), else four
            const bool two = n <= 2 * 16 * (16 / (int64_t)sizeof(TG));
            const bool l = last && !has_c && !has_l;
            const int rc = two ? launch_bwd_cs<TG, 2>(p, n, B, ldb, da, dA, s, true, l)
                               : launch_bwd_cs<TG, 4>(p, n, B, ldb, da, dA, s, true, l);
            HSPMM_TRY(rc);
        } else {
            return fail(HSPMM_ERR_ARG, "fused backward: BCSR-part of a low-precision plan");
        }
    }
    if (has_c) {
        const int rc = launch_bwd_csr<TB, TG>(p, n, B, ldb, da, dA, s, !has_b, last && !has_l);
        HSPMM_TRY(rc);
    }
    if (has_l) {
        launch_long_reduce<TG, TG>(X, da, s);
        HIP_LAUNCH_CHECK();
    }
    return HSPMM_OK;
}
}  // namespace

int launch_bwd_fused_kernel(Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc,
                            void* dB, int64_t lddb, void* dA_canon, hipStream_t s, bool last) {
    switch (p.compute) {
        case HSPMM_F64: return launch_bwd_parts<double, double>(p, n, B, ldb, dC, lddc, dB, lddb, dA_canon, s, last);
        case HSPMM_F32: return launch_bwd_parts<float, float>(p, n, B, ldb, dC, lddc, dB, lddb, dA_canon, s, last);
        case HSPMM_F16: return launch_bwd_parts<half_t, float>(p, n, B, ldb, dC, lddc, dB, lddb, dA_canon, s, last);
        case HSPMM_BF16: return launch_bwd_parts<bf16_t, float>(p, n, B, ldb, dC, lddc, dB, lddb, dA_canon, s, last);
        default: return fail(HSPMM_ERR_DTYPE, "bad compute dtype");
    }
}

size_t forward_scratch_bytes(const SubPlan& X, int64_t n) {
    const size_t acc_b = X.ct == HSPMM_F64 ? 8 : 4;
    return (size_t)X.n_partials * (size_t)n * acc_b;
}

int launch_forward(Plan& p, SubPlan& X, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc,
                   hipStream_t s, LaunchQuery* q, const Workspace* ext) {
    if (X.m == 0 || n == 0) {
        if (q) *q = LaunchQuery{};
        return HSPMM_OK;
    }
    const size_t eb = dtype_size(X.ct);
    const size_t ec = dtype_size(out_dtype(X.ct));
    // partial rows of split CSR rows: every slot is written by its segment
    // before the reduction reads it, so the scratch needs no clearing
    void* ws = nullptr;
    if (X.n_partials > 0) {
        const size_t need = forward_scratch_bytes(X, n);
        if (ext) {
            if (need > ext->bytes)
                return fail(HSPMM_ERR_OOM, "split rows need " + std::to_string(need) +
                                               " bytes of scratch at this n; the static scratch holds " +
                                               std::to_string(ext->bytes));
            ws = ext->ptr;
        } else {
            HSPMM_TRY(ensure_ws(p, need));
            ws = p.ws.ptr;
        }
    }
    DenseArgs d{B, ldb, C, ldc, n, X.m, ws, X.scaled ? X.scale.as<double>() : nullptr};
    const int vec_elems = (int)(16 / eb);
    // every lane must be able to issue full 16-byte loads of B and the
    // matching stores of C
    const bool vec_ok = (n % vec_elems == 0) && (ldb % vec_elems == 0) && (ldc % vec_elems == 0) &&
                        aligned(B, 16) && aligned(C, 16) && (ec * vec_elems) % 16 == 0;
    switch (X.ct) {
        case HSPMM_F32: return dispatch_dtype<float, float, float>(X, d, vec_ok, s, q);
        case HSPMM_F64: return dispatch_dtype<double, double, double>(X, d, vec_ok, s, q);
        case HSPMM_F16: return dispatch_half<half_t>(X, d, vec_ok, s, q);
        case HSPMM_BF16: return dispatch_half<bf16_t>(X, d, vec_ok, s, q);
        default: return fail(HSPMM_ERR_DTYPE, "unsupported compute dtype");
    }
}

}  // namespace hspmm
