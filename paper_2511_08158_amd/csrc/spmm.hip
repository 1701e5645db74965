// Forward kernels: C = X * B for one sub-plan, both parts in one launch.
//
// CSR-part (the AXPY kernel of Sec. 3.3): a wavefront serves 64/LPR virtual
// rows, LPR lanes per row, each lane owning VEC consecutive columns of C.
// The row's (column, value) pairs are fetched once, coalesced, one entry
// per lane, and broadcast inside the lane group; every entry then costs one
// coalesced VEC-wide load of a B row segment and VEC FMAs.
//
// BCSR-part (the outer-product kernel of Sec. 3.3, Alg. 2-3): a wavefront
// owns one 16-row block and one column panel of C.  Each MFMA step takes
// kc tiles of the block (a 16 x kc slab of A, packed in lane order at plan
// time) and the kc gathered B rows, so every gathered B row serves 16 rows
// of C.  FP64/FP32 use 16x16x4 MFMAs (kc = 4); FP16/BF16 use 16x16x32
// MFMAs (kc = 32, the widening accumulate of Alg. 3, with FP32 sums).
// Partial K steps are zero-filled, as Alg. 3 pairs an odd tile with zeros.
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
    if constexpr (N == 1) {
        out[0] = *p;
    } else {
        typedef T V __attribute__((ext_vector_type(N)));
        const V v = *reinterpret_cast<const V*>(p);
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = v[i];
    }
}

// stores of up to 16 bytes per instruction (callers guarantee 16-byte
// alignment of every chunk)
template <class T, int N>
__device__ inline void store_vec(T* p, const T (&in)[N]) {
    constexpr int C = (N * (int)sizeof(T) > 16) ? 16 / (int)sizeof(T) : N;
    if constexpr (C == 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) p[i] = in[i];
    } else {
        typedef T V __attribute__((ext_vector_type(C)));
#pragma unroll
        for (int q = 0; q < N; q += C) {
            V v;
#pragma unroll
            for (int i = 0; i < C; ++i) v[i] = in[q + i];
            *reinterpret_cast<V*>(p + q) = v;
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
                TB bv[U][VEC];
#pragma unroll
                for (int uu = 0; uu < U; ++uu) {
                    if (cc[uu] >= 0 && colok && u0 + uu < cnt) {
                        load_vec<TB, VEC>(B + (int64_t)cc[uu] * d.ldb + col0, bv[uu]);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v) bv[uu][v] = TB(0);
                    }
                }
#pragma unroll
                for (int uu = 0; uu < U; ++uu)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[v] += vv[uu] * Elem<TB>::to_acc(bv[uu][v]);
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

template <class T, int VEC, int NL>
__device__ void bcsr_wave_f(const BcsrArgs& a, const DenseArgs& d, int64_t wave) {
    typedef typename AccOf<T>::type acc_v;
    constexpr int PANEL = 16 * VEC * NL;
    constexpr int TILES = VEC * NL;
    const int64_t slot = wave / a.n_panels;
    if (slot >= a.n_rb) return;  // wave-uniform
    const int panel = (int)(wave - slot * a.n_panels);
    const int lane = threadIdx.x & 63, j = lane & 15, kq = lane >> 4;
    const int rb = a.rb[slot];
    const int b0 = a.blk_ptr[slot];
    const int cnt = a.blk_cnt[slot];
    const int64_t cbase = (int64_t)panel * PANEL + (int64_t)j * VEC;
    const T* __restrict__ vals = static_cast<const T*>(a.val);
    const T* __restrict__ B = static_cast<const T*>(d.B);
    acc_v acc[TILES];
#pragma unroll
    for (int t = 0; t < TILES; ++t) acc[t] = acc_v{0, 0, 0, 0};

    for (int c = 0; c < cnt; c += 8) {
        // two K steps in flight
        T av[2];
        T bv[2][NL][VEC];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int kk = c + 4 * s + kq;
            const bool ok = kk < cnt;
            av[s] = (c + 4 * s < cnt) ? vals[(int64_t)(b0 + c + 4 * s) * 16 + lane] : T(0);
            const int bc = ok ? a.blk_col[b0 + kk] : 0;
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                const int64_t col = cbase + (int64_t)h * 16 * VEC;
                if (ok && col < d.n) {
                    load_vec<T, VEC>(B + (int64_t)bc * d.ldb + col, bv[s][h]);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) bv[s][h][v] = T(0);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int h = 0; h < NL; ++h)
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[h * VEC + v] = mfma4(av[s], bv[s][h][v], acc[h * VEC + v]);
    }
    const T sc = d.scale ? (T)d.scale[rb] : T(1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = (int64_t)rb * 16 + out_row<T>(kq, r);
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

template <class T, int CPL>
__device__ void bcsr_wave_h(const BcsrArgs& a, const DenseArgs& d, int64_t wave) {
    typedef typename V8Of<T>::type v8;
    constexpr int PANEL = 16 * CPL;
    const int64_t slot = wave / a.n_panels;
    if (slot >= a.n_rb) return;
    const int panel = (int)(wave - slot * a.n_panels);
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
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

    for (int c = 0; c < cnt; c += 32) {
        const v8 av = *reinterpret_cast<const v8*>(vals + ((int64_t)(b0 + c) * 16 + lane * 8));
        T raw[8][CPL];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int kk = c + 8 * g + u;
            const bool ok = kk < cnt && colok;
            const int bc = ok ? a.blk_col[b0 + kk] : 0;
            if (ok) {
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
    const float sc = d.scale ? (float)d.scale[rb] : 1.0f;
    if (!colok) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = (int64_t)rb * 16 + 4 * g + r;
        if (row >= d.m) continue;
        float o[CPL];
#pragma unroll
        for (int t = 0; t < CPL; ++t) o[t] = acc[t][r] * sc;
        float* dst = static_cast<float*>(d.C) + row * d.ldc + cbase;
        if constexpr (CPL >= 4) {
#pragma unroll
            for (int q = 0; q < CPL; q += 4) {
                float4 w = make_float4(o[q], o[q + 1], o[q + 2], o[q + 3]);
                *reinterpret_cast<float4*>(dst + q) = w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < CPL; ++t) dst[t] = o[t];
        }
    }
}

// ---------------------------------------------------------------------------
// fused launch: workgroups [0, g_bcsr) run the BCSR-part, the rest the CSR-part
// ---------------------------------------------------------------------------
template <class TV, class TB, class TC, int VEC, int LPR, int BV, int BNL>
__global__ __launch_bounds__(256) void k_hybrid(CsrArgs ca, BcsrArgs ba, DenseArgs da, uint32_t g_bcsr,
                                                uint32_t g_csr) {
    const uint32_t bid = blockIdx.x;
    const int w = threadIdx.x >> 6;
    if (bid < g_bcsr) {
        const int64_t wave = (int64_t)xcd_remap(bid, g_bcsr) * 4 + w;
        if constexpr (sizeof(TV) == 2) {
            bcsr_wave_h<TV, BV>(ba, da, wave);
        } else {
            bcsr_wave_f<TV, BV, BNL>(ba, da, wave);
        }
    } else {
        const int64_t wave = (int64_t)xcd_remap(bid - g_bcsr, g_csr) * 4 + w;
        csr_wave<TV, TB, TC, VEC, LPR, 8>(ca, da, wave);
    }
}

template <class TC, class Acc>
__global__ __launch_bounds__(256) void k_long_reduce(const int32_t* __restrict__ long_row,
                                                     const int32_t* __restrict__ long_first,
                                                     const int32_t* __restrict__ long_cnt, int64_t n_long,
                                                     const Acc* __restrict__ ws, TC* __restrict__ C,
                                                     int64_t ldc, int64_t n, const double* __restrict__ scale) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= n_long) return;
    const int row = long_row[w], first = long_first[w], cnt = long_cnt[w];
    const Acc s = scale ? (Acc)scale[row >> 4] : Acc(1);
    for (int64_t c = lane; c < n; c += 64) {
        Acc sum = Acc(0);
        for (int q = 0; q < cnt; ++q) sum += ws[(int64_t)(first + q) * n + c];
        C[(int64_t)row * ldc + c] = (TC)(sum * s);
    }
}

inline uint32_t pad8(int64_t g) { return (uint32_t)(ceil_div(g, 8) * 8); }

template <class TV, class TB, class TC, int VEC, int LPR, int BV, int BNL>
int launch_cfg(const SubPlan& X, const DenseArgs& d, hipStream_t s) {
    CsrArgs ca{X.vr_start.as<int32_t>(), X.vr_end.as<int32_t>(), X.vr_out.as<int32_t>(),
               X.csr_col.as<int32_t>(), X.csr_val.ptr, X.n_vrows};
    constexpr int PANEL = (sizeof(TV) == 2) ? 16 * BV : 16 * BV * BNL;
    const int32_t n_panels = (int32_t)ceil_div(d.n, PANEL);
    BcsrArgs ba{X.bcsr_rb.as<int32_t>(), X.blk_ptr.as<int32_t>(), X.blk_cnt.as<int32_t>(),
                X.blk_col.as<int32_t>(), X.blk_val.ptr, X.rb_bcsr, n_panels};
    constexpr int R = 64 / LPR;
    const int64_t csr_waves = ceil_div(X.n_vrows, R);
    const int64_t bcsr_waves = X.rb_bcsr * (int64_t)n_panels;
    const uint32_t g_csr = csr_waves ? pad8(ceil_div(csr_waves, 4)) : 0;
    const uint32_t g_bcsr = bcsr_waves ? pad8(ceil_div(bcsr_waves, 4)) : 0;
    if (g_csr + g_bcsr == 0) return HSPMM_OK;
    hipLaunchKernelGGL((k_hybrid<TV, TB, TC, VEC, LPR, BV, BNL>), dim3(g_bcsr + g_csr), dim3(256), 0, s, ca, ba,
                       d, g_bcsr, g_csr);
    HIP_LAUNCH_CHECK();
    if (X.n_long > 0) {
        typedef typename Elem<TB>::acc_t acc_t;
        const unsigned blocks = (unsigned)ceil_div(X.n_long, 4);
        hipLaunchKernelGGL((k_long_reduce<TC, acc_t>), dim3(blocks), dim3(256), 0, s, X.long_row.as<int32_t>(),
                           X.long_first.as<int32_t>(), X.long_cnt.as<int32_t>(), X.n_long,
                           static_cast<const acc_t*>(d.ws), static_cast<TC*>(d.C), d.ldc, d.n, d.scale);
        HIP_LAUNCH_CHECK();
    }
    return HSPMM_OK;
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
int dispatch_dtype(const SubPlan& X, const DenseArgs& d, bool vec_ok, hipStream_t s);

// FP32: VEC 4 (16-byte loads) when n, ld and pointers allow, else scalar
template <>
int dispatch_dtype<float, float, float>(const SubPlan& X, const DenseArgs& d, bool vec_ok, hipStream_t s) {
    if (vec_ok) {
        const int lpr = lpr_for(d.n, 4);
        if (d.n <= 64) {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<float, float, float, 4, LPR, 4, 1>(X, d, s)));
        } else {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<float, float, float, 4, LPR, 4, 2>(X, d, s)));
        }
    }
    return launch_cfg<float, float, float, 1, 64, 1, 4>(X, d, s);
}

template <>
int dispatch_dtype<double, double, double>(const SubPlan& X, const DenseArgs& d, bool vec_ok, hipStream_t s) {
    if (vec_ok) {
        const int lpr = lpr_for(d.n, 2);
        if (d.n <= 32) {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<double, double, double, 2, LPR, 2, 1>(X, d, s)));
        } else {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<double, double, double, 2, LPR, 2, 2>(X, d, s)));
        }
    }
    return launch_cfg<double, double, double, 1, 64, 1, 4>(X, d, s);
}

template <class TH>
int dispatch_half(const SubPlan& X, const DenseArgs& d, bool vec_ok, hipStream_t s) {
    if (vec_ok) {
        const int lpr = lpr_for(d.n, 8);
        if (d.n <= 64) {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<TH, TH, float, 8, LPR, 4, 1>(X, d, s)));
        } else {
            HSPMM_LPR_SWITCH(lpr, return (launch_cfg<TH, TH, float, 8, LPR, 8, 1>(X, d, s)));
        }
    }
    return launch_cfg<TH, TH, float, 1, 64, 1, 1>(X, d, s);
}

}  // namespace

int launch_forward(Plan& p, SubPlan& X, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc,
                   hipStream_t s) {
    if (X.m == 0 || n == 0) return HSPMM_OK;
    const size_t eb = dtype_size(X.ct);
    const size_t ec = dtype_size(out_dtype(X.ct));
    // partial rows of split CSR rows
    if (X.n_partials > 0) {
        const size_t acc_b = X.ct == HSPMM_F64 ? 8 : 4;
        HSPMM_TRY(ensure_ws(p, (size_t)X.n_partials * (size_t)n * acc_b));
    }
    DenseArgs d{B, ldb, C, ldc, n, X.m, p.ws.ptr, X.scaled ? X.scale.as<double>() : nullptr};
    const int vec_elems = (int)(16 / eb);
    // every lane must be able to issue full 16-byte loads of B and the
    // matching stores of C
    const bool vec_ok = (n % vec_elems == 0) && (ldb % vec_elems == 0) && (ldc % vec_elems == 0) &&
                        aligned(B, 16) && aligned(C, 16) && (ec * vec_elems) % 16 == 0;
    switch (X.ct) {
        case HSPMM_F32: return dispatch_dtype<float, float, float>(X, d, vec_ok, s);
        case HSPMM_F64: return dispatch_dtype<double, double, double>(X, d, vec_ok, s);
        case HSPMM_F16: return dispatch_half<half_t>(X, d, vec_ok, s);
        case HSPMM_BF16: return dispatch_half<bf16_t>(X, d, vec_ok, s);
        default: return fail(HSPMM_ERR_DTYPE, "unsupported compute dtype");
    }
}

}  // namespace hspmm
