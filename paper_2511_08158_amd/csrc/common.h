// Shared definitions of the hspmm HIP library (gfx950 only).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hspmm.h"

namespace hspmm {

// ---------------------------------------------------------------------------
// error handling: every internal step returns a status; the first failure
// records a message for hybrid_spmm_last_error()
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

struct Status {
    int code = HSPMM_OK;
    bool ok() const { return code == HSPMM_OK; }
};

#define HSPMM_TRY(expr)                         \
    do {                                        \
        int _rc = (expr);                       \
        if (_rc != HSPMM_OK) return _rc;        \
    } while (0)

int hip_fail(hipError_t e, const char* what, const char* file, int line);
#define HIP_TRY(expr)                                                    \
    do {                                                                 \
        hipError_t _e = (expr);                                          \
        if (_e != hipSuccess) return hip_fail(_e, #expr, __FILE__, __LINE__); \
    } while (0)
#define HIP_LAUNCH_CHECK() HIP_TRY(hipGetLastError())

int fail(int code, const std::string& msg);

// ---------------------------------------------------------------------------
// device memory owned by a plan
// ---------------------------------------------------------------------------
struct Allocator;

// A device allocation; releasing it (explicitly or at destruction) returns
// its bytes to the allocator that made it.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    Allocator* owner = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), bytes(o.bytes), owner(o.owner) {
        o.ptr = nullptr; o.bytes = 0; o.owner = nullptr;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            ptr = o.ptr; bytes = o.bytes; owner = o.owner;
            o.ptr = nullptr; o.bytes = 0; o.owner = nullptr;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release();
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// Allocation accounting with an optional ceiling (max_workspace_bytes).
// While a plan is built (`keep` set), released buffers are kept and handed
// to later allocations of the build instead of being freed: hipFree waits
// for the device, and all of the build's work is queued on one stream, so a
// buffer reused in stream order needs no wait.  drop_kept() frees them.
struct Allocator {
    uint64_t limit = 0;      // 0 = unlimited
    uint64_t in_use = 0;
    uint64_t peak = 0;
    bool keep = false;
    struct Kept {
        void* ptr;
        size_t bytes;
    };
    std::vector<Kept> kept;
    uint64_t kept_bytes = 0;
    int alloc(DevBuf& b, size_t bytes);
    void free(DevBuf& b) { b.release(); }
    void drop_kept();
};

// Keeps released buffers of `a` for reuse until it goes out of scope, then
// frees them (one wait for the device instead of one per buffer).
struct KeepBuffers {
    Allocator& a;
    explicit KeepBuffers(Allocator& x) : a(x) { a.keep = true; }
    ~KeepBuffers() {
        a.keep = false;
        a.drop_kept();
    }
};

// Wait for the stream before a buffer it uses is released, unless the
// allocator keeps released buffers (stream-ordered reuse needs no wait).
int sync_for_release(const Allocator& a, hipStream_t s);

// ---------------------------------------------------------------------------
// element types
// ---------------------------------------------------------------------------
typedef _Float16 half_t;
typedef __bf16 bf16_t;
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));

inline size_t dtype_size(int dt) {
    switch (dt) {
        case HSPMM_F64: return 8;
        case HSPMM_F32: return 4;
        case HSPMM_F16: return 2;
        case HSPMM_BF16: return 2;
        default: return 0;
    }
}
inline bool dtype_valid(int dt) { return dt >= HSPMM_F64 && dt <= HSPMM_BF16; }
// dtype of C, dB and dA for a compute dtype
inline int out_dtype(int compute) { return compute == HSPMM_F64 ? HSPMM_F64 : HSPMM_F32; }

// ---------------------------------------------------------------------------
// device conversions
// ---------------------------------------------------------------------------
// Round a double to the nearest FP16 / BF16 code, ties to even, straight
// from the 53-bit significand (no intermediate FP32 rounding).
// P = significant bits incl. the hidden one, EMIN = exponent of the
// smallest normal, EBIAS = exponent bias of the target format.
template <int P, int EMIN, int EBITS>
__host__ __device__ inline uint16_t round_double_to_code(double x) {
    uint64_t b;
    memcpy(&b, &x, 8);
    const uint16_t sign = (uint16_t)((b >> 63) << 15);
    const int ebias = (1 << (EBITS - 1)) - 1;
    const uint16_t inf = (uint16_t)(((1u << EBITS) - 1u) << (P - 1));
    int e = (int)((b >> 52) & 0x7ff);
    uint64_t man = b & ((1ull << 52) - 1);
    if (e == 0x7ff) return man ? (uint16_t)(sign | inf | (1u << (P - 2))) : (uint16_t)(sign | inf);
    if (e == 0) return sign;                     // double subnormals are far below any target
    e -= 1023;                                   // x = 1.man * 2^e
    uint64_t sig = (1ull << 52) | man;           // 53 bits
    // target quantum exponent: e - (P-1) for normals, EMIN - (P-1) below
    int qexp = (e >= EMIN ? e : EMIN) - (P - 1);
    int shift = qexp - (e - 52);                 // bits of sig below the quantum
    uint64_t q;
    if (shift >= 64) {
        q = 0;
        // everything is below half a quantum unless shift == 54 exactly... sig < 2^53
        // so x < 2^(qexp-1) -> rounds to zero
    } else {
        q = sig >> shift;
        uint64_t rem = sig & ((1ull << shift) - 1);
        uint64_t half = 1ull << (shift - 1);
        if (rem > half || (rem == half && (q & 1))) q += 1;
    }
    // q is the magnitude in units of 2^qexp; encode
    uint32_t code;
    if (e >= EMIN) {
        // normal: q in [2^(P-1), 2^P]; q == 2^P means the carry bumped the exponent
        int be = e + ebias;
        if (q >> P) { q >>= 1; be += 1; }
        if (be >= (1 << EBITS) - 1) return (uint16_t)(sign | inf);
        code = ((uint32_t)be << (P - 1)) | (uint32_t)(q & ((1ull << (P - 1)) - 1));
    } else {
        // subnormal: q < 2^(P-1), or == 2^(P-1) which is the smallest normal
        code = (uint32_t)q;
    }
    return (uint16_t)(sign | code);
}

__host__ __device__ inline uint16_t double_to_f16_code(double x) { return round_double_to_code<11, -14, 5>(x); }
__host__ __device__ inline uint16_t double_to_bf16_code(double x) { return round_double_to_code<8, -126, 8>(x); }

__device__ inline float bf16_to_float(bf16_t v) {
    uint16_t c;
    memcpy(&c, &v, 2);
    uint32_t u = (uint32_t)c << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// Dense-operand element -> accumulation type
template <class T> struct Elem;
template <> struct Elem<double> {
    typedef double acc_t;
    __device__ static double to_acc(double v) { return v; }
};
template <> struct Elem<float> {
    typedef float acc_t;
    __device__ static float to_acc(float v) { return v; }
};
template <> struct Elem<half_t> {
    typedef float acc_t;
    __device__ static float to_acc(half_t v) { return (float)v; }
};
template <> struct Elem<bf16_t> {
    typedef float acc_t;
    __device__ static float to_acc(bf16_t v) { return bf16_to_float(v); }
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workgroup -> XCD mapping.  The dispatcher hands consecutive workgroups to
// the 8 XCDs in turn; remapping id -> (id % 8) * (G / 8) + id / 8 gives each
// XCD a contiguous range of logical tiles so neighbouring tiles share its L2.
// G must be a multiple of 8 (launchers pad the grid).  mode 0 keeps the
// dispatch order (tuning knob HSPMM_XCD_REMAP=0).
__device__ inline uint32_t xcd_remap(uint32_t id, uint32_t G, int mode) {
    if (!mode) return id;
    const uint32_t per = G >> 3;
    return (id & 7u) * per + (id >> 3);
}
int xcd_remap_mode();

// Index of the calling wave in its workgroup, as a value the compiler knows
// to be uniform over the wave (loops bounded by it stay scalar loops, whose
// memory waits the compiler can count precisely).
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }
// 0 (default): one workgroup per row block of the BCSR-part; 1
// (HSPMM_BCSR_PERSIST=1): resident workgroups that each take a contiguous
// range of row blocks, prefetching the next one's metadata (measured
// slower on the block stencil, kept as a tuning knob).
int bcsr_persistent();
// 0 (default): the backward runs dB then dA on the caller's stream; 1
// (HSPMM_BWD_CONCURRENT=1): dA = SDDMM on a plan-owned side stream beside dB
// (each kernel fills the GPU on large matrices, and the fork/join cost more
// than the overlap gained on the block stencil; kept as a tuning knob).
int bwd_concurrent();
// launch of a plan with both parts: 1 one fused kernel, 2 one kernel per
// part (HSPMM_HYBRID_LAUNCH; read on every call)
int hybrid_launch_mode();
// 1 (default): a backward that qualifies computes dB and dA in one pass over
// A^T's tiles; 0 (HSPMM_BWD_FUSED=0): dB and the SDDMM as separate kernels
// (read on every backward call)
int bwd_fused_mode();

constexpr int kNumXcd = 8;

// Events the caller asked the next products to carry (hybrid_spmm_set_
// timing_events; this thread only): the first kernel a product launches
// records `start` as it begins and the last records `stop` as it ends, from
// the kernels' own dispatch timestamps (no marker between the kernels).
struct KernelTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
const KernelTiming& kernel_timing();

#define HSPMM_LAUNCH(KERNEL, GRID, BLOCK, LDS, STREAM, FIRST, LAST, ...)                                  \
    do {                                                                                                \
        const ::hspmm::KernelTiming& _kt = ::hspmm::kernel_timing();                                    \
        if (_kt.start || _kt.stop)                                                                      \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, (FIRST) ? _kt.start : nullptr,     \
                                  (LAST) ? _kt.stop : nullptr, 0, __VA_ARGS__);                         \
        else                                                                                            \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, __VA_ARGS__);                          \
    } while (0)

// LDS stage of the group kernels: rows of 256 bytes of the dense operand
// (one column panel); the default and the largest number of staged rows a
// group may hold
constexpr int kGroupRowBytes = 256;
constexpr int kGroupStageRows = 300;
constexpr int kGroupMaxBlocks = 4;
constexpr int kGroupStageRowsMax = 620;

}  // namespace hspmm
