// hybrid_spmm_run_noalloc: the forward product with no device allocation.
//
// The only scratch a forward product needs is the partial rows of split CSR
// rows (rows cut into segments that separate waves sum; a second kernel adds
// the segments in a fixed order).  hybrid_spmm_run keeps that buffer in the
// plan and grows it when a wider n comes; this entry point uses instead a
// file-scope device array of fixed size, `scratch`, so it never allocates.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is ever
// handed to kernels.
#include <mutex>

#include "plan.h"

namespace hspmm {

namespace {

constexpr size_t kScratchBytes = HSPMM_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of the current device's copy of `scratch`
int scratch_ptr(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HSPMM_ERR_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(HSPMM_ERR_HIP, "hipGetSymbolAddress returned NULL for the static scratch");
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return HSPMM_OK;
}

}  // namespace

}  // namespace hspmm

using namespace hspmm;

extern "C" int hybrid_spmm_run_noalloc(hspmm_plan_t h, int64_t n, const void* B, int64_t ldb, void* C,
                                       int64_t ldc, void* stream) {
    clear_error();
    if (!h) return fail(HSPMM_ERR_ARG, "plan is NULL");
    Plan& p = h->p;
    if (n < 0) return fail(HSPMM_ERR_ARG, "n < 0");
    if (n == 0 || p.m == 0) return HSPMM_OK;
    if (!C) return fail(HSPMM_ERR_ARG, "C is NULL");
    if (p.k > 0 && !B) return fail(HSPMM_ERR_ARG, "B is NULL");
    if (ldc < n || (p.k > 0 && ldb < n)) return fail(HSPMM_ERR_ARG, "leading dimension smaller than n");
    const size_t need = forward_scratch_bytes(p.A, n);
    if (need > kScratchBytes)
        return fail(HSPMM_ERR_OOM, "hybrid_spmm_run_noalloc: split rows need " + std::to_string(need) +
                                       " bytes of scratch at n = " + std::to_string(n) + ", above the static " +
                                       std::to_string(kScratchBytes));
    Workspace ws;
    if (need > 0) {
        HSPMM_TRY(scratch_ptr(&ws.ptr));
        ws.bytes = kScratchBytes;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    return launch_forward(p, p.A, n, B, ldb, C, ldc, s, nullptr, &ws);
}
