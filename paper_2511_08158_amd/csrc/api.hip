// C ABI of the hspmm library (include/hspmm.h).
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <new>

#include "plan.h"

namespace hspmm {

namespace {
thread_local std::string g_last_error;
thread_local KernelTiming g_timing;
}

const KernelTiming& kernel_timing() { return g_timing; }

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
    std::string m = std::string("HIP error ") + hipGetErrorString(e) + " in " + what + " (" + file + ":" +
                    std::to_string(line) + ")";
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(HSPMM_ERR_OOM, m);
    return fail(HSPMM_ERR_HIP, m);
}

void DevBuf::release() {
    if (ptr) {
        if (owner && owner->keep) {
            owner->kept.push_back({ptr, bytes});
            owner->kept_bytes += bytes;
        } else {
            (void)hipFree(ptr);
        }
        if (owner) owner->in_use -= bytes;
    }
    ptr = nullptr;
    bytes = 0;
    owner = nullptr;
}

void Allocator::drop_kept() {
    for (const Kept& k : kept) (void)hipFree(k.ptr);
    kept.clear();
    kept_bytes = 0;
}

int sync_for_release(const Allocator& a, hipStream_t s) {
    if (!a.keep) HIP_TRY(hipStreamSynchronize(s));
    return HSPMM_OK;
}

int Allocator::alloc(DevBuf& b, size_t nbytes) {
    b.release();
    if (nbytes == 0) nbytes = 4;
    if (keep) {
        // the smallest kept buffer that holds nbytes and is at most twice
        // that (plus a page)
        size_t best = kept.size();
        for (size_t i = 0; i < kept.size(); ++i)
            if (kept[i].bytes >= nbytes && kept[i].bytes <= 2 * nbytes + 4096 &&
                (best == kept.size() || kept[i].bytes < kept[best].bytes))
                best = i;
        if (best < kept.size()) {
            b.ptr = kept[best].ptr;
            b.bytes = kept[best].bytes;
            b.owner = this;
            kept_bytes -= b.bytes;
            kept.erase(kept.begin() + (std::ptrdiff_t)best);
            in_use += b.bytes;
            peak = std::max(peak, in_use);
            return HSPMM_OK;
        }
        if (limit && in_use + kept_bytes + nbytes > limit) drop_kept();
    }
    if (limit && in_use + nbytes > limit)
        return fail(HSPMM_ERR_OOM, "plan exceeds max_workspace_bytes (" + std::to_string(limit) + ")");
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HSPMM_ERR_OOM, std::string("hipMalloc of ") + std::to_string(nbytes) +
                                       " bytes failed: " + hipGetErrorString(e));
    }
    b.ptr = p;
    b.bytes = nbytes;
    b.owner = this;
    in_use += nbytes;
    peak = std::max(peak, in_use);
    return HSPMM_OK;
}

int xcd_remap_mode() {
    static const int mode = [] {
        const char* e = getenv("HSPMM_XCD_REMAP");
        return (e && e[0] == '0') ? 0 : 1;
    }();
    return mode;
}

int bcsr_persistent() {
    static const int mode = [] {
        const char* e = getenv("HSPMM_BCSR_PERSIST");
        return (e && e[0] == '1') ? 1 : 0;
    }();
    return mode;
}

int bwd_concurrent() {
    // read on every backward call, so a process can switch it between calls
    const char* e = getenv("HSPMM_BWD_CONCURRENT");
    return (e && e[0] == '1') ? 1 : 0;
}

int bwd_fused_mode() {
    const char* e = getenv("HSPMM_BWD_FUSED");
    return (e && e[0] == '0') ? 0 : 1;
}

int hybrid_launch_mode() {
    const char* e = getenv("HSPMM_HYBRID_LAUNCH");
    return (e && e[0] == '2') ? 2 : 1;
}

Plan::~Plan() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
}

int grow_buf(Plan& p, DevBuf& b, size_t bytes) {
    if (bytes <= b.bytes) return HSPMM_OK;
    if (b.ptr) p.retired.push_back(std::move(b));
    return p.al.alloc(b, bytes);
}

int ensure_ws(Plan& p, size_t bytes) { return grow_buf(p, p.ws, bytes); }

}  // namespace hspmm

using namespace hspmm;

namespace {

int check_opts(const hspmm_plan_opts* o, hspmm_plan_opts* out) {
    hspmm_plan_opts d{};
    d.struct_size = sizeof(hspmm_plan_opts);
    d.compute = HSPMM_F32;
    d.split = HSPMM_SPLIT_AUTO;
    d.block_rows = 16;
    d.r_boundary = -1;
    d.n_hint = 128;
    d.want_backward = 0;
    d.max_workspace_bytes = 0;
    if (o) {
        if (o->struct_size != sizeof(hspmm_plan_opts))
            return fail(HSPMM_ERR_ARG, "hspmm_plan_opts.struct_size mismatch");
        d = *o;
        if (d.block_rows == 0) d.block_rows = 16;
        if (d.n_hint <= 0) d.n_hint = 128;
    }
    if (!dtype_valid(d.compute)) return fail(HSPMM_ERR_DTYPE, "unsupported compute dtype");
    if (d.split < HSPMM_SPLIT_AUTO || d.split > HSPMM_SPLIT_BOUNDARY) return fail(HSPMM_ERR_ARG, "bad split mode");
    if (d.block_rows != 16) return fail(HSPMM_ERR_ARG, "block_rows must be 16 (the MFMA tile height)");
    *out = d;
    return HSPMM_OK;
}

}  // namespace

extern "C" {

int hybrid_spmm_plan(hspmm_plan_t* out, int64_t m, int64_t k, int64_t nnz, const int32_t* row_ptr,
                     const int32_t* col_idx, const void* vals, int32_t vals_dtype, const hspmm_plan_opts* opts,
                     void* stream) {
    clear_error();
    if (!out) return fail(HSPMM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (m < 0 || k < 0 || nnz < 0) return fail(HSPMM_ERR_ARG, "negative dimension");
    if (m >= (int64_t(1) << 31) - 1 || k >= (int64_t(1) << 31) - 1 || nnz >= (int64_t(1) << 31) - 1)
        return fail(HSPMM_ERR_OVERFLOW, "m, k and nnz must be below 2^31 - 1");
    if (!row_ptr) return fail(HSPMM_ERR_ARG, "row_ptr is NULL");
    if (nnz > 0 && (!col_idx || !vals)) return fail(HSPMM_ERR_ARG, "col_idx or vals is NULL");
    if (!dtype_valid(vals_dtype)) return fail(HSPMM_ERR_DTYPE, "unsupported vals dtype");
    if (nnz > 0 && k == 0) return fail(HSPMM_ERR_CSR, "entries in a matrix with no columns");
    hspmm_plan_opts o;
    int rc = check_opts(opts, &o);
    if (rc) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    hspmm_plan* h = new (std::nothrow) hspmm_plan();
    if (!h) return fail(HSPMM_ERR_OOM, "host allocation failed");
    Plan& p = h->p;
    p.opts = o;
    p.compute = o.compute;
    p.m = m;
    p.k = k;
    p.nnz_in = nnz;
    p.br = o.block_rows;
    p.al.limit = o.max_workspace_bytes;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = build_plan(p, row_ptr, col_idx, vals, vals_dtype, s);
    if (rc) {
        (void)hipStreamSynchronize(s);
        delete h;
        return rc;
    }
    p.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return HSPMM_OK;
}

int hybrid_spmm_run(hspmm_plan_t h, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc, void* stream) {
    clear_error();
    if (!h) return fail(HSPMM_ERR_ARG, "plan is NULL");
    Plan& p = h->p;
    if (n < 0) return fail(HSPMM_ERR_ARG, "n < 0");
    if (n == 0 || p.m == 0) return HSPMM_OK;
    if (!C) return fail(HSPMM_ERR_ARG, "C is NULL");
    if (p.k > 0 && !B) return fail(HSPMM_ERR_ARG, "B is NULL");
    if (ldc < n || (p.k > 0 && ldb < n)) return fail(HSPMM_ERR_ARG, "leading dimension smaller than n");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HSPMM_TRY(launch_forward(p, p.A, n, B, ldb, C, ldc, s));
    return HSPMM_OK;
}

int hybrid_spmm_backward(hspmm_plan_t h, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc,
                         void* dB, int64_t lddb, void* dA_vals, void* stream) {
    clear_error();
    if (!h) return fail(HSPMM_ERR_ARG, "plan is NULL");
    Plan& p = h->p;
    if (n < 0) return fail(HSPMM_ERR_ARG, "n < 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool do_dB = dB && n > 0 && p.k > 0;
    const bool do_dA = dA_vals && p.nnz_in > 0;
    if (dB) {
        if (!p.has_T) return fail(HSPMM_ERR_NO_BACKWARD, "plan was built without want_backward");
        if (do_dB) {
            if (lddb < n || (p.m > 0 && lddc < n)) return fail(HSPMM_ERR_ARG, "leading dimension smaller than n");
            if (p.m > 0 && !dC) return fail(HSPMM_ERR_ARG, "dC is NULL");
        }
    }
    if (do_dA) {
        if (n > 0 && (!B || !dC)) return fail(HSPMM_ERR_ARG, "B or dC is NULL");
        if (n > 0 && (ldb < n || lddc < n)) return fail(HSPMM_ERR_ARG, "leading dimension smaller than n");
    }
    if (do_dB && do_dA && bwd_fusable(p, n, B, ldb, dC, lddc, dB, lddb)) {
        HSPMM_TRY(launch_backward_fused(p, n, B, ldb, dC, lddc, dB, lddb, dA_vals, s));
        return HSPMM_OK;
    }
    if (do_dB && do_dA && bwd_concurrent()) {
        // the two gradients are independent: SDDMM on the side stream,
        // forked from and joined back into the caller's stream
        if (!p.side) {
            HIP_TRY(hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&p.ev_fork, hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&p.ev_join, hipEventDisableTiming));
        }
        HIP_TRY(hipEventRecord(p.ev_fork, s));
        HIP_TRY(hipStreamWaitEvent(p.side, p.ev_fork, 0));
        const int rc = launch_sddmm(p, n, B, ldb, dC, lddc, dA_vals, p.side, &p.ws2);
        HIP_TRY(hipEventRecord(p.ev_join, p.side));
        HSPMM_TRY(rc);
        const int rc2 = launch_forward(p, p.T, n, dC, lddc, dB, lddb, s);
        HIP_TRY(hipStreamWaitEvent(s, p.ev_join, 0));
        HSPMM_TRY(rc2);
        return HSPMM_OK;
    }
    if (do_dB) HSPMM_TRY(launch_forward(p, p.T, n, dC, lddc, dB, lddb, s));
    if (do_dA) HSPMM_TRY(launch_sddmm(p, n, B, ldb, dC, lddc, dA_vals, s, nullptr));
    return HSPMM_OK;
}

int hybrid_spmm_backward_fused(hspmm_plan_t h, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc,
                               const void* dB, int64_t lddb, int32_t* fused) {
    clear_error();
    if (!h || !fused) return fail(HSPMM_ERR_ARG, "NULL argument");
    static const unsigned char aligned_stand_in[16] __attribute__((aligned(16))) = {0};
    *fused = bwd_fusable(h->p, n, B, ldb, dC, lddc, dB ? dB : aligned_stand_in, lddb) ? 1 : 0;
    return HSPMM_OK;
}

int hybrid_spmm_update_values(hspmm_plan_t h, const void* vals, int32_t vals_dtype, void* stream) {
    clear_error();
    if (!h) return fail(HSPMM_ERR_ARG, "plan is NULL");
    if (!dtype_valid(vals_dtype)) return fail(HSPMM_ERR_DTYPE, "unsupported vals dtype");
    Plan& p = h->p;
    if (p.nnz_in > 0 && !vals) return fail(HSPMM_ERR_ARG, "vals is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HSPMM_TRY(pack_values(p, vals, vals_dtype, s));
    return HSPMM_OK;
}

int hybrid_spmm_plan_info(hspmm_plan_t h, hspmm_plan_info* info) {
    clear_error();
    if (!h || !info) return fail(HSPMM_ERR_ARG, "NULL argument");
    if (info->struct_size != sizeof(hspmm_plan_info)) return fail(HSPMM_ERR_ARG, "hspmm_plan_info.struct_size mismatch");
    const Plan& p = h->p;
    hspmm_plan_info i{};
    i.struct_size = sizeof(hspmm_plan_info);
    i.compute = p.compute;
    i.m = p.m;
    i.k = p.k;
    i.nnz_input = p.nnz_in;
    i.nnz = p.nnz;
    i.block_rows = p.br;
    i.canonical_input = p.canonical ? 1 : 0;
    i.rows_csr = p.A.rows_csr;
    i.nnz_csr = p.A.nnz_csr;
    i.long_rows = p.A.n_long;
    i.rb_bcsr = p.A.rb_bcsr;
    i.nblk = p.A.nblk;
    i.nblk_padded = p.A.nblk_pad;
    i.nnz_bcsr = p.A.nnz_bcsr;
    i.fill = p.A.nblk ? (double)p.A.nnz_bcsr / ((double)p.A.nblk * p.br) : 0.0;
    i.pred_us_csr = p.A.pred_csr * 1e6;
    i.pred_us_bcsr = p.A.pred_bcsr * 1e6;
    i.r_boundary = p.A.r_boundary;
    i.bytes_device = (int64_t)p.al.in_use;
    i.plan_ms = p.plan_ms;
    i.has_backward = p.has_T ? 1 : 0;
    i.t_rows_csr = p.T.rows_csr;
    i.t_rb_bcsr = p.T.rb_bcsr;
    i.t_nblk = p.T.nblk;
    i.pred_us_csr_all = p.A.pred_all_csr * 1e6;
    i.pred_us_bcsr_all = p.A.pred_all_bcsr * 1e6;
    i.ngroups = p.A.grouped ? p.A.ngroups : 0;
    i.grp_staged_tiles = p.A.grouped ? p.A.grp_staged : 0;
    i.grp_stage_rows = p.A.grouped ? p.A.grp_union : 0;
    i.meas_us_csr_all = p.meas_csr * 1e6;
    i.meas_us_bcsr_all = p.meas_bcsr * 1e6;
    *info = i;
    return HSPMM_OK;
}

int hybrid_spmm_export(hspmm_plan_t h, int32_t which, int32_t field, void* dst, int64_t capacity, int64_t* bytes) {
    clear_error();
    if (!h || !bytes) return fail(HSPMM_ERR_ARG, "NULL argument");
    Plan& p = h->p;
    if (which != 0 && which != 1) return fail(HSPMM_ERR_ARG, "which must be 0 (A) or 1 (A^T)");
    if (which == 1 && !p.has_T) return fail(HSPMM_ERR_NO_BACKWARD, "no transposed plan");
    SubPlan& X = which ? p.T : p.A;
    const bool half = X.ct == HSPMM_F16 || X.ct == HSPMM_BF16;
    const size_t ev = dtype_size(X.ct);
    std::vector<uint8_t> buf;
    auto put_i32 = [&](const std::vector<int32_t>& v) {
        buf.resize(v.size() * 4);
        if (!v.empty()) memcpy(buf.data(), v.data(), buf.size());
    };
    auto fetch = [&](const DevBuf& d, size_t nb, std::vector<uint8_t>& out) -> int {
        out.resize(nb);
        if (nb) HIP_TRY(hipMemcpy(out.data(), d.ptr, nb, hipMemcpyDeviceToHost));
        return HSPMM_OK;
    };
    switch (field) {
        case HSPMM_F_RB_CLASS: {
            std::vector<int32_t> v(X.h_cls.begin(), X.h_cls.end());
            put_i32(v);
            break;
        }
        case HSPMM_F_RB_NNZ: put_i32(X.h_rb_nnz); break;
        case HSPMM_F_RB_NBLK: put_i32(X.h_rb_nblk); break;
        case HSPMM_F_CSR_ROWS: HSPMM_TRY(fetch(X.csr_rows, X.rows_csr * 4, buf)); break;
        case HSPMM_F_CSR_PTR: HSPMM_TRY(fetch(X.csr_ptr, (X.rows_csr + 1) * 4, buf)); break;
        case HSPMM_F_CSR_COL: HSPMM_TRY(fetch(X.csr_col, X.nnz_csr * 4, buf)); break;
        case HSPMM_F_CSR_VAL: HSPMM_TRY(fetch(X.csr_val, X.nnz_csr * ev, buf)); break;
        case HSPMM_F_BCSR_RB: put_i32(X.h_bcsr_rb); break;
        case HSPMM_F_BLK_PTR: {
            std::vector<int32_t> v(1, 0);
            for (int32_t c : X.h_blk_cnt) v.push_back(v.back() + c);
            put_i32(v);
            break;
        }
        case HSPMM_F_BLK_COL:
        case HSPMM_F_BLK_VAL: {
            std::vector<uint8_t> raw;
            const bool val = field == HSPMM_F_BLK_VAL;
            HSPMM_TRY(fetch(val ? X.blk_val : X.blk_col, (size_t)X.nblk_pad * (val ? 16 * ev : 4), raw));
            const size_t per = val ? 16 * ev : 4;
            buf.resize((size_t)X.nblk * per);
            size_t o = 0;
            for (size_t sl = 0; sl < X.h_blk_cnt.size(); ++sl) {
                for (int32_t b = 0; b < X.h_blk_cnt[sl]; ++b) {
                    const int64_t blk = (int64_t)X.h_blk_ptr[sl] + b;
                    if (!val) {
                        memcpy(buf.data() + o, raw.data() + blk * 4, 4);
                        o += 4;
                    } else {
                        for (int i = 0; i < 16; ++i) {
                            const int64_t pi = half ? (blk >> 5) * 512 + ((blk & 31) >> 3) * 128 + i * 8 + (blk & 7)
                                                    : blk * 16 + i;
                            memcpy(buf.data() + o, raw.data() + pi * ev, ev);
                            o += ev;
                        }
                    }
                }
            }
            break;
        }
        case HSPMM_F_GRP_PTR:
        case HSPMM_F_GRP_RB:
        case HSPMM_F_GRP_UPTR:
        case HSPMM_F_GRP_UCOL: {
            std::vector<int32_t> v;
            if (X.grouped) {
                if (field == HSPMM_F_GRP_RB) {
                    for (int32_t o : X.h_order) v.push_back(X.h_bcsr_rb[o]);
                } else {
                    const DevBuf& d = field == HSPMM_F_GRP_PTR ? X.grp_ptr
                                      : field == HSPMM_F_GRP_UPTR ? X.grp_uptr : X.grp_ucol;
                    size_t cnt = field == HSPMM_F_GRP_UCOL ? (size_t)X.grp_union : (size_t)X.ngroups + 1;
                    v.resize(cnt);
                    if (cnt) HIP_TRY(hipMemcpy(v.data(), d.ptr, cnt * 4, hipMemcpyDeviceToHost));
                }
            }
            put_i32(v);
            break;
        }
        case HSPMM_F_BLK_BSRC: {
            std::vector<int32_t> v;
            if (X.grouped) {
                std::vector<uint8_t> raw;
                HSPMM_TRY(fetch(X.blk_bsrc, (size_t)X.nblk_pad * 4, raw));
                for (size_t sl = 0; sl < X.h_blk_cnt.size(); ++sl)
                    for (int32_t b = 0; b < X.h_blk_cnt[sl]; ++b) {
                        int32_t x;
                        memcpy(&x, raw.data() + ((size_t)X.h_blk_ptr[sl] + b) * 4, 4);
                        v.push_back(x);
                    }
            }
            put_i32(v);
            break;
        }
        case HSPMM_F_RB_SCALE: {
            if (X.scaled) {
                HSPMM_TRY(fetch(X.scale, X.nrb * 8, buf));
            } else {
                std::vector<double> one((size_t)X.nrb, 1.0);
                buf.resize(one.size() * 8);
                if (!one.empty()) memcpy(buf.data(), one.data(), buf.size());
            }
            break;
        }
        default: return fail(HSPMM_ERR_ARG, "unknown field");
    }
    *bytes = (int64_t)buf.size();
    if (dst && capacity >= (int64_t)buf.size() && !buf.empty()) memcpy(dst, buf.data(), buf.size());
    return HSPMM_OK;
}

int hybrid_spmm_calibrate(hspmm_plan_t h, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc,
                          int32_t reps, hspmm_calib_info* info, void* stream) {
    clear_error();
    if (!h || !info) return fail(HSPMM_ERR_ARG, "NULL argument");
    if (info->struct_size != sizeof(hspmm_calib_info))
        return fail(HSPMM_ERR_ARG, "hspmm_calib_info.struct_size mismatch");
    Plan& p = h->p;
    if (n <= 0 || reps < 1) return fail(HSPMM_ERR_ARG, "n and reps must be positive");
    if (!C || (p.k > 0 && !B)) return fail(HSPMM_ERR_ARG, "B or C is NULL");
    if (ldc < n || (p.k > 0 && ldb < n)) return fail(HSPMM_ERR_ARG, "leading dimension smaller than n");
    return calibrate(p, n, B, ldb, C, ldc, reps, info, static_cast<hipStream_t>(stream));
}

void hybrid_spmm_destroy(hspmm_plan_t h) {
    if (!h) return;
    // The products leave nothing on their streams for destroy to wait on: an
    // event recorded after every product delayed the next kernel on the
    // stream by about 4.5 us (block stencil, FP32, n = 128).  hipFree waits
    // for the whole device before it frees, so destroy waits for the device
    // here, where that wait happens in any case.
    (void)hipDeviceSynchronize();
    delete h;
}

const char* hybrid_spmm_last_error(void) { return hspmm::last_error_cstr(); }

int hybrid_spmm_set_timing_events(void* start, void* stop) {
    clear_error();
    g_timing.start = static_cast<hipEvent_t>(start);
    g_timing.stop = static_cast<hipEvent_t>(stop);
    return HSPMM_OK;
}

const char* hybrid_spmm_version(void) { return "hspmm 0.2.0 (gfx950)"; }

}  // extern "C"
