// In-memory form of a hybrid plan.
#pragma once

#include "common.h"
#include "cost_model.h"

namespace hspmm {

// One sparse matrix (A, or A^T for the backward) in hybrid form.
struct SubPlan {
    int ct = HSPMM_F32;           // dtype of the stored part values and of the dense operand
    int64_t m = 0, k = 0, nnz = 0;
    int br = 16;                  // tile height B_r
    int kc = 4;                   // tiles per MFMA step (K depth); tiles of a row block padded to it
    int64_t nrb = 0;
    bool scaled = false;          // FP16/BF16 values stored as value / scale[row block]

    std::vector<int32_t> h_rb_nnz, h_rb_nblk;
    std::vector<uint8_t> h_cls;   // 1 = BCSR-part
    double pred_csr = 0.0, pred_bcsr = 0.0;       // predicted time of each part of the chosen split
    double pred_all_csr = 0.0, pred_all_bcsr = 0.0;  // ... of the whole matrix in one part (Eq. 1 inputs)
    int64_t r_boundary = -1;

    // CSR-part (Alg. 1 step 1): rows ascending, entries copied
    int64_t rows_csr = 0, nnz_csr = 0;
    DevBuf csr_rows, csr_ptr, csr_col, csr_val, csr_src;
    // its work list: virtual rows of at most `seg` entries; vr_out >= 0 is a
    // row of C, vr_out < 0 is partial slot (-vr_out - 1) of a split row
    int64_t n_vrows = 0, n_long = 0, n_partials = 0;
    int32_t seg = 0;
    DevBuf vr_start, vr_end, vr_out, vr_row;
    DevBuf long_row, long_first, long_cnt;

    // BCSR-part (Alg. 1 step 2): B_r x 1 tiles, values packed in MFMA lane order
    int64_t rb_bcsr = 0, nblk = 0, nblk_pad = 0, nnz_bcsr = 0;
    DevBuf bcsr_rb, blk_ptr, blk_cnt, blk_col, blk_val, blk_src;
    // SDDMM destinations (A only), per chunk of 16 consecutive tiles of a
    // BCSR row block, the SDDMM's unit of work.  For row R of the block at
    // position p (R in the order in which the MFMA output holds rows:
    // lane group p / 4, register p % 4): bit t of chunk_mask[c][p] is set
    // when tile t of the chunk holds an entry of row R, and chunk_base[c][p]
    // is the canonical index of row R's first entry at or after the chunk
    DevBuf chunk_ptr;     // int32 [rb_bcsr + 1]: first chunk of each BCSR row block
    DevBuf chunk_base;    // int32 [nchunks][16]
    DevBuf chunk_mask;    // uint16 [nchunks][16]
    int64_t nchunks = 0;
    std::vector<int32_t> h_bcsr_rb, h_blk_ptr, h_blk_cnt;
    int64_t max_rb_tiles = 0;  // most tiles in one row block of the BCSR-part
    int32_t max_long_cnt = 0;  // most segments of one split CSR row

    DevBuf scale;                 // double [nrb] (scaled sub-plans only)

    // fused backward (A^T only): per stored tile, the canonical index of the
    // first entry of A it holds and which of its 16 rows hold one (a tile of
    // A^T is 16 consecutive columns of one row of A, so its entries are
    // consecutive in A's canonical order)
    DevBuf tile_base;             // int32 [nblk_pad]
    DevBuf tile_mask;             // uint16 [nblk_pad]

    // groups of row blocks that share columns (group.h): the group kernels
    // visit the BCSR row blocks in the order kslot_* (groups contiguous,
    // group g = kernel slots [grp_ptr[g], grp_ptr[g + 1])), stage the columns
    // grp_ucol[grp_uptr[g] ..] in LDS and read each tile's B row from the
    // stage row blk_bsrc[tile] >= 0 or from column -(blk_bsrc + 1)
    bool grouped = false;
    int64_t ngroups = 0, grp_max_u = 0, grp_staged = 0, grp_union = 0;
    DevBuf kslot_rb, kslot_ptr, kslot_cnt, kslot_chunk;
    DevBuf grp_ptr, grp_uptr, grp_ucol, blk_bsrc;
    std::vector<int32_t> h_order;  // kernel slot -> canonical slot (grouped only)

    // workgroup partition of the fused launch (0 = one workgroup per work
    // unit); set by calibration
    int32_t part_csr = 0, part_bcsr = 0;

    int64_t bytes() const;
};

struct Plan {
    int compute = HSPMM_F32;
    int64_t m = 0, k = 0, nnz_in = 0, nnz = 0;
    int br = 16;
    bool canonical = true;
    hspmm_plan_opts opts{};
    Allocator al;
    MachineModel mm;

    // canonicalisation (non-canonical input only)
    DevBuf perm;          // int32 [nnz_in]: sorted position -> input entry
    DevBuf seg;           // int32 [nnz + 1]: canonical entry -> first sorted position
    DevBuf canon_of_orig; // int32 [nnz_in]: input entry -> canonical entry
    DevBuf row_of;        // int32 [nnz]: row of each canonical entry
    DevBuf canon_rp;      // int32 [m + 1]: canonical row pointer of A

    SubPlan A, T;
    bool has_T = false;

    double meas_csr = 0.0, meas_bcsr = 0.0;  // measured whole-matrix forward time of each part (s)

    DevBuf ws;            // run/backward scratch
    DevBuf ws2;           // scratch of the SDDMM when it runs beside dB
    // scratch buffers replaced by larger ones: work already queued may still
    // read them, so they are kept until the plan is destroyed (growth is
    // geometric and rare: it needs an n beyond every earlier one)
    std::vector<DevBuf> retired;
    double plan_ms = 0.0;

    // side stream of the backward: dA = SDDMM runs on it concurrently with
    // dB = A^T dC, forked from and joined back to the caller's stream by
    // events (default stream priority)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    ~Plan();
};

// vals/row_of helpers shared by the plan build and update_values
int pack_values(Plan& p, const void* vals, int vals_dtype, hipStream_t s);

// geometry of a forward launch (filled instead of launching when requested)
struct LaunchQuery {
    uint32_t g_csr = 0, g_bcsr = 0;  // default workgroups of each part
    int wg_per_cu = 0;               // resident workgroups per CU for the kernel
};

// A caller-provided scratch buffer for the partial rows of split CSR rows
// (used instead of the plan's own, which may grow): device pointer and
// capacity in bytes; a launch needing more fails with HSPMM_ERR_OOM.
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// forward product of one sub-plan: C = X * B
int launch_forward(Plan& p, SubPlan& X, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc,
                   hipStream_t s, LaunchQuery* q = nullptr, const Workspace* ext = nullptr);
// bytes of split-row scratch a forward product of X at width n needs
size_t forward_scratch_bytes(const SubPlan& X, int64_t n);
// SDDMM on A's pattern: dA_canon[c] (or dA_in[e] via canon_of_orig)
int launch_sddmm(Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc, void* dA,
                 hipStream_t s, DevBuf* ws);
int ensure_ws(Plan& p, size_t bytes);
// grow `b` to at least `bytes` without waiting for the device: the old
// buffer goes to p.retired
int grow_buf(Plan& p, DevBuf& b, size_t bytes);

// Both gradients from one pass over A^T's BCSR-part (FP32 / FP64, A^T all
// BCSR, n within one column panel, 16-byte rows): bwd_fusable says whether
// the call qualifies, launch_backward_fused computes dB and dA (input order)
bool bwd_fusable(const Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc,
                 const void* dB, int64_t lddb);
int launch_backward_fused(Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc, void* dB,
                          int64_t lddb, void* dA, hipStream_t s);
// the fused kernel alone: dA in canonical order; `last` = no kernel follows
int launch_bwd_fused_kernel(Plan& p, int64_t n, const void* B, int64_t ldb, const void* dC, int64_t lddc,
                            void* dB, int64_t lddb, void* dA_canon, hipStream_t s, bool last);

int calibrate(Plan& p, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc, int reps,
              hspmm_calib_info* info, hipStream_t s);

int build_plan(Plan& p, const int32_t* row_ptr, const int32_t* col_idx, const void* vals, int vals_dtype,
               hipStream_t s);

}  // namespace hspmm

// the opaque handle of the C ABI
struct hspmm_plan {
    hspmm::Plan p;
};
