// Host cost model: which part each B_r-row block goes to, the contiguous
// boundary of Eq. 1, and the quadratic performance model of Eq. 2-3.
#pragma once

#include <cstdint>
#include <vector>

namespace hspmm {

// Machine constants of one MI355X used by the byte/time model.  The
// bandwidths are effective figures (achievable HBM streaming, and the rate
// at which gathered rows of B arrive through L2/MALL), not peaks.
struct MachineModel {
    double bw_stream = 5.0e12;   // B/s for streamed A-part arrays
    double bw_gather = 12.0e12;  // B/s for gathered B rows (cache hits dominate)
    double t_entry_csr = 0.0;    // extra s per CSR entry per wave (issue cost)
    double t_blk_bcsr = 0.0;     // extra s per tile
    int cus = 256;
};

struct RowBlockCost {
    double t_csr;   // predicted seconds if the row block runs in the CSR-part
    double t_bcsr;  // ... in the BCSR-part
};

// Predicted time of one row block with `nnz` entries spread over `nblk`
// non-empty tiles, for dense width n, value bytes sv, dense bytes sb, and
// the MFMA K depth kc (tiles are padded to a multiple of kc).
RowBlockCost rowblock_cost(const MachineModel& mm, int64_t nnz, int64_t nblk, int64_t n, int sv, int sb,
                           int br, int kc);

// AUTO split: class[q] = 1 (BCSR) iff the BCSR-part is predicted faster.
void choose_auto(const MachineModel& mm, const std::vector<int32_t>& rb_nnz,
                 const std::vector<int32_t>& rb_nblk, int64_t n, int sv, int sb, int br, int kc,
                 std::vector<uint8_t>& cls, double& t_csr_total, double& t_bcsr_total);

// Eq. 1 read as balancing the two parts' predicted times:
// r / (TP_c t_c) = (R - r) / (TP_b t_b)  =>  r = R TP_c t_c / (TP_c t_c + TP_b t_b),
// rounded to the nearest multiple of br and clamped to [0, R].
int64_t eq1_boundary(int64_t r_total, double tp_csr, double t_csr, double tp_bcsr, double t_bcsr,
                     int br);

// Eq. 2: least-squares coefficients a0..a4 of perf = a0 + a1 x + a2 y + a3 x^2 + a4 y^2.
// Terms whose mask bit (1 << i) is clear are left out of the fit (a[i] = 0),
// e.g. the x terms when one part is empty.
bool fit_quadratic(const std::vector<double>& x, const std::vector<double>& y,
                   const std::vector<double>& perf, double a[5], unsigned mask = 0x1f);
// Eq. 3: argmax over integers x in [xlo, xhi], y in [ylo, yhi] with
// 1 <= x + y <= T (first in lexicographic order on ties).
void argmax_quadratic(const double a[5], int T, int* x, int* y, int xlo = 0, int xhi = -1, int ylo = 0,
                      int yhi = -1);

}  // namespace hspmm
