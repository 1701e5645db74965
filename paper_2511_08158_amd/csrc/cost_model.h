// Host cost model: which part each B_r-row block goes to, the contiguous
// boundary of Eq. 1, and the quadratic performance model of Eq. 2-3.
#pragma once

#include <cstdint>
#include <vector>

namespace hspmm {

// Machine constants of one MI355X used by the time model, one set per
// precision of the dense operand (its element size s_b).  The rates are
// effective figures of this library's two kernels, fitted by relative least
// squares (with a per-launch constant that every plan pays alike) to the
// forward times of the CSR-only and BCSR-only plans of the 64-matrix
// structure sweep at its full sizes, n = 16..256, in that precision:
//   CSR-part  = nnz * (t_entry + n s_b / bw_csr)       (one gathered B row
//               segment per entry, through L2/MALL);
//   BCSR-part = padded tiles * max(t_blk, n s_b / bw_bcsr)   (a tile costs
//               its MFMA step, value and index loads until its gathered
//               B row segment takes longer; FP16/BF16 row blocks are padded
//               to 32 tiles, FP32/FP64 to 4).
struct PartRates {
    double bw_csr, t_entry, bw_bcsr, t_blk;
};
struct MachineModel {
    PartRates f64{16.0e12, 0.0, 6.5e12, 34.6e-12};
    PartRates f32{18.7e12, 1.0e-12, 6.5e12, 32.2e-12};
    PartRates f16{13.4e12, 1.9e-12, 6.5e12, 17.3e-12};  // FP16 and BF16
    // extra time of a plan with both parts over a one-part plan (measured:
    // one ragged CSR row block beside a BCSR-part added 4.5 us)
    double t_mixed = 4.0e-6;
    int cus = 256;
    const PartRates& rates(int sb) const { return sb >= 8 ? f64 : (sb == 4 ? f32 : f16); }
};

struct RowBlockCost {
    double t_csr;   // predicted seconds if the row block runs in the CSR-part
    double t_bcsr;  // ... in the BCSR-part
};

// Predicted time of one row block with `nnz` entries spread over `nblk`
// non-empty tiles, for dense width n, value bytes sv, dense bytes sb, and
// the MFMA K depth kc (tiles are padded to a multiple of kc).  Each CSR
// entry gathers one B row segment; each BCSR tile gathers one and serves
// all br rows with it.
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
