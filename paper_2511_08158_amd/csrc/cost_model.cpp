// Host cost model (pure host arithmetic, no device calls).
#include "cost_model.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace hspmm {

RowBlockCost rowblock_cost(const MachineModel& mm, int64_t nnz, int64_t nblk, int64_t n, int sv, int sb,
                           int br, int kc) {
    (void)sv;
    (void)br;
    const PartRates& r = mm.rates(sb);
    RowBlockCost c;
    c.t_csr = (double)nnz * (r.t_entry + (double)n * sb / r.bw_csr);
    const int64_t padded = nblk == 0 ? 0 : ((nblk + kc - 1) / kc) * kc;
    c.t_bcsr = (double)padded * std::max(r.t_blk, (double)n * sb / r.bw_bcsr);
    return c;
}

void choose_auto(const MachineModel& mm, const std::vector<int32_t>& rb_nnz,
                 const std::vector<int32_t>& rb_nblk, int64_t n, int sv, int sb, int br, int kc,
                 std::vector<uint8_t>& cls, double& t_csr_total, double& t_bcsr_total) {
    const size_t nrb = rb_nnz.size();
    cls.assign(nrb, 0);
    t_csr_total = 0.0;
    t_bcsr_total = 0.0;
    double all_csr = 0.0, all_bcsr = 0.0;
    for (size_t q = 0; q < nrb; ++q) {
        if (rb_nnz[q] == 0) continue;
        RowBlockCost c = rowblock_cost(mm, rb_nnz[q], rb_nblk[q], n, sv, sb, br, kc);
        all_csr += c.t_csr;
        all_bcsr += c.t_bcsr;
        if (c.t_bcsr < c.t_csr) {
            cls[q] = 1;
            t_bcsr_total += c.t_bcsr;
        } else {
            t_csr_total += c.t_csr;
        }
    }
    // a plan with both parts pays for them (the fused launch's register
    // budget, a small CSR-part's split rows and their reduction launch):
    // keep the split only if it beats the better one-part plan by more
    // than mm.t_mixed
    if (t_csr_total > 0.0 && t_bcsr_total > 0.0 && t_csr_total + t_bcsr_total + mm.t_mixed >= std::min(all_csr, all_bcsr)) {
        const uint8_t to = all_bcsr <= all_csr ? 1 : 0;
        for (size_t q = 0; q < nrb; ++q)
            if (rb_nnz[q] != 0) cls[q] = to;
        t_csr_total = to ? 0.0 : all_csr;
        t_bcsr_total = to ? all_bcsr : 0.0;
    }
}

int64_t eq1_boundary(int64_t r_total, double tp_csr, double t_csr, double tp_bcsr, double t_bcsr,
                     int br) {
    const double wc = tp_csr * t_csr, wb = tp_bcsr * t_bcsr;
    if (wb <= 0.0) return r_total;
    if (wc <= 0.0) return 0;
    const double r = (double)r_total * wc / (wc + wb);
    int64_t rb = (int64_t)std::floor(r / br + 0.5) * br;
    if (rb < 0) rb = 0;
    if (rb > r_total) rb = r_total;
    return rb;
}

// Normal equations solved by Gaussian elimination with partial pivoting on
// the system of the active terms, (A^T A) a = A^T perf.
bool fit_quadratic(const std::vector<double>& x, const std::vector<double>& y,
                   const std::vector<double>& perf, double a[5], unsigned mask) {
    const size_t n = x.size();
    int idx[5], k = 0;
    for (int i = 0; i < 5; ++i)
        if (mask & (1u << i)) idx[k++] = i;
    for (int i = 0; i < 5; ++i) a[i] = 0.0;
    if (k == 0 || n < (size_t)k || y.size() != n || perf.size() != n) return false;
    double M[5][6] = {};
    for (size_t s = 0; s < n; ++s) {
        const double full[5] = {1.0, x[s], y[s], x[s] * x[s], y[s] * y[s]};
        for (int i = 0; i < k; ++i) {
            for (int j = 0; j < k; ++j) M[i][j] += full[idx[i]] * full[idx[j]];
            M[i][k] += full[idx[i]] * perf[s];
        }
    }
    for (int c = 0; c < k; ++c) {
        int p = c;
        for (int r = c + 1; r < k; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[p][c])) p = r;
        if (std::fabs(M[p][c]) < 1e-300) return false;
        if (p != c)
            for (int j = 0; j <= k; ++j) std::swap(M[p][j], M[c][j]);
        for (int r = 0; r < k; ++r) {
            if (r == c) continue;
            const double f = M[r][c] / M[c][c];
            for (int j = c; j <= k; ++j) M[r][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < k; ++i) a[idx[i]] = M[i][k] / M[i][i];
    return true;
}

void argmax_quadratic(const double a[5], int T, int* bx, int* by, int xlo, int xhi, int ylo, int yhi) {
    if (xhi < 0) xhi = T;
    if (yhi < 0) yhi = T;
    double best = -std::numeric_limits<double>::infinity();
    *bx = xlo;
    *by = ylo;
    for (int x = xlo; x <= xhi; ++x)
        for (int y = ylo; y <= yhi && x + y <= T; ++y) {
            if (x + y < 1) continue;
            const double v = a[0] + a[1] * x + a[2] * y + a[3] * x * x + a[4] * y * y;
            if (v > best) {
                best = v;
                *bx = x;
                *by = y;
            }
        }
}

}  // namespace hspmm
