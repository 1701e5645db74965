// Warm-up calibration of the workgroup partition of the fused forward
// launch: the GPU analogue of the thread split (t_neon, t_sme) chosen by
// the quadratic performance model of Sec. 3.5 (Eq. 2 fitted by least
// squares over a candidate set, Eq. 3 its argmax over x + y <= T).
#include <algorithm>
#include <cmath>

#include "plan.h"

namespace hspmm {

namespace {

int time_forward(Plan& p, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc, int reps, hipStream_t s,
                 double* gflops) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int rc = HSPMM_OK;
    for (int i = 0; i < 2 && rc == HSPMM_OK; ++i) rc = launch_forward(p, p.A, n, B, ldb, C, ldc, s);
    if (rc == HSPMM_OK) {
        (void)hipEventRecord(e0, s);
        for (int i = 0; i < reps && rc == HSPMM_OK; ++i) rc = launch_forward(p, p.A, n, B, ldb, C, ldc, s);
        (void)hipEventRecord(e1, s);
    }
    float ms = 0.f;
    if (rc == HSPMM_OK) {
        hipError_t e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) rc = hip_fail(e, "calibration timing", __FILE__, __LINE__);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    const double t = (double)ms * 1e-3 / reps;
    *gflops = t > 0 ? 2.0 * (double)p.A.nnz * (double)n / t * 1e-9 : 0.0;
    return HSPMM_OK;
}

}  // namespace

int calibrate(Plan& p, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc, int reps,
              hspmm_calib_info* info, hipStream_t s) {
    SubPlan& X = p.A;
    hspmm_calib_info out{};
    out.struct_size = sizeof(hspmm_calib_info);
    const int32_t save_c = X.part_csr, save_b = X.part_bcsr;
    X.part_csr = X.part_bcsr = 0;
    LaunchQuery q;
    HSPMM_TRY(launch_forward(p, X, n, B, ldb, C, ldc, s, &q));
    if (q.g_csr + q.g_bcsr == 0) {  // nothing to run
        *info = out;
        return HSPMM_OK;
    }
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // T: resident workgroups of the whole GPU, in units of 8 (one per XCD)
    const int T = std::max(2, cus * std::max(1, q.wg_per_cu) / 8);
    const bool has_c = q.g_csr > 0, has_b = q.g_bcsr > 0;
    const int xmax = has_c ? std::min<int>(T, (int)ceil_div(q.g_csr, 8)) : 0;
    const int ymax = has_b ? std::min<int>(T, (int)ceil_div(q.g_bcsr, 8)) : 0;
    out.T = T;
    out.x_max = xmax;
    out.y_max = ymax;

    // candidate set: fractions of each present part's default size, pairs
    // within the budget x + y <= T (5 x 5 at most, below HSPMM_CALIB_MAX)
    const double fr[] = {0.125, 0.25, 0.5, 0.75, 1.0};
    std::vector<std::pair<int, int>> cand;
    auto clampx = [&](double f) { return std::max(1, (int)std::lround(f * xmax)); };
    auto clampy = [&](double f) { return std::max(1, (int)std::lround(f * ymax)); };
    if (has_c && has_b) {
        for (double fx : fr)
            for (double fy : fr)
                if (clampx(fx) + clampy(fy) <= T) cand.emplace_back(clampx(fx), clampy(fy));
        if (cand.empty()) cand.emplace_back(1, 1);
    } else if (has_c) {
        for (double fx : fr) cand.emplace_back(clampx(fx), 0);
    } else {
        for (double fy : fr) cand.emplace_back(0, clampy(fy));
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    if ((int)cand.size() > HSPMM_CALIB_MAX) cand.resize(HSPMM_CALIB_MAX);

    std::vector<double> xs, ys, perf;
    int rc = time_forward(p, n, B, ldb, C, ldc, reps, s, &out.default_gflops);
    for (size_t i = 0; i < cand.size() && rc == HSPMM_OK; ++i) {
        X.part_csr = cand[i].first * 8;
        X.part_bcsr = cand[i].second * 8;
        double g = 0;
        rc = time_forward(p, n, B, ldb, C, ldc, reps, s, &g);
        out.cand_x[i] = cand[i].first;
        out.cand_y[i] = cand[i].second;
        out.cand_gflops[i] = g;
        xs.push_back(cand[i].first);
        ys.push_back(cand[i].second);
        perf.push_back(g);
    }
    out.n_candidates = (int32_t)xs.size();
    if (rc) {
        X.part_csr = save_c;
        X.part_bcsr = save_b;
        return rc;
    }
    // Eq. 2 (terms of an absent part dropped; the squared term is dropped
    // too when a part was sampled at fewer than three distinct sizes)
    auto distinct = [](const std::vector<double>& v) {
        std::vector<double> u(v);
        std::sort(u.begin(), u.end());
        return (int)(std::unique(u.begin(), u.end()) - u.begin());
    };
    unsigned mask = 1u;
    if (has_c && distinct(xs) >= 2) mask |= 1u << 1;
    if (has_b && distinct(ys) >= 2) mask |= 1u << 2;
    if (has_c && distinct(xs) >= 3) mask |= 1u << 3;
    if (has_b && distinct(ys) >= 3) mask |= 1u << 4;
    if (!fit_quadratic(xs, ys, perf, out.coef, mask)) {
        for (double& c : out.coef) c = 0.0;
    }
    // Eq. 3 over every integer partition of the present parts
    argmax_quadratic(out.coef, T, &out.best_x, &out.best_y, has_c ? 1 : 0, xmax, has_b ? 1 : 0, ymax);
    X.part_csr = out.best_x * 8;
    X.part_bcsr = out.best_y * 8;
    HSPMM_TRY(time_forward(p, n, B, ldb, C, ldc, reps, s, &out.best_gflops));
    out.applied = out.best_gflops >= out.default_gflops ? 1 : 0;
    if (!out.applied) X.part_csr = X.part_bcsr = 0;
    *info = out;
    return HSPMM_OK;
}

}  // namespace hspmm
