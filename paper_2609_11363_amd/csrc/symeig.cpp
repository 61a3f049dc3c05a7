// Eigenpairs of a small dense symmetric matrix on the host: the projected
// problem T = V^T E V of the Lanczos iteration for the eigen step of the
// spectral correction (Section 2.5). Cyclic Jacobi: each rotation
// annihilates one off-diagonal entry (p, q), with the tangent t of the
// rotation angle taken as the root of smaller magnitude of
// t^2 + 2 theta t - 1 = 0, theta = (a_qq - a_pp) / (2 a_pq), and the
// entries updated in Rutishauser's form (tau = s / (1 + c)), which keeps the
// rotation orthogonal to rounding. Quadratically convergent; the
// eigenvectors accumulate the rotations.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "asi.h"

extern "C" asi_status asi_dense_symeig(int32_t m, const double *T, double *theta, double *Y) {
    if (m < 1 || m > 4096 || !T || !theta || !Y) return ASI_E_ARG;
    const size_t mm = (size_t)m * m;
    std::vector<double> a(mm), v(mm, 0.0);
    for (int32_t i = 0; i < m; ++i) {
        for (int32_t j = 0; j < m; ++j) {
            const double x = T[(size_t)i * m + j], y = T[(size_t)j * m + i];
            if (!std::isfinite(x)) return ASI_E_NONFINITE;
            a[(size_t)i * m + j] = 0.5 * (x + y);
        }
        v[(size_t)i * m + i] = 1.0;
    }
    auto A = [&](int32_t i, int32_t j) -> double & { return a[(size_t)i * m + j]; };
    auto Vr = [&](int32_t i, int32_t j) -> double & { return v[(size_t)i * m + j]; };
    bool converged = false;
    for (int sweep = 0; sweep < 100 && !converged; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            diag += A(i, i) * A(i, i);
            for (int32_t j = i + 1; j < m; ++j) off += A(i, j) * A(i, j);
        }
        if (std::sqrt(2.0 * off) <= 1e-15 * std::sqrt(diag + 2.0 * off)) {
            converged = true;
            break;
        }
        bool rotated = false;
        for (int32_t p = 0; p < m - 1; ++p) {
            for (int32_t q = p + 1; q < m; ++q) {
                const double apq = A(p, q);
                if (apq == 0.0) continue;
                const double th = (A(q, q) - A(p, p)) / (2.0 * apq);
                double t;
                if (std::fabs(th) > 1e150)
                    t = 0.5 / th;  // theta^2 would overflow; t ~ 1 / (2 theta)
                else
                    t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c, tau = s / (1.0 + c);
                if (t == 0.0) continue;
                rotated = true;
                A(p, p) -= t * apq;
                A(q, q) += t * apq;
                A(p, q) = A(q, p) = 0.0;
                for (int32_t r = 0; r < m; ++r) {
                    if (r == p || r == q) continue;
                    const double g = A(r, p), h = A(r, q);
                    A(r, p) = A(p, r) = g - s * (h + g * tau);
                    A(r, q) = A(q, r) = h + s * (g - h * tau);
                }
                for (int32_t r = 0; r < m; ++r) {
                    const double g = Vr(r, p), h = Vr(r, q);
                    Vr(r, p) = g - s * (h + g * tau);
                    Vr(r, q) = h + s * (g - h * tau);
                }
            }
        }
        if (!rotated) converged = true;
    }
    if (!converged) return ASI_E_NONFINITE;
    std::vector<int32_t> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return A(x, x) < A(y, y); });
    for (int32_t t = 0; t < m; ++t) {
        theta[t] = A(ord[t], ord[t]);
        if (!std::isfinite(theta[t])) return ASI_E_NONFINITE;
        for (int32_t r = 0; r < m; ++r) Y[(size_t)r * m + t] = Vr(r, ord[t]);
    }
    return ASI_OK;
}
