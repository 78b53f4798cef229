// Iterative solution of the BEM collocation system with the matrix-free product.
//
// The paper computes the charge densities with KEMField's iterative methods on matrices
// that are never stored (Sec. 5); here: restarted GMRES, right-preconditioned by the
// diagonal of the collocation matrix (the exact on-element potentials), with classical
// Gram-Schmidt and one reorthogonalisation, and optionally mixed-precision iterative
// refinement around it.  Each product is bemc_collocation_matvec.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "bemc.h"
#include "bemc_internal.h"

namespace bemc {

int solve_gmres(bemc_handle h, const Elements& el, const double* b, double* x, double tol, int max_iter, int m,
                int precision, bemc_solve_info* info, hipStream_t s, std::string& err)
{
    using clock = std::chrono::steady_clock;
    const auto t_start = clock::now();
    const int64_t n = el.ne;
    const int kDotBlocks = 256;
    double *V = nullptr, *w = nullptr, *t = nullptr, *diag = nullptr, *partial = nullptr, *coef = nullptr;
    double* h_partial = nullptr;
    int rc = BEMC_OK;
    auto check = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == BEMC_OK) {
            err = std::string(what) + ": " + hipGetErrorString(e);
            rc = BEMC_E_DEVICE;
        }
        return rc == BEMC_OK;
    };
    if (hipMalloc(reinterpret_cast<void**>(&V), sizeof(double) * (size_t)(m + 1) * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&w), sizeof(double) * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&t), sizeof(double) * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&diag), sizeof(double) * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&partial), sizeof(double) * (size_t)(m + 1) * kDotBlocks) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&coef), sizeof(double) * (m + 1)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h_partial), sizeof(double) * (size_t)(m + 1) * kDotBlocks,
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        err = "solver workspace";
        rc = BEMC_E_OUT_OF_MEMORY;
    }
    // <V_j, v> for j < k, summed on the host in fixed order
    auto dots = [&](const double* Vb, int k, const double* v, double* out) {
        if (!check(launch_multi_dot(Vb, k, n, v, partial, kDotBlocks, s), "dot")) return false;
        if (!check(hipMemcpyAsync(h_partial, partial, sizeof(double) * (size_t)k * kDotBlocks, hipMemcpyDeviceToHost, s),
                   "copy"))
            return false;
        if (!check(hipStreamSynchronize(s), "sync")) return false;
        for (int j = 0; j < k; ++j) {
            double acc = 0.0;
            for (int bb = 0; bb < kDotBlocks; ++bb) acc += h_partial[(size_t)j * kDotBlocks + bb];
            out[j] = acc;
        }
        return true;
    };
    auto put_coef = [&](const double* c, int k) {
        return check(hipMemcpyAsync(coef, c, sizeof(double) * k, hipMemcpyHostToDevice, s), "copy") &&
               check(hipStreamSynchronize(s), "sync");
    };
    // y = A v (potential at all centroids from densities v)
    int products = 0;
    auto apply = [&](const double* v, double* y) {
        const int r = bemc_collocation_matvec(h, v, 1, precision, y, s);
        ++products;
        if (r != BEMC_OK && rc == BEMC_OK) {
            err = std::string("collocation product: ") + bemc_last_error();
            rc = r;
        }
        return rc == BEMC_OK;
    };

    double bnorm = 0.0, res = 0.0;
    bool converged = false;
    if (rc == BEMC_OK && check(launch_self_diag(el, coulomb_constant(), diag, s), "diag") &&
        check(hipMemsetAsync(x, 0, sizeof(double) * n, s), "memset") &&
        check(hipMemcpyAsync(V, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "copy") && dots(V, 1, V, &bnorm)) {
        bnorm = std::sqrt(bnorm);
        res = bnorm;
        converged = bnorm == 0.0;
        std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hcol(m + 1), h2(m + 1);
        double beta = bnorm;  // V[0] holds the unnormalised residual
        while (!converged && rc == BEMC_OK && products < max_iter) {
            const double inv = 1.0 / beta;
            if (!put_coef(&inv, 1) || !check(launch_combine(V, 0.0, V, coef, 1, n, nullptr, s), "scale")) break;
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int j = 0;
            for (; j < m && products < max_iter; ++j) {
                // w = A D^-1 v_j
                if (!check(launch_divide(t, V + (size_t)j * n, diag, n, s), "precond") || !apply(t, w)) break;
                // two passes of classical Gram-Schmidt against v_0 .. v_j
                if (!dots(V, j + 1, w, hcol.data())) break;
                for (int i = 0; i <= j; ++i) hcol[i] = -hcol[i];
                if (!put_coef(hcol.data(), j + 1) || !check(launch_combine(w, 1.0, V, coef, j + 1, n, nullptr, s), "axpy"))
                    break;
                if (!dots(V, j + 1, w, h2.data())) break;
                for (int i = 0; i <= j; ++i) h2[i] = -h2[i];
                if (!put_coef(h2.data(), j + 1) || !check(launch_combine(w, 1.0, V, coef, j + 1, n, nullptr, s), "axpy"))
                    break;
                double hn = 0.0;
                if (!dots(w, 1, w, &hn)) break;
                hn = std::sqrt(hn);
                for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = -(hcol[i] + h2[i]);
                H[(size_t)(j + 1) * m + j] = hn;
                if (hn > 0.0) {
                    const double invh = 1.0 / hn;
                    if (!check(hipMemcpyAsync(V + (size_t)(j + 1) * n, w, sizeof(double) * n, hipMemcpyDeviceToDevice, s),
                               "copy") ||
                        !put_coef(&invh, 1) ||
                        !check(launch_combine(V + (size_t)(j + 1) * n, 0.0, V + (size_t)(j + 1) * n, coef, 1, n, nullptr, s),
                               "scale"))
                        break;
                }
                // Givens rotations on column j
                for (int i = 0; i < j; ++i) {
                    const double a0 = H[(size_t)i * m + j], a1 = H[(size_t)(i + 1) * m + j];
                    H[(size_t)i * m + j] = cs[i] * a0 + sn[i] * a1;
                    H[(size_t)(i + 1) * m + j] = -sn[i] * a0 + cs[i] * a1;
                }
                const double a0 = H[(size_t)j * m + j], a1 = H[(size_t)(j + 1) * m + j];
                const double r = std::hypot(a0, a1);
                cs[j] = r > 0 ? a0 / r : 1.0;
                sn[j] = r > 0 ? a1 / r : 0.0;
                H[(size_t)j * m + j] = r;
                H[(size_t)(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                res = std::fabs(g[j + 1]);
                if (res <= tol * bnorm || hn == 0.0) {
                    ++j;
                    converged = true;
                    break;
                }
            }
            if (rc != BEMC_OK || j == 0) break;
            // y = H^-1 g (upper triangular), x += D^-1 V y
            for (int i = j - 1; i >= 0; --i) {
                double acc = g[i];
                for (int k = i + 1; k < j; ++k) acc -= H[(size_t)i * m + k] * y[k];
                y[i] = acc / H[(size_t)i * m + i];
            }
            if (!put_coef(y.data(), j) || !check(launch_combine(x, 1.0, V, coef, j, n, diag, s), "update")) break;
            // true residual b - A x for the restart (and the final report)
            if (!apply(x, w)) break;
            const double minus1 = -1.0;
            if (!check(hipMemcpyAsync(V, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "copy") ||
                !put_coef(&minus1, 1) || !check(launch_combine(V, 1.0, w, coef, 1, n, nullptr, s), "residual"))
                break;
            double rr = 0.0;
            if (!dots(V, 1, V, &rr)) break;
            beta = std::sqrt(rr);
            res = beta;
            converged = beta <= tol * bnorm;
        }
    }
    if (info) {
        info->iterations = products;
        info->converged = converged ? 1 : 0;
        info->rel_residual = bnorm > 0 ? res / bnorm : 0.0;
        info->seconds = std::chrono::duration<double>(clock::now() - t_start).count();
    }
    if (V) (void)hipFree(V);
    if (w) (void)hipFree(w);
    if (t) (void)hipFree(t);
    if (diag) (void)hipFree(diag);
    if (partial) (void)hipFree(partial);
    if (coef) (void)hipFree(coef);
    if (h_partial) (void)hipHostFree(h_partial);
    return rc;
}

// Mixed-precision iterative refinement: the residual r = b - A x is formed with FP64
// products, each correction A d = r is solved by GMRES on mixed products to kInnerTol of
// |r| (their accuracy is ~1e-7), and x += d, until |r| <= tol |b|.  Stops early when an
// outer step no longer reduces |r| tenfold.
int solve_refined(bemc_handle h, const Elements& el, const double* b, double* x, double tol, int max_iter, int m,
                  bemc_solve_info* info, hipStream_t s, std::string& err)
{
    using clock = std::chrono::steady_clock;
    const auto t_start = clock::now();
    constexpr double kInnerTol = 1e-6;
    constexpr int kMaxOuter = 20;
    const int64_t n = el.ne;
    const int kDotBlocks = 256;
    double *r = nullptr, *d = nullptr, *ax = nullptr, *coef = nullptr, *partial = nullptr, *h_partial = nullptr;
    int rc = BEMC_OK;
    auto check = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == BEMC_OK) {
            err = std::string(what) + ": " + hipGetErrorString(e);
            rc = BEMC_E_DEVICE;
        }
        return rc == BEMC_OK;
    };
    if (hipMalloc(reinterpret_cast<void**>(&r), sizeof(double) * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d), sizeof(double) * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&ax), sizeof(double) * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&coef), sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&partial), sizeof(double) * kDotBlocks) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h_partial), sizeof(double) * kDotBlocks, hipHostMallocDefault) !=
            hipSuccess) {
        (void)hipGetLastError();
        err = "refinement workspace";
        rc = BEMC_E_OUT_OF_MEMORY;
    }
    // |v|, partial sums added on the host in fixed order
    auto norm = [&](const double* v, double* out) {
        if (!check(launch_multi_dot(v, 1, n, v, partial, kDotBlocks, s), "dot") ||
            !check(hipMemcpyAsync(h_partial, partial, sizeof(double) * kDotBlocks, hipMemcpyDeviceToHost, s), "copy") ||
            !check(hipStreamSynchronize(s), "sync"))
            return false;
        double acc = 0.0;
        for (int i = 0; i < kDotBlocks; ++i) acc += h_partial[i];
        *out = std::sqrt(acc);
        return true;
    };
    // y = y + c v
    auto axpy = [&](double* y, double c, const double* v) {
        return check(hipMemcpyAsync(coef, &c, sizeof(double), hipMemcpyHostToDevice, s), "copy") &&
               check(hipStreamSynchronize(s), "sync") && check(launch_combine(y, 1.0, v, coef, 1, n, nullptr, s), "axpy");
    };
    int products = 0, outer = 0;
    double bnorm = 0.0, rnorm = 0.0;
    bool converged = false;
    if (rc == BEMC_OK && check(hipMemsetAsync(x, 0, sizeof(double) * n, s), "memset") &&
        check(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "copy") && norm(b, &bnorm)) {
        rnorm = bnorm;
        converged = bnorm == 0.0;
        while (!converged && products < max_iter && outer < kMaxOuter) {
            bemc_solve_info inner{};
            const double inner_tol = std::max(kInnerTol, tol * bnorm / rnorm);
            const int r2 = solve_gmres(h, el, r, d, inner_tol, max_iter - products, m, BEMC_MIXED, &inner, s, err);
            products += inner.iterations;
            if (r2 != BEMC_OK) {
                rc = r2;
                break;
            }
            if (!axpy(x, 1.0, d)) break;
            // r = b - A x with an FP64 product
            const int r3 = bemc_collocation_matvec(h, x, 1, BEMC_FP64, ax, s);
            ++products;
            ++outer;
            if (r3 != BEMC_OK) {
                err = std::string("collocation product: ") + bemc_last_error();
                rc = r3;
                break;
            }
            if (!check(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "copy") ||
                !axpy(r, -1.0, ax))
                break;
            const double prev = rnorm;
            if (!norm(r, &rnorm)) break;
            converged = rnorm <= tol * bnorm;
            if (!converged && rnorm > 0.1 * prev) break;  // no longer converging
        }
    }
    if (info) {
        info->iterations = products;
        info->converged = converged ? 1 : 0;
        info->rel_residual = bnorm > 0 ? rnorm / bnorm : 0.0;
        info->seconds = std::chrono::duration<double>(clock::now() - t_start).count();
        info->refinements = outer;
    }
    if (r) (void)hipFree(r);
    if (d) (void)hipFree(d);
    if (ax) (void)hipFree(ax);
    if (coef) (void)hipFree(coef);
    if (partial) (void)hipFree(partial);
    if (h_partial) (void)hipHostFree(h_partial);
    return rc;
}

}  // namespace bemc
