/*
 * CP-APR MU reference oracle: plain, single-threaded, FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library. The GPU library
 * shares no code, header, table or helper with it.
 *
 * What it computes (paper: "Analyzing the Performance Portability of Tensor
 * Decomposition", Anderson, Teranishi, Dunlavy, Choi, arXiv:2307.03276):
 *
 *   Phi(n) = (X_(n) ./ max(B Pi, eps)) Pi^T          Algorithm 2
 *
 * evaluated one nonzero at a time, as the paper's Section 3.1 describes
 * (forming X_(n) and Pi explicitly is avoided): for nonzero k with
 * coordinates (i_1..i_N) and value x_k,
 *   pi_k[r] = prod_{m != n} A(m)[i_m, r]           (row k of Pi^T, Algorithm 1 Pi line)
 *   m_k     = sum_r B[i_n, r] * pi_k[r]            (entry of B Pi)
 *   s_k     = x_k / max(m_k, eps)                  (elementwise divide with clamp)
 *   Phi[i_n, r] += s_k * pi_k[r]                   (product with Pi^T)
 * Entries of Phi are accumulated with Neumaier's compensated summation so
 * that the oracle's own rounding error is far below the parity tolerance.
 *
 * The MU inner loop, outer loop, lambda update and normalisation follow
 * Algorithm 1. The paper leaves three things open; the readings taken here:
 *   - KKT test: viol = max |min(B, 1 - Phi)| over all entries, checked after
 *     each Phi and before the update; the inner loop stops when viol < tau
 *     (tau <= 0 disables the test, giving Algorithm 1's fixed schedule).
 *   - S (inadmissible zeros): from the second outer iteration on, an entry
 *     with A(n)[i,r] < kappa_tol and the previous outer iteration's
 *     Phi(n)[i,r] > 1 is raised by kappa before B is formed.
 *   - lambda = e^T B (column sums, 1-norm); a zero column keeps A = 0.
 * The outer loop stops early (tau > 0) when no mode performed an update.
 *
 * Log-likelihood (evaluation only): sum_k x_k log(max(m_k, eps)) -
 * sum_r lambda_r prod_m sum_i A(m)[i, r], the Poisson log-likelihood without
 * the constant -sum log(x_k!).
 *
 * Tensor layout: idx[m * nnz + k] is the 0-based mode-m coordinate of nonzero
 * k (int32), vals[k] its value. Matrices are row-major I x R.
 * Return codes: 0 OK, -1 invalid argument, -2 out of memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Neumaier compensated add of x into (*s, *c). */
static void neumaier_add(double* s, double* c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

static int check_args(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                      const double* vals, int R)
{
    if (nmodes < 2 || R < 1 || nnz < 0 || !dims) return -1;
    if (nnz > 0 && (!idx || !vals)) return -1;
    for (int m = 0; m < nmodes; ++m)
        if (dims[m] < 1) return -1;
    return 0;
}

/* Phi restricted to the rows i with row_mask[i] != 0 (row_mask NULL = all rows).
 * Rows outside the mask are left untouched; rows inside are overwritten. */
int oracle_phi_rows(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                    const double* vals, int mode, int R, const double* B,
                    const double* const* A, double eps, const uint8_t* row_mask, double* Phi)
{
    if (check_args(nmodes, dims, nnz, idx, vals, R) || mode < 0 || mode >= nmodes || !B || !Phi)
        return -1;
    const int64_t In = dims[mode];
    double* comp = (double*)calloc((size_t)In * R, sizeof(double));
    double* pi = (double*)malloc((size_t)R * sizeof(double));
    if (!comp || !pi) { free(comp); free(pi); return -2; }
    for (int64_t i = 0; i < In; ++i)
        if (!row_mask || row_mask[i])
            for (int r = 0; r < R; ++r) Phi[i * R + r] = 0.0;

    for (int64_t k = 0; k < nnz; ++k) {
        const int64_t i = idx[(int64_t)mode * nnz + k];
        if (row_mask && !row_mask[i]) continue;
        /* pi_k: product over the other modes, ascending m */
        for (int r = 0; r < R; ++r) pi[r] = 1.0;
        for (int m = 0; m < nmodes; ++m) {
            if (m == mode) continue;
            const double* row = A[m] + (int64_t)idx[(int64_t)m * nnz + k] * R;
            for (int r = 0; r < R; ++r) pi[r] *= row[r];
        }
        /* m_k = <B[i,:], pi_k>, ascending r */
        double mk = 0.0;
        for (int r = 0; r < R; ++r) mk += B[i * R + r] * pi[r];
        const double s = vals[k] / (mk > eps ? mk : eps);
        for (int r = 0; r < R; ++r)
            neumaier_add(&Phi[i * R + r], &comp[i * R + r], s * pi[r]);
    }
    for (int64_t i = 0; i < In; ++i)
        if (!row_mask || row_mask[i])
            for (int r = 0; r < R; ++r) Phi[i * R + r] += comp[i * R + r];
    free(comp);
    free(pi);
    return 0;
}

int oracle_phi(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
               const double* vals, int mode, int R, const double* B, const double* const* A,
               double eps, double* Phi)
{
    return oracle_phi_rows(nmodes, dims, nnz, idx, vals, mode, R, B, A, eps, NULL, Phi);
}

/* max over entries of |min(B, 1 - Phi)| (rows restricted by row_mask if given) */
static double kkt_violation(int64_t In, int R, const double* B, const double* Phi,
                            const uint8_t* row_mask)
{
    double v = 0.0;
    for (int64_t i = 0; i < In; ++i) {
        if (row_mask && !row_mask[i]) continue;
        for (int r = 0; r < R; ++r) {
            double b = B[i * R + r], q = 1.0 - Phi[i * R + r];
            double t = fabs(b < q ? b : q);
            if (t > v) v = t;
        }
    }
    return v;
}

/* MU inner iterations for one mode (Algorithm 1, inner loop). B is updated in
 * place; Phi_last receives the last Phi computed. viol_hist (may be NULL, lmax
 * entries) receives each iteration's KKT violation. With a row mask the work is
 * restricted to those rows; this is exact only when tau <= 0, because the inner
 * loop is otherwise row-separable (Pi is fixed inside it). */
int oracle_mu_inner_rows(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                         const double* vals, int mode, int R, double* B, const double* const* A,
                         int lmax, double tau, double eps, const uint8_t* row_mask,
                         double* Phi_last, double* viol_hist, int* n_updates, double* last_viol)
{
    if (check_args(nmodes, dims, nnz, idx, vals, R) || mode < 0 || mode >= nmodes || lmax < 1)
        return -1;
    const int64_t In = dims[mode];
    int upd = 0;
    double viol = 0.0;
    for (int l = 0; l < lmax; ++l) {
        int rc = oracle_phi_rows(nmodes, dims, nnz, idx, vals, mode, R, B, A, eps, row_mask,
                                 Phi_last);
        if (rc) return rc;
        viol = kkt_violation(In, R, B, Phi_last, row_mask);
        if (viol_hist) viol_hist[l] = viol;
        if (tau > 0.0 && viol < tau) break;
        for (int64_t i = 0; i < In; ++i) {
            if (row_mask && !row_mask[i]) continue;
            for (int r = 0; r < R; ++r) B[i * R + r] *= Phi_last[i * R + r];
        }
        ++upd;
    }
    if (n_updates) *n_updates = upd;
    if (last_viol) *last_viol = viol;
    return 0;
}

int oracle_mu_inner(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                    const double* vals, int mode, int R, double* B, const double* const* A,
                    int lmax, double tau, double eps, double* Phi_last, double* viol_hist,
                    int* n_updates, double* last_viol)
{
    return oracle_mu_inner_rows(nmodes, dims, nnz, idx, vals, mode, R, B, A, lmax, tau, eps,
                                NULL, Phi_last, viol_hist, n_updates, last_viol);
}

/* Full CP-APR MU (Algorithm 1). lam (R) and A[m] (I_m x R) are in/out.
 * Outputs: outer iterations run, total inner updates, converged flag, and the
 * last KKT violation seen per mode maximised over modes of the final sweep. */
int oracle_solve(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                 const double* vals, int R, double* lam, double* const* A, int kmax, int lmax,
                 double tau, double eps, double kappa, double kappa_tol, int* outer_iters,
                 int64_t* inner_updates, int* converged, double* kkt)
{
    if (check_args(nmodes, dims, nnz, idx, vals, R) || kmax < 1 || lmax < 1 || !lam || !A)
        return -1;
    int64_t maxI = 0;
    for (int m = 0; m < nmodes; ++m) if (dims[m] > maxI) maxI = dims[m];
    double* B = (double*)malloc((size_t)maxI * R * sizeof(double));
    double** phi_prev = (double**)calloc((size_t)(unsigned)nmodes, sizeof(double*));
    if (!B || !phi_prev) { free(B); free(phi_prev); return -2; }
    for (int m = 0; m < nmodes; ++m) {
        phi_prev[m] = (double*)calloc((size_t)dims[m] * R, sizeof(double));
        if (!phi_prev[m]) {
            for (int q = 0; q < m; ++q) free(phi_prev[q]);
            free(phi_prev); free(B);
            return -2;
        }
    }
    int k, conv = 0, rc = 0;
    int64_t total_upd = 0;
    double kkt_sweep = 0.0;
    for (k = 1; k <= kmax; ++k) {
        int any_update = 0;
        kkt_sweep = 0.0;
        for (int n = 0; n < nmodes; ++n) {
            const int64_t In = dims[n];
            double* An = A[n];
            /* S: lift inadmissible zeros (from the second outer iteration on) */
            if (k > 1)
                for (int64_t e = 0; e < In * R; ++e)
                    if (An[e] < kappa_tol && phi_prev[n][e] > 1.0) An[e] += kappa;
            /* B = (A + S) Lambda */
            for (int64_t i = 0; i < In; ++i)
                for (int r = 0; r < R; ++r) B[i * R + r] = An[i * R + r] * lam[r];
            int upd = 0;
            double v = 0.0;
            rc = oracle_mu_inner(nmodes, dims, nnz, idx, vals, n, R, B,
                                 (const double* const*)A, lmax, tau, eps, phi_prev[n], NULL,
                                 &upd, &v);
            if (rc) goto done;
            if (upd > 0) any_update = 1;
            total_upd += upd;
            if (v > kkt_sweep) kkt_sweep = v;
            /* lambda = e^T B; A(n) = B Lambda^-1 */
            for (int r = 0; r < R; ++r) {
                double s = 0.0, c = 0.0;
                for (int64_t i = 0; i < In; ++i) neumaier_add(&s, &c, B[i * R + r]);
                lam[r] = s + c;
            }
            for (int64_t i = 0; i < In; ++i)
                for (int r = 0; r < R; ++r)
                    An[i * R + r] = lam[r] > 0.0 ? B[i * R + r] / lam[r] : 0.0;
        }
        if (tau > 0.0 && !any_update) { conv = 1; break; }
    }
    if (k > kmax) k = kmax;
done:
    if (outer_iters) *outer_iters = k;
    if (inner_updates) *inner_updates = total_upd;
    if (converged) *converged = conv;
    if (kkt) *kkt = kkt_sweep;
    for (int m = 0; m < nmodes; ++m) free(phi_prev[m]);
    free(phi_prev);
    free(B);
    return rc;
}

/* Poisson log-likelihood without the -log(x!) constant. */
int oracle_loglik(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                  const double* vals, int R, const double* lam, const double* const* A,
                  double eps, double* out)
{
    if (check_args(nmodes, dims, nnz, idx, vals, R) || !lam || !A || !out) return -1;
    double s = 0.0, c = 0.0;
    for (int64_t k = 0; k < nnz; ++k) {
        double mk = 0.0;
        for (int r = 0; r < R; ++r) {
            double p = lam[r];
            for (int m = 0; m < nmodes; ++m) p *= A[m][(int64_t)idx[(int64_t)m * nnz + k] * R + r];
            mk += p;
        }
        neumaier_add(&s, &c, vals[k] * log(mk > eps ? mk : eps));
    }
    double mass = 0.0;
    for (int r = 0; r < R; ++r) {
        double p = lam[r];
        for (int m = 0; m < nmodes; ++m) {
            double cs = 0.0, cc = 0.0;
            for (int64_t i = 0; i < dims[m]; ++i) neumaier_add(&cs, &cc, A[m][i * R + r]);
            p *= cs + cc;
        }
        mass += p;
    }
    *out = (s + c) - mass;
    return 0;
}

/* MTTKRP for CP-ALS (the paper's Experiment 8, Eqs. 10-12): for every nonzero,
 * M[i_n, :] += x_k * prod_{m != n} A(m)[i_m, :]. Neumaier per entry. */
int oracle_mttkrp(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                  const double* vals, int mode, int R, const double* const* A, double* M)
{
    if (check_args(nmodes, dims, nnz, idx, vals, R) || mode < 0 || mode >= nmodes || !M)
        return -1;
    const int64_t In = dims[mode];
    double* comp = (double*)calloc((size_t)In * R, sizeof(double));
    double* t = (double*)malloc((size_t)R * sizeof(double));
    if (!comp || !t) { free(comp); free(t); return -2; }
    memset(M, 0, (size_t)In * R * sizeof(double));
    for (int64_t k = 0; k < nnz; ++k) {
        const int64_t i = idx[(int64_t)mode * nnz + k];
        for (int r = 0; r < R; ++r) t[r] = 1.0;
        for (int m = 0; m < nmodes; ++m) {
            if (m == mode) continue;
            const double* row = A[m] + (int64_t)idx[(int64_t)m * nnz + k] * R;
            for (int r = 0; r < R; ++r) t[r] *= row[r];
        }
        for (int r = 0; r < R; ++r) neumaier_add(&M[i * R + r], &comp[i * R + r], vals[k] * t[r]);
    }
    for (int64_t e = 0; e < In * R; ++e) M[e] += comp[e];
    free(comp);
    free(t);
    return 0;
}
