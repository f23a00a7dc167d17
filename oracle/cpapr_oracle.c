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

/* ------------------------------------------------------------------------
 * PQNR: projected quasi-Newton for the row subproblems.
 *
 * The paper names this CP-APR variant (Background: each row of a mode's
 * factor is its own subproblem and converges independently) but prints no
 * algorithm; the readings below follow the row-subproblem formulation of the
 * method it cites, written from that formulation:
 *
 *   f_i(b) = sum_r b_r - sum_{k in row i} x_k log(max(b . pi_k, eps)),  b >= 0,
 *
 * the negative Poisson log-likelihood of row i of B = A(n) Lambda with the
 * other factors' columns summing to one (so the linear term is sum_r b_r).
 * Its gradient is g = 1 - phi_i with phi_i row i of Phi(n) (Algorithm 2), so
 * KKT is min(b, g) = 0, the same test as the MU loop.
 *
 * One iteration of one row, given b >= 0:
 *   1. phi = sum_k x_k/max(m_k, eps) pi_k, g = 1 - phi, viol = max|min(b, g)|;
 *      stop the row when tau > 0 and viol < tau.
 *   2. After a step: s = last step, y = g - g_prev; keep (s, y) (at most
 *      PQNR_MEM pairs, oldest dropped) when s.y > PQNR_CURV |s| |y|.
 *   3. Bound set: b_r == 0 and g_r > 0; the others are free.
 *   4. Direction: without pairs the scaled gradient -b .* g (the MU step);
 *      with pairs the L-BFGS two-loop recursion over the free set (pairs with
 *      free-set curvature <= 0 skipped, initial scaling s.y / y.y of the newest
 *      usable pair), zero on bound entries; if g.d >= 0, or no pair is usable,
 *      the scaled gradient.
 *   5. Projected backtracking: for alpha = 1, 1/2, ... (PQNR_TRIALS trials)
 *      delta = max(b + alpha d, 0) - b; accept the first with g.delta < 0 and
 *      f(b + delta) - f(b) <= PQNR_SIGMA g.delta, where the decrease is
 *      formed term by term (sum_r delta_r - sum_k x_k log1p(delta.pi_k / m_k))
 *      instead of as a difference of two large sums. The objective is the
 *      negative log-likelihood, finite only while every model value of the
 *      row is positive: a trial that brings some m_k (above eps now) down to
 *      eps or below is rejected (the floor only guards a point that is
 *      already there, for which the clamped logarithms are used). With no
 *      acceptable trial the MU step b .* phi = b + (-b .* g) is taken (it
 *      never increases f and keeps every m_k positive) and the kept pairs
 *      are dropped (they led to a direction without sufficient decrease).
 *   6. b <- b + delta; the iteration counts as an update.
 * The outer loop is Algorithm 1's, S shift included: a row entry held at
 * zero whose gradient is negative (Phi > 1) is an inadmissible zero for any
 * inner solver, and the shift lifts it before B is formed.
 * ------------------------------------------------------------------------ */
#define PQNR_MEM 3
#define PQNR_CURV 1e-10
#define PQNR_SIGMA 1e-4
#define PQNR_TRIALS 4

typedef struct {
    int R, count, head; /* ring of pairs: newest at head - 1 */
    double s[PQNR_MEM][256], y[PQNR_MEM][256];
} pqnr_pairs;

static double dot_masked(int R, const double* a, const double* b, const uint8_t* free_set)
{
    double t = 0.0;
    for (int r = 0; r < R; ++r)
        if (!free_set || free_set[r]) t += a[r] * b[r];
    return t;
}

/* one row of one mode: nz[] are the row's nonzero ids, pis[j*R..] their pi */
static void pqnr_row(int R, int64_t nrow, const double* xs, const double* pis, double* b,
                     int lmax, double tau, double eps, int* steps_out, double* viol_out, double* phi_out)
{
    pqnr_pairs P;
    P.R = R;
    P.count = 0;
    P.head = 0;
    double phi[256], comp[256], g[256], gprev[256], d[256], q[256], delta[256], slast[256];
    double a[PQNR_MEM];
    uint8_t fr[256];
    int steps = 0;
    double viol = 0.0;
    for (int l = 0; l < lmax; ++l) {
        /* 1. gradient from Phi's row */
        for (int r = 0; r < R; ++r) phi[r] = comp[r] = 0.0;
        for (int64_t j = 0; j < nrow; ++j) {
            const double* pi = pis + j * R;
            double m = 0.0;
            for (int r = 0; r < R; ++r) m += b[r] * pi[r];
            const double sc = xs[j] / (m > eps ? m : eps);
            for (int r = 0; r < R; ++r) neumaier_add(&phi[r], &comp[r], sc * pi[r]);
        }
        viol = 0.0;
        for (int r = 0; r < R; ++r) {
            phi[r] += comp[r];
            g[r] = 1.0 - phi[r];
            const double t = fabs(b[r] < g[r] ? b[r] : g[r]);
            if (t > viol) viol = t;
        }
        if (tau > 0.0 && viol < tau) break;
        /* 2. curvature pair from the previous step */
        if (l > 0) {
            double y[256];
            for (int r = 0; r < R; ++r) y[r] = g[r] - gprev[r];
            const double sy = dot_masked(R, slast, y, NULL);
            const double ss = dot_masked(R, slast, slast, NULL), yy = dot_masked(R, y, y, NULL);
            if (sy > PQNR_CURV * sqrt(ss * yy)) {
                for (int r = 0; r < R; ++r) {
                    P.s[P.head][r] = slast[r];
                    P.y[P.head][r] = y[r];
                }
                P.head = (P.head + 1) % PQNR_MEM;
                if (P.count < PQNR_MEM) ++P.count;
            }
        }
        /* 3. free set */
        for (int r = 0; r < R; ++r) fr[r] = !(b[r] == 0.0 && g[r] > 0.0);
        /* 4. direction */
        int use_mu = 1;
        if (P.count > 0) {
            for (int r = 0; r < R; ++r) q[r] = fr[r] ? g[r] : 0.0;
            double gamma = 0.0;
            int usable = 0;
            for (int c = 0; c < P.count; ++c) { /* newest to oldest */
                const int j = (P.head - 1 - c + 2 * PQNR_MEM) % PQNR_MEM;
                const double sy = dot_masked(R, P.s[j], P.y[j], fr);
                a[c] = 0.0;
                if (sy <= 0.0) continue;
                if (!usable) {
                    const double yy = dot_masked(R, P.y[j], P.y[j], fr);
                    gamma = yy > 0.0 ? sy / yy : 0.0;
                }
                usable = 1;
                a[c] = dot_masked(R, P.s[j], q, fr) / sy;
                for (int r = 0; r < R; ++r)
                    if (fr[r]) q[r] -= a[c] * P.y[j][r];
            }
            if (usable && gamma > 0.0) {
                for (int r = 0; r < R; ++r) q[r] *= gamma;
                for (int c = P.count - 1; c >= 0; --c) { /* oldest to newest */
                    const int j = (P.head - 1 - c + 2 * PQNR_MEM) % PQNR_MEM;
                    const double sy = dot_masked(R, P.s[j], P.y[j], fr);
                    if (sy <= 0.0) continue;
                    const double beta = dot_masked(R, P.y[j], q, fr) / sy;
                    for (int r = 0; r < R; ++r)
                        if (fr[r]) q[r] += (a[c] - beta) * P.s[j][r];
                }
                double gd = 0.0;
                for (int r = 0; r < R; ++r) {
                    d[r] = fr[r] ? -q[r] : 0.0;
                    gd += g[r] * d[r];
                }
                use_mu = !(gd < 0.0);
            }
        }
        if (use_mu)
            for (int r = 0; r < R; ++r) d[r] = -b[r] * g[r];
        /* 5. projected backtracking line search */
        int accepted = 0;
        double alpha = 1.0;
        for (int t = 0; t < PQNR_TRIALS && !accepted; ++t, alpha *= 0.5) {
            double gdel = 0.0, lin = 0.0;
            for (int r = 0; r < R; ++r) {
                const double nb = b[r] + alpha * d[r];
                delta[r] = (nb > 0.0 ? nb : 0.0) - b[r];
                gdel += g[r] * delta[r];
                lin += delta[r];
            }
            if (!(gdel < 0.0)) continue;
            double ls = 0.0, lc = 0.0;
            int outside = 0;
            for (int64_t j = 0; j < nrow; ++j) {
                const double* pi = pis + j * R;
                double m = 0.0, dm = 0.0;
                for (int r = 0; r < R; ++r) {
                    m += b[r] * pi[r];
                    dm += delta[r] * pi[r];
                }
                const double m1 = m + dm;
                double term;
                if (m > eps && m1 > eps) {
                    term = log1p(dm / m);
                } else if (m > eps) {
                    outside = 1; /* the trial leaves the domain of f */
                    break;
                } else {
                    term = log(m1 > eps ? m1 : eps) - log(eps);
                }
                neumaier_add(&ls, &lc, xs[j] * term);
            }
            if (outside) continue;
            const double df = lin - (ls + lc);
            if (df <= PQNR_SIGMA * gdel) accepted = 1;
        }
        if (!accepted) P.count = 0; /* the curvature pairs misled the search: drop them */
        if (!accepted) /* the MU step b .* phi, written as b + (-b .* g) */
            for (int r = 0; r < R; ++r) delta[r] = -b[r] * g[r];
        /* 6. step */
        for (int r = 0; r < R; ++r) {
            b[r] += delta[r];
            slast[r] = delta[r];
            gprev[r] = g[r];
        }
        ++steps;
    }
    *steps_out = steps;
    *viol_out = viol;
    if (phi_out)
        for (int r = 0; r < R; ++r) phi_out[r] = phi[r]; /* the last Phi row computed */
}

/* ------------------------------------------------------------------------
 * PDNR: projected damped Newton for the row subproblems, the other row-wise
 * variant the Background names. Same row objective f_i, gradient g = 1 - phi
 * and KKT test as PQNR above; the direction comes from the row's Hessian
 *
 *   H = sum_{k in row i} x_k / max(m_k, eps)^2  pi_k pi_k^T,   m_k = b . pi_k
 *
 * (the second derivative of -x log(b . pi) is x pi pi^T / (b . pi)^2; with the
 * floor it is taken at the clamped value, as phi is). The paper prints no
 * algorithm for the variant; the readings below are this library's:
 *
 * One iteration of one row, given b >= 0 and the row's damping mu:
 *   1. phi, g, viol as PQNR; stop the row when tau > 0 and viol < tau.
 *   2. H as above (w_k = (x_k / mm_k) / mm_k, mm_k = max(m_k, eps)).
 *   3. Held set: g_r > 0 and b_r <= PDNR_HELD; the other entries are free.
 *   4. Direction: d = -g on held entries; on the free set F the damped Newton
 *      system (H_FF + mu t I) d_F = -g_F, t = trace(H_FF) / |F| (so the
 *      damping scales with the row's curvature), solved by Cholesky in index
 *      order. If F is empty, d = -g. If t is not > 0, a Cholesky pivot is not
 *      > 0, or g.d >= 0: the MU direction -b .* g.
 *   5. Projected backtracking along d exactly as PQNR's (PDNR_TRIALS trials,
 *      sufficient decrease PDNR_SIGMA, trials leaving the objective's domain
 *      rejected). With no acceptable trial: the MU step b + (-b .* g) and
 *      mu <- min(PDNR_MU_STEP mu, PDNR_MU_MAX).
 *   6. Accepted step delta with change df: predicted change of the quadratic
 *      model pred = -(g.delta + delta^T H delta / 2), rho = -df / pred (0 if
 *      pred <= 0); rho < 1/4: mu <- min(PDNR_MU_STEP mu, PDNR_MU_MAX);
 *      rho > 3/4: mu <- max(mu / PDNR_MU_STEP, PDNR_MU_MIN).
 *   7. b <- b + delta; the iteration counts as a step.
 * mu starts at PDNR_MU0 for every row at the start of an inner loop.
 * ------------------------------------------------------------------------ */
#define PDNR_TRIALS 4
#define PDNR_SIGMA 1e-4
#define PDNR_HELD 1e-10
#define PDNR_MU0 1e-3
#define PDNR_MU_MIN 1e-8
#define PDNR_MU_MAX 1e8
#define PDNR_MU_STEP 4.0

/* Projected backtracking from b along d (gradient g): trials alpha = 1, 1/2,
 * ...; the first with g.delta < 0 and f(b + delta) - f(b) <= sigma g.delta
 * whose model values all stay in the objective's domain is accepted (delta
 * and df written, returns 1); none: returns 0. */
static int projected_search(int R, int64_t nrow, const double* xs, const double* pis, const double* b,
                            const double* g, const double* d, double eps, int trials, double sigma,
                            double* delta, double* df_out)
{
    double alpha = 1.0;
    for (int t = 0; t < trials; ++t, alpha *= 0.5) {
        double gdel = 0.0, lin = 0.0;
        for (int r = 0; r < R; ++r) {
            const double nb = b[r] + alpha * d[r];
            delta[r] = (nb > 0.0 ? nb : 0.0) - b[r];
            gdel += g[r] * delta[r];
            lin += delta[r];
        }
        if (!(gdel < 0.0)) continue;
        double ls = 0.0, lc = 0.0;
        int outside = 0;
        for (int64_t j = 0; j < nrow; ++j) {
            const double* pi = pis + j * R;
            double m = 0.0, dm = 0.0;
            for (int r = 0; r < R; ++r) {
                m += b[r] * pi[r];
                dm += delta[r] * pi[r];
            }
            const double m1 = m + dm;
            double term;
            if (m > eps && m1 > eps) {
                term = log1p(dm / m);
            } else if (m > eps) {
                outside = 1;
                break;
            } else {
                term = log(m1 > eps ? m1 : eps) - log(eps);
            }
            neumaier_add(&ls, &lc, xs[j] * term);
        }
        if (outside) continue;
        const double df = lin - (ls + lc);
        if (df <= sigma * gdel) {
            *df_out = df;
            return 1;
        }
    }
    return 0;
}

/* one row of one mode; work holds 3 R x R matrices */
static void pdnr_row(int R, int64_t nrow, const double* xs, const double* pis, double* b, int lmax,
                     double tau, double eps, int* steps_out, double* viol_out, double* phi_out, double* work)
{
    double* H = work;              /* Hessian */
    double* Hc = work + R * R;     /* its compensation terms */
    double* L = work + 2 * R * R;  /* damped free-set matrix, overwritten by its Cholesky factor */
    double phi[256], comp[256], g[256], d[256], delta[256], y[256];
    int fidx[256];
    double mu = PDNR_MU0;
    int steps = 0;
    double viol = 0.0;
    for (int l = 0; l < lmax; ++l) {
        /* 1-2. gradient and Hessian */
        for (int r = 0; r < R; ++r) phi[r] = comp[r] = 0.0;
        for (int e = 0; e < R * R; ++e) H[e] = Hc[e] = 0.0;
        for (int64_t j = 0; j < nrow; ++j) {
            const double* pi = pis + j * R;
            double m = 0.0;
            for (int r = 0; r < R; ++r) m += b[r] * pi[r];
            const double mm = m > eps ? m : eps;
            const double sc = xs[j] / mm;
            const double w = sc / mm;
            for (int r = 0; r < R; ++r) {
                neumaier_add(&phi[r], &comp[r], sc * pi[r]);
                for (int c = 0; c < R; ++c) neumaier_add(&H[r * R + c], &Hc[r * R + c], w * pi[r] * pi[c]);
            }
        }
        for (int e = 0; e < R * R; ++e) H[e] += Hc[e];
        viol = 0.0;
        for (int r = 0; r < R; ++r) {
            phi[r] += comp[r];
            g[r] = 1.0 - phi[r];
            const double t = fabs(b[r] < g[r] ? b[r] : g[r]);
            if (t > viol) viol = t;
        }
        if (tau > 0.0 && viol < tau) break;
        /* 3. held and free entries */
        int nf = 0;
        double trace = 0.0;
        for (int r = 0; r < R; ++r) {
            if (g[r] > 0.0 && b[r] <= PDNR_HELD) continue;
            fidx[nf++] = r;
            trace += H[r * R + r];
        }
        /* 4. direction */
        int newton = 0;
        for (int r = 0; r < R; ++r) d[r] = -g[r]; /* held entries (and all of d if F is empty) */
        if (nf == 0) {
            newton = 1;
        } else if (trace > 0.0) {
            const double damp = mu * (trace / nf);
            for (int a = 0; a < nf; ++a)
                for (int c = 0; c < nf; ++c)
                    L[a * nf + c] = H[fidx[a] * R + fidx[c]] + (a == c ? damp : 0.0);
            newton = 1;
            for (int c = 0; c < nf && newton; ++c) { /* Cholesky, column by column */
                double piv = L[c * nf + c];
                for (int k = 0; k < c; ++k) piv -= L[c * nf + k] * L[c * nf + k];
                if (!(piv > 0.0)) {
                    newton = 0;
                    break;
                }
                const double lcc = sqrt(piv);
                L[c * nf + c] = lcc;
                for (int a = c + 1; a < nf; ++a) {
                    double v = L[a * nf + c];
                    for (int k = 0; k < c; ++k) v -= L[a * nf + k] * L[c * nf + k];
                    L[a * nf + c] = v / lcc;
                }
            }
            if (newton) {
                for (int a = 0; a < nf; ++a) { /* L y = -g_F */
                    double v = -g[fidx[a]];
                    for (int k = 0; k < a; ++k) v -= L[a * nf + k] * y[k];
                    y[a] = v / L[a * nf + a];
                }
                for (int a = nf - 1; a >= 0; --a) { /* L^T d_F = y */
                    double v = y[a];
                    for (int k = a + 1; k < nf; ++k) v -= L[k * nf + a] * d[fidx[k]];
                    d[fidx[a]] = v / L[a * nf + a];
                }
            }
        }
        if (newton) {
            double gd = 0.0;
            for (int r = 0; r < R; ++r) gd += g[r] * d[r];
            newton = gd < 0.0;
        }
        if (!newton)
            for (int r = 0; r < R; ++r) d[r] = -b[r] * g[r];
        /* 5-6. line search and damping */
        double df = 0.0;
        if (projected_search(R, nrow, xs, pis, b, g, d, eps, PDNR_TRIALS, PDNR_SIGMA, delta, &df)) {
            double gdel = 0.0, quad = 0.0;
            for (int r = 0; r < R; ++r) {
                double hd = 0.0;
                for (int c = 0; c < R; ++c) hd += H[r * R + c] * delta[c];
                gdel += g[r] * delta[r];
                quad += delta[r] * hd;
            }
            const double pred = -(gdel + 0.5 * quad);
            const double rho = pred > 0.0 ? -df / pred : 0.0;
            if (rho < 0.25)
                mu = mu * PDNR_MU_STEP < PDNR_MU_MAX ? mu * PDNR_MU_STEP : PDNR_MU_MAX;
            else if (rho > 0.75)
                mu = mu / PDNR_MU_STEP > PDNR_MU_MIN ? mu / PDNR_MU_STEP : PDNR_MU_MIN;
        } else {
            for (int r = 0; r < R; ++r) delta[r] = -b[r] * g[r];
            mu = mu * PDNR_MU_STEP < PDNR_MU_MAX ? mu * PDNR_MU_STEP : PDNR_MU_MAX;
        }
        /* 7. step */
        for (int r = 0; r < R; ++r) b[r] += delta[r];
        ++steps;
    }
    *steps_out = steps;
    *viol_out = viol;
    if (phi_out)
        for (int r = 0; r < R; ++r) phi_out[r] = phi[r];
}

enum { ROWS_PQNR = 0, ROWS_PDNR = 1 };

/* Row-subproblem inner iterations of one mode (PQNR or PDNR), row by row
 * (rows are independent). B in/out (I_n x R). Outputs: the largest number of
 * steps any row took (n_updates), the sum of steps over rows (row_steps), the
 * largest last violation over rows (last_viol) and per-row steps
 * (row_steps_out, may be NULL). With row_mask only those rows are solved.
 * R <= 256. */
static int rows_inner(int method, int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                      const double* vals, int mode, int R, double* B, const double* const* A, int lmax,
                      double tau, double eps, const uint8_t* row_mask, int* n_updates, int64_t* row_steps,
                      double* last_viol, int* row_steps_out, double* Phi_last)
{
    if (check_args(nmodes, dims, nnz, idx, vals, R) || mode < 0 || mode >= nmodes || lmax < 1 ||
        R > 256 || !B)
        return -1;
    const int64_t In = dims[mode];
    /* rows' nonzero lists by counting sort (input order inside a row) */
    int64_t* start = (int64_t*)calloc((size_t)In + 1, sizeof(int64_t));
    int64_t* order = (int64_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
    if (!start || !order) { free(start); free(order); return -2; }
    for (int64_t k = 0; k < nnz; ++k) ++start[idx[(int64_t)mode * nnz + k] + 1];
    for (int64_t i = 0; i < In; ++i) start[i + 1] += start[i];
    {
        int64_t* fill = (int64_t*)malloc((size_t)In * sizeof(int64_t));
        if (!fill) { free(start); free(order); return -2; }
        for (int64_t i = 0; i < In; ++i) fill[i] = start[i];
        for (int64_t k = 0; k < nnz; ++k) order[fill[idx[(int64_t)mode * nnz + k]]++] = k;
        free(fill);
    }
    int64_t maxrow = 0;
    for (int64_t i = 0; i < In; ++i)
        if (start[i + 1] - start[i] > maxrow) maxrow = start[i + 1] - start[i];
    double* xs = (double*)malloc((size_t)(maxrow > 0 ? maxrow : 1) * sizeof(double));
    double* pis = (double*)malloc((size_t)(maxrow > 0 ? maxrow : 1) * R * sizeof(double));
    double* work = (double*)malloc((size_t)4 * R * R * sizeof(double)); /* PDNR matrices */
    if (!xs || !pis || !work) { free(start); free(order); free(xs); free(pis); free(work); return -2; }
    int maxsteps = 0;
    int64_t total = 0;
    double vmax = 0.0;
    for (int64_t i = 0; i < In; ++i) {
        if (row_mask && !row_mask[i]) continue;
        const int64_t nrow = start[i + 1] - start[i];
        for (int64_t j = 0; j < nrow; ++j) {
            const int64_t k = order[start[i] + j];
            xs[j] = vals[k];
            double* pi = pis + j * R;
            for (int r = 0; r < R; ++r) pi[r] = 1.0;
            for (int m = 0; m < nmodes; ++m) {
                if (m == mode) continue;
                const double* row = A[m] + (int64_t)idx[(int64_t)m * nnz + k] * R;
                for (int r = 0; r < R; ++r) pi[r] *= row[r];
            }
        }
        int st = 0;
        double v = 0.0;
        if (method == ROWS_PDNR)
            pdnr_row(R, nrow, xs, pis, B + i * R, lmax, tau, eps, &st, &v, Phi_last ? Phi_last + i * R : NULL,
                     work);
        else
            pqnr_row(R, nrow, xs, pis, B + i * R, lmax, tau, eps, &st, &v, Phi_last ? Phi_last + i * R : NULL);
        if (row_steps_out) row_steps_out[i] = st;
        if (st > maxsteps) maxsteps = st;
        total += st;
        if (v > vmax) vmax = v;
    }
    if (n_updates) *n_updates = maxsteps;
    if (row_steps) *row_steps = total;
    if (last_viol) *last_viol = vmax;
    free(start); free(order); free(xs); free(pis); free(work);
    return 0;
}

int oracle_pqnr_inner_rows(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                           const double* vals, int mode, int R, double* B,
                           const double* const* A, int lmax, double tau, double eps,
                           const uint8_t* row_mask, int* n_updates, int64_t* row_steps,
                           double* last_viol, int* row_steps_out, double* Phi_last)
{
    return rows_inner(ROWS_PQNR, nmodes, dims, nnz, idx, vals, mode, R, B, A, lmax, tau, eps, row_mask,
                      n_updates, row_steps, last_viol, row_steps_out, Phi_last);
}

int oracle_pdnr_inner_rows(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                           const double* vals, int mode, int R, double* B,
                           const double* const* A, int lmax, double tau, double eps,
                           const uint8_t* row_mask, int* n_updates, int64_t* row_steps,
                           double* last_viol, int* row_steps_out, double* Phi_last)
{
    return rows_inner(ROWS_PDNR, nmodes, dims, nnz, idx, vals, mode, R, B, A, lmax, tau, eps, row_mask,
                      n_updates, row_steps, last_viol, row_steps_out, Phi_last);
}

/* CP-APR with row-subproblem solves (PQNR or PDNR): the outer loop of
 * Algorithm 1 (S shift included, from the last Phi of each mode) with the MU
 * inner loop replaced by the row solves. lam and A[m] in/out. */
static int rows_solve(int method, int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                      const double* vals, int R, double* lam, double* const* A, int kmax, int lmax,
                      double tau, double eps, double kappa, double kappa_tol, int* outer_iters,
                      int64_t* row_steps, int* converged, double* kkt)
{
    if (check_args(nmodes, dims, nnz, idx, vals, R) || kmax < 1 || lmax < 1 || !lam || !A || R > 256)
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
    int64_t total = 0;
    double kkt_sweep = 0.0;
    for (k = 1; k <= kmax; ++k) {
        int any_update = 0;
        kkt_sweep = 0.0;
        for (int n = 0; n < nmodes; ++n) {
            const int64_t In = dims[n];
            double* An = A[n];
            if (k > 1) /* S, as in Algorithm 1 */
                for (int64_t e = 0; e < In * R; ++e)
                    if (An[e] < kappa_tol && phi_prev[n][e] > 1.0) An[e] += kappa;
            for (int64_t i = 0; i < In; ++i)
                for (int r = 0; r < R; ++r) B[i * R + r] = An[i * R + r] * lam[r];
            int upd = 0;
            int64_t st = 0;
            double v = 0.0;
            rc = rows_inner(method, nmodes, dims, nnz, idx, vals, n, R, B, (const double* const*)A, lmax,
                            tau, eps, NULL, &upd, &st, &v, NULL, phi_prev[n]);
            if (rc) goto done;
            if (upd > 0) any_update = 1;
            total += st;
            if (v > kkt_sweep) kkt_sweep = v;
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
    if (row_steps) *row_steps = total;
    if (converged) *converged = conv;
    if (kkt) *kkt = kkt_sweep;
    for (int m = 0; m < nmodes; ++m) free(phi_prev[m]);
    free(phi_prev);
    free(B);
    return rc;
}

int oracle_pqnr_solve(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                      const double* vals, int R, double* lam, double* const* A, int kmax, int lmax,
                      double tau, double eps, double kappa, double kappa_tol, int* outer_iters,
                      int64_t* row_steps, int* converged, double* kkt)
{
    return rows_solve(ROWS_PQNR, nmodes, dims, nnz, idx, vals, R, lam, A, kmax, lmax, tau, eps, kappa,
                      kappa_tol, outer_iters, row_steps, converged, kkt);
}

int oracle_pdnr_solve(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                      const double* vals, int R, double* lam, double* const* A, int kmax, int lmax,
                      double tau, double eps, double kappa, double kappa_tol, int* outer_iters,
                      int64_t* row_steps, int* converged, double* kkt)
{
    return rows_solve(ROWS_PDNR, nmodes, dims, nnz, idx, vals, R, lam, A, kmax, lmax, tau, eps, kappa,
                      kappa_tol, outer_iters, row_steps, converged, kkt);
}
