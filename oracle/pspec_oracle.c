/*
 * FP64 CPU oracle for the graph p-Laplacian hot path of p-spectral clustering on the
 * Grassmann manifold (Pasadakis, Schenk, Vlacic, Yzelman, "Nonlinear spectral clustering
 * with C++ GraphBLAS").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity reference for the HIP library.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header or constant with the HIP path, and the HIP path must never call it.
 *
 * Plain loops, IEEE double, libm pow(), rows in ascending order.  OpenMP only runs
 * independent per-row work in parallel; every sum over rows is taken afterwards, sequentially,
 * in ascending row order, in long double.
 *
 * Notation (Section 2, Eq. (1) and the definitions that follow it):
 *   graph: symmetric CSR (rowptr[n+1], col[nnz], w[nnz]) storing both directions of every edge;
 *   U: n x k, row-major with leading dimension ldu; column l is the vector u^l;
 *   F_p(U) = sum_l sum_{i,j} w_ij |u_i^l - u_j^l|^p / (2 ||u^l||_p^p)            (Eq. (1))
 *   (Delta_p u)_i = sum_j w_ij phi_p(u_i - u_j),  phi_p(x) = |x|^(p-1) sign(x)    (Section 2)
 *   ||u||_p^p = sum_i |u_i|^p                                                     (Section 2)
 *
 * The gradient and the Hessian-vector product are not printed in the paper; they are the
 * calculus of Eq. (1), written out once here (column l, u = u^l, N = numerator, D = ||u||_p^p,
 * F_l = N / D):
 *   dN/du_i = p (Delta_p u)_i            (needs w symmetric and phi_p odd)
 *   dD/du_i = p phi_p(u_i)
 *   g_i     = (p/D) [ (Delta_p u)_i - F_l phi_p(u_i) ]
 *   (H v)_i = (p/D) [ (p-1) sum_j w_ij psi(u_i-u_j) (v_i - v_j)
 *                     - F_l (p-1) psi(u_i) v_i - g_i (phi^T v) - phi_p(u_i) (g^T v) ]
 * where psi(x) = max(|x|, eps)^(p-2) is the derivative |x|^(p-2) of phi_p / (p-1), with its
 * singularity at x = 0 removed by the caller's eps (the paper is silent there).  Algorithm 1
 * applies the same operator per column as diag(H^l) eta - (diag(H^l) - H^l) eta.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* phi_p(x) = |x|^(p-1) sign(x), with sign(0) = 0 (Section 2). */
static double phi_p(double x, double p)
{
    if (x == 0.0) return 0.0;
    double m = pow(fabs(x), p - 1.0);
    return x > 0.0 ? m : -m;
}

/* |x|^p, with 0^p = 0 for p > 1. */
static double abs_pow(double x, double p)
{
    if (x == 0.0) return 0.0;
    return pow(fabs(x), p);
}

/* psi(x) = max(|x|, eps)^(p-2): phi_p'(x) / (p-1) away from 0, capped at eps^(p-2) near 0. */
static double psi_eps(double x, double p, double eps)
{
    double a = fabs(x);
    if (a < eps) a = eps;
    return pow(a, p - 2.0);
}

/*
 * Per-column numerator N_l = 1/2 sum_i sum_{j in row i} w_ij |u_i - u_j|^p and denominator
 * D_l = sum_i |u_i|^p; F_l = N_l / D_l; *F = sum_l F_l (Eq. (1)).  Any of the outputs may be NULL.
 */
void oracle_objective(int64_t n, const int64_t *rowptr, const int32_t *col, const double *w,
                      int k, const double *U, int64_t ldu, double p,
                      double *Ncol, double *Dcol, double *Fcol, double *F)
{
    double *rowN = (double *)malloc(sizeof(double) * (size_t)n * (size_t)k);
    int64_t i;
#pragma omp parallel for schedule(dynamic, 512)
    for (i = 0; i < n; ++i) {
        for (int l = 0; l < k; ++l) {
            long double s = 0.0L;
            double ui = U[i * ldu + l];
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                double uj = U[(int64_t)col[e] * ldu + l];
                s += (long double)(w[e] * abs_pow(ui - uj, p));
            }
            rowN[i * k + l] = (double)s;
        }
    }
    long double Ftot = 0.0L;
    for (int l = 0; l < k; ++l) {
        long double N = 0.0L, D = 0.0L;
        for (i = 0; i < n; ++i) {
            N += (long double)rowN[i * k + l];
            D += (long double)abs_pow(U[i * ldu + l], p);
        }
        N *= 0.5L;
        double Fl = (double)(N / D);
        if (Ncol) Ncol[l] = (double)N;
        if (Dcol) Dcol[l] = (double)D;
        if (Fcol) Fcol[l] = Fl;
        Ftot += (long double)Fl;
    }
    if (F) *F = (double)Ftot;
    free(rowN);
}

/* L = Delta_p U, column by column: L[i*k + l] = sum_{j in row i} w_ij phi_p(u_i^l - u_j^l). */
void oracle_plap(int64_t n, const int64_t *rowptr, const int32_t *col, const double *w,
                 int k, const double *U, int64_t ldu, double p, double *L)
{
    int64_t i;
#pragma omp parallel for schedule(dynamic, 512)
    for (i = 0; i < n; ++i) {
        for (int l = 0; l < k; ++l) {
            long double s = 0.0L;
            double ui = U[i * ldu + l];
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                double uj = U[(int64_t)col[e] * ldu + l];
                s += (long double)(w[e] * phi_p(ui - uj, p));
            }
            L[i * k + l] = (double)s;
        }
    }
}

/*
 * Euclidean gradient of F_p (the EucGrad callback of Section 2):
 * G[i*k + l] = (p / D_l) (L_il - F_l phi_p(u_il)).  Fcol (k values) may be NULL.
 */
void oracle_grad(int64_t n, const int64_t *rowptr, const int32_t *col, const double *w,
                 int k, const double *U, int64_t ldu, double p, double *G, double *Fcol)
{
    double *D = (double *)malloc(sizeof(double) * (size_t)k);
    double *Fl = (double *)malloc(sizeof(double) * (size_t)k);
    oracle_objective(n, rowptr, col, w, k, U, ldu, p, NULL, D, Fl, NULL);
    oracle_plap(n, rowptr, col, w, k, U, ldu, p, G);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        for (int l = 0; l < k; ++l) {
            double Lil = G[i * k + l];
            G[i * k + l] = (p / D[l]) * (Lil - Fl[l] * phi_p(U[i * ldu + l], p));
        }
    }
    if (Fcol)
        for (int l = 0; l < k; ++l) Fcol[l] = Fl[l];
    free(D);
    free(Fl);
}

/*
 * Hessian-vector product of F_p (the EucHessianEta callback of Section 2 / Algorithm 1),
 * exact, per column, with psi regularised by eps as documented at the top of this file.
 * HV[i*k + l] = (H^l v^l)_i.  G (n*k, may be NULL) receives the gradient, Fcol (k, may be NULL)
 * the per-column objective values.
 */
void oracle_hvp(int64_t n, const int64_t *rowptr, const int32_t *col, const double *w,
                int k, const double *U, int64_t ldu, const double *V, int64_t ldv,
                double p, double eps, double *HV, double *G, double *Fcol)
{
    double *g = (double *)malloc(sizeof(double) * (size_t)n * (size_t)k);
    double *D = (double *)malloc(sizeof(double) * (size_t)k);
    double *Fl = (double *)malloc(sizeof(double) * (size_t)k);
    double *a = (double *)malloc(sizeof(double) * (size_t)k);
    double *b = (double *)malloc(sizeof(double) * (size_t)k);
    oracle_objective(n, rowptr, col, w, k, U, ldu, p, NULL, D, Fl, NULL);
    oracle_grad(n, rowptr, col, w, k, U, ldu, p, g, NULL);

    /* a_l = phi_p(u^l)^T v^l and b_l = (g^l)^T v^l: the two inner products of the rank-2 part. */
    for (int l = 0; l < k; ++l) {
        long double sa = 0.0L, sb = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            double vi = V[i * ldv + l];
            sa += (long double)(phi_p(U[i * ldu + l], p) * vi);
            sb += (long double)(g[i * k + l] * vi);
        }
        a[l] = (double)sa;
        b[l] = (double)sb;
    }

    int64_t i;
#pragma omp parallel for schedule(dynamic, 512)
    for (i = 0; i < n; ++i) {
        for (int l = 0; l < k; ++l) {
            double ui = U[i * ldu + l], vi = V[i * ldv + l];
            long double s = 0.0L;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                int64_t j = col[e];
                double x = ui - U[j * ldu + l];
                s += (long double)(w[e] * psi_eps(x, p, eps) * (vi - V[j * ldv + l]));
            }
            double JL = (p - 1.0) * (double)s;
            double diag = Fl[l] * (p - 1.0) * psi_eps(ui, p, eps) * vi;
            double rank2 = g[i * k + l] * a[l] + phi_p(ui, p) * b[l];
            HV[i * k + l] = (p / D[l]) * (JL - diag - rank2);
        }
    }
    if (G)
        for (int64_t q = 0; q < n * (int64_t)k; ++q) G[q] = g[q];
    if (Fcol)
        for (int l = 0; l < k; ++l) Fcol[l] = Fl[l];
    free(g);
    free(D);
    free(Fl);
    free(a);
    free(b);
}

/* The sparse part of the Hessian applied to V (the exact operator of oracle_hvp without its rank-2
 * term): HV = (p/D) (J_L v - F J_phi v), J_L v = (p-1) sum_j w psi(u_i - u_j)(v_i - v_j),
 * J_phi v = (p-1) psi(u_i) v_i, the derivatives of the p-Laplacian and of phi_p along v. */
void oracle_hvp_sparse(int64_t n, const int64_t *rowptr, const int32_t *col, const double *w,
                       int k, const double *U, int64_t ldu, const double *V, int64_t ldv,
                       double p, double eps, double *HV)
{
    double *D = (double *)malloc(sizeof(double) * (size_t)k);
    double *Fl = (double *)malloc(sizeof(double) * (size_t)k);
    oracle_objective(n, rowptr, col, w, k, U, ldu, p, NULL, D, Fl, NULL);
    int64_t i;
#pragma omp parallel for schedule(dynamic, 512)
    for (i = 0; i < n; ++i) {
        for (int l = 0; l < k; ++l) {
            double ui = U[i * ldu + l], vi = V[i * ldv + l];
            long double s = 0.0L;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                int64_t j = col[e];
                s += (long double)(w[e] * psi_eps(ui - U[j * ldu + l], p, eps) * (vi - V[j * ldv + l]));
            }
            double JL = (p - 1.0) * (double)s;
            double Jphi = (p - 1.0) * psi_eps(ui, p, eps) * vi;
            HV[i * k + l] = (p / D[l]) * (JL - Fl[l] * Jphi);
        }
    }
    free(D);
    free(Fl);
}

/*
 * Forward-error scales of the gradient and the Hessian-vector product (for parity tolerances, not a
 * result of the method).  Each entry of G and HV is a signed sum; its scale is the same sum taken
 * over absolute values, every term weighted by the conditioning of the power that forms it: an
 * absolute error d in log2|x| perturbs |x|^(p-2) = 2^((p-2) log2|x|) by the relative amount
 * |p-2| ln2 d, and log2|x| is known to a relative accuracy, so a power term carries the weight
 *   kappa(x) = 1 + |p - 2| |log2|x||  (phi_p, x != 0),   kappa_eps(x) = kappa(max(|x|, eps))  (psi).
 * With x = u_i - u_j, phi = phi_p, psi = psi_eps, D = D_l, F = F_l, g = the gradient (column l):
 *   SG_i = (p/D) [ sum_j w_ij |phi(x)| kappa(x) + F |phi(u_i)| kappa(u_i) ]
 *   SH_i = (p/D) [ (p-1) sum_j w_ij psi(x) |v_i - v_j| kappa_eps(x)
 *                  + F (p-1) psi(u_i) |v_i| kappa_eps(u_i) + SG_i |a| + |g_i| A + |phi(u_i)| B ]
 * where a = phi^T v, A = sum_i |phi(u_i) v_i| kappa(u_i) and B = sum_i SG_i |v_i| bound the errors
 * of the two inner products of the rank-2 part.  SHs (may be NULL) receives the scale of the sparse
 * part alone (the first line of SH_i: the Hessian without its rank-2 term).  An evaluation whose every elementary operation
 * has a relative error below r in any order agrees with the exact value to (c + m) r times the
 * scale, m being the longest sequential sum; SG_i >= |g_i| and SH_i >= |(Hv)_i| always.
 */
static double kappa(double x, double q) { return 1.0 + q * fabs(log2(fabs(x))); }
static double kappa_eps(double x, double q, double eps) { return 1.0 + q * fabs(log2(fabs(x) > eps ? fabs(x) : eps)); }

void oracle_error_scales(int64_t n, const int64_t *rowptr, const int32_t *col, const double *w,
                         int k, const double *U, int64_t ldu, const double *V, int64_t ldv,
                         double p, double eps, double *SG, double *SH, double *SHs)
{
    double *g = (double *)malloc(sizeof(double) * (size_t)n * (size_t)k);
    double *D = (double *)malloc(sizeof(double) * (size_t)k);
    double *Fl = (double *)malloc(sizeof(double) * (size_t)k);
    double *a = (double *)malloc(sizeof(double) * (size_t)k);
    double *A = (double *)malloc(sizeof(double) * (size_t)k);
    double *B = (double *)malloc(sizeof(double) * (size_t)k);
    const double q = fabs(p - 2.0);
    oracle_objective(n, rowptr, col, w, k, U, ldu, p, NULL, D, Fl, NULL);
    oracle_grad(n, rowptr, col, w, k, U, ldu, p, g, NULL);
    int64_t i;
#pragma omp parallel for schedule(dynamic, 512)
    for (i = 0; i < n; ++i) {
        for (int l = 0; l < k; ++l) {
            double ui = U[i * ldu + l], vi = V[i * ldv + l];
            long double sg = 0.0L, sh = 0.0L;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                int64_t j = col[e];
                double x = ui - U[j * ldu + l];
                if (x != 0.0) sg += (long double)(w[e] * fabs(phi_p(x, p)) * kappa(x, q));
                sh += (long double)(w[e] * psi_eps(x, p, eps) * fabs(vi - V[j * ldv + l]) * kappa_eps(x, q, eps));
            }
            double phi_i = ui != 0.0 ? fabs(phi_p(ui, p)) * kappa(ui, q) : 0.0;
            SG[i * k + l] = (p / D[l]) * ((double)sg + Fl[l] * phi_i);
            SH[i * k + l] = (double)sh * (p - 1.0) + Fl[l] * (p - 1.0) * psi_eps(ui, p, eps) * fabs(vi) *
                                                         kappa_eps(ui, q, eps);
        }
    }
    for (int l = 0; l < k; ++l) {
        long double sa = 0.0L, sA = 0.0L, sB = 0.0L;
        for (i = 0; i < n; ++i) {
            double ui = U[i * ldu + l], vi = V[i * ldv + l];
            sa += (long double)(phi_p(ui, p) * vi);
            if (ui != 0.0) sA += (long double)(fabs(phi_p(ui, p) * vi) * kappa(ui, q));
            sB += (long double)(SG[i * k + l] * fabs(vi));
        }
        a[l] = (double)sa;
        A[l] = (double)sA;
        B[l] = (double)sB;
    }
    if (SHs)
        for (int64_t q2 = 0; q2 < n * (int64_t)k; ++q2) SHs[q2] = (p / D[q2 % k]) * SH[q2];
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        for (int l = 0; l < k; ++l) {
            double ui = U[i * ldu + l];
            double rank2 = SG[i * k + l] * fabs(a[l]) + fabs(g[i * k + l]) * A[l] + fabs(phi_p(ui, p)) * B[l];
            SH[i * k + l] = (p / D[l]) * (SH[i * k + l] + rank2);
        }
    }
    free(g);
    free(D);
    free(Fl);
    free(a);
    free(A);
    free(B);
}

/* Threads of the parallel regions that follow (ignored without OpenMP; t < 1 is taken as 1). */
void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    omp_set_num_threads(t < 1 ? 1 : t);
#else
    (void)t;
#endif
}

/* Number of OpenMP threads a parallel region of this library uses (1 without OpenMP). */
int oracle_num_threads(void)
{
    int t = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
#endif
    return t;
}
