/* A plain C client of libpspec.so on the GPU: device memory from the HIP runtime (including the graph
 * handle's workspace, sized by pspec_graph_workspace_bytes), a graph handle,
 * F_p of Eq. (1) in FP64, checked against the C oracle (test infrastructure) on the same inputs.
 * No Python or torch.  Prints "ok" and the relative difference; tests/test_gpu_c_client.py runs it. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "pspec.h"

void oracle_objective(int64_t n, const int64_t *rowptr, const int32_t *col, const double *w, int k,
                      const double *U, int64_t ldu, double p, double *Ncol, double *Dcol, double *Fcol,
                      double *F);

#define CHECK_HIP(x)                                                     \
    do {                                                                 \
        hipError_t e_ = (x);                                             \
        if (e_ != hipSuccess) {                                          \
            printf("HIP error %d at %s\n", (int)e_, #x);                 \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(void) {
    /* a ring of n nodes with chords i <-> i + 7 (mod n): every row has 4 neighbours, ascending */
    const int64_t n = 5000;
    const int k = 3;
    const double p = 1.4;
    int64_t *rowptr = malloc(sizeof(int64_t) * (n + 1));
    int32_t *col = malloc(sizeof(int32_t) * 4 * n);
    double *w = malloc(sizeof(double) * 4 * n);
    double *U = malloc(sizeof(double) * n * k);
    rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t nb[4] = {(i + n - 7) % n, (i + n - 1) % n, (i + 1) % n, (i + 7) % n};
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b)
                if (nb[b] < nb[a]) {
                    int64_t t = nb[a];
                    nb[a] = nb[b];
                    nb[b] = t;
                }
        for (int a = 0; a < 4; ++a) {
            col[4 * i + a] = (int32_t)nb[a];
            const int64_t lo = i < nb[a] ? i : nb[a], hi = i < nb[a] ? nb[a] : i;
            w[4 * i + a] = 0.5 + (double)((lo * 131 + hi * 17) % 97) / 97.0; /* symmetric in (i, j) */
        }
        rowptr[i + 1] = 4 * (i + 1);
        for (int l = 0; l < k; ++l) U[i * k + l] = sin(0.001 * (double)(i + 1) * (double)(l + 2)) + 0.1 * l;
    }
    const int64_t nnz = rowptr[n];

    int64_t *d_rowptr;
    int32_t *d_col;
    double *d_w, *d_U, *d_Fcol, *d_F;
    CHECK_HIP(hipMalloc((void **)&d_rowptr, sizeof(int64_t) * (n + 1)));
    CHECK_HIP(hipMalloc((void **)&d_col, sizeof(int32_t) * nnz));
    CHECK_HIP(hipMalloc((void **)&d_w, sizeof(double) * nnz));
    CHECK_HIP(hipMalloc((void **)&d_U, sizeof(double) * n * k));
    CHECK_HIP(hipMalloc((void **)&d_Fcol, sizeof(double) * k));
    CHECK_HIP(hipMalloc((void **)&d_F, sizeof(double)));
    CHECK_HIP(hipMemcpy(d_rowptr, rowptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_col, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_w, w, sizeof(double) * nnz, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_U, U, sizeof(double) * n * k, hipMemcpyHostToDevice));

    /* the handle's schedule and scratch live in a workspace the caller allocates */
    const size_t ws_bytes = pspec_graph_workspace_bytes(n, nnz, k);
    void *d_ws = NULL;
    CHECK_HIP(hipMalloc(&d_ws, ws_bytes));
    pspec_graph g = NULL;
    pspec_status st = pspec_graph_create(n, nnz, d_rowptr, d_col, d_w, PSPEC_F64, k, d_ws, ws_bytes, NULL, &g);
    if (st != PSPEC_OK) {
        printf("graph_create: %d %s\n", (int)st, pspec_last_error());
        return 1;
    }
    st = pspec_objective(g, PSPEC_F64, k, d_U, k, p, d_Fcol, d_F, NULL);
    if (st != PSPEC_OK) {
        printf("objective: %d %s\n", (int)st, pspec_last_error());
        return 1;
    }
    double F = 0.0;
    CHECK_HIP(hipMemcpy(&F, d_F, sizeof(double), hipMemcpyDeviceToHost));

    double N[3], D[3], Fc[3], Fo = 0.0;
    oracle_objective(n, rowptr, col, w, k, U, k, p, N, D, Fc, &Fo);
    const double rel = fabs(F - Fo) / fabs(Fo);
    printf("F gpu %.17g oracle %.17g rel %.3g\n", F, Fo, rel);
    pspec_graph_destroy(g);
    CHECK_HIP(hipFree(d_ws));
    CHECK_HIP(hipFree(d_rowptr));
    CHECK_HIP(hipFree(d_col));
    CHECK_HIP(hipFree(d_w));
    CHECK_HIP(hipFree(d_U));
    CHECK_HIP(hipFree(d_Fcol));
    CHECK_HIP(hipFree(d_F));
    if (rel < 1e-12) printf("ok\n");
    return rel < 1e-12 ? 0 : 1;
}
