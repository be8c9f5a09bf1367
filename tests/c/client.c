/* A plain C client of libpspec.so: compiled with gcc against include/pspec.h, no Python or torch.
 * It calls the entry points that need no GPU (host-side argument checks, workspace sizes and the
 * host RCM relabelling) and prints what it finds; tests/test_c_client.py checks the output. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "pspec.h"

int main(void) {
    /* a 6-node path 0-1-2-3-4-5, numbered 3 0 5 1 4 2 along the path */
    const int64_t n = 6;
    const int order_along_path[6] = {3, 0, 5, 1, 4, 2};
    int64_t rowptr[7] = {0};
    int32_t col[10];
    int nbr[6][2], deg[6] = {0};
    for (int t = 0; t + 1 < 6; ++t) {
        const int a = order_along_path[t], b = order_along_path[t + 1];
        nbr[a][deg[a]++] = b;
        nbr[b][deg[b]++] = a;
    }
    int e = 0;
    for (int i = 0; i < 6; ++i) {
        if (deg[i] == 2 && nbr[i][0] > nbr[i][1]) {
            const int x = nbr[i][0];
            nbr[i][0] = nbr[i][1];
            nbr[i][1] = x;
        }
        for (int j = 0; j < deg[i]; ++j) col[e++] = nbr[i][j];
        rowptr[i + 1] = e;
    }
    int64_t perm[6];
    pspec_status st = pspec_rcm_order(n, rowptr, col, perm);
    if (st != PSPEC_OK) {
        printf("rcm_order failed: %d %s\n", (int)st, pspec_last_error());
        return 1;
    }
    int64_t bw = 0;
    for (int i = 0; i < 6; ++i)
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            const int64_t d = perm[i] - perm[col[q]];
            if ((d < 0 ? -d : d) > bw) bw = d < 0 ? -d : d;
        }
    printf("rcm bandwidth %lld\n", (long long)bw);

    /* host-side errors, no device memory touched */
    st = pspec_project(0, 4, PSPEC_F32, NULL, 4, NULL, 4, NULL, 0, NULL, NULL, 4, NULL, NULL, 0, NULL);
    printf("project n=0 -> %d (%s)\n", (int)st, pspec_last_error());
    st = pspec_kmeans_step(10, 40, PSPEC_F32, (void *)256, 40, 4, (const double *)512, NULL, NULL,
                           (double *)768, (void *)1024, (size_t)1 << 30, NULL);
    printf("kmeans d=40 -> %d (%s)\n", (int)st, pspec_last_error());
    pspec_graph g = NULL;
    st = pspec_graph_create(6, 10, (const int64_t *)256, (const int32_t *)512, (const void *)768, PSPEC_F32, 4,
                            NULL, 0, NULL, &g);
    printf("graph_create no workspace -> %d (%s)\n", (int)st, pspec_last_error());
    st = pspec_graph_create(6, 10, (const int64_t *)256, (const int32_t *)512, (const void *)768, PSPEC_F32, 4,
                            (void *)1024, 64, NULL, &g);
    printf("graph_create small workspace -> %d (%s)\n", (int)st, pspec_last_error());
    printf("graph workspace n=8000000 nnz=95998824 k=16: %zu bytes\n",
           pspec_graph_workspace_bytes(8000000, 95998824, 16));
    printf("graph workspace k=65: %zu bytes\n", pspec_graph_workspace_bytes(100, 100, 65));
    printf("dense workspace k=16: %zu bytes\n", pspec_dense_workspace_bytes(16));
    printf("kmeans workspace c=4 d=4: %zu bytes\n", pspec_kmeans_workspace_bytes(4, 4));
    return 0;
}
