// k-means (Lloyd) step on the rows of an n x d block: the discretisation that turns the rows of the
// minimiser U into cluster labels (Section 1; the paper names k-means but not its variant).
//
// One pass over the rows.  A thread owns a row: it computes the squared Euclidean distance to every
// centroid as sum_t (x_t - c_t)^2 in t order with no fused multiply-add, and keeps the first
// centroid of smallest distance, so labels and distances are a plain function of the inputs (no
// summation order to choose).  The per-cluster statistics (coordinate sums, count, distance sum) of
// each 64-row wave batch are reduced across the wave (DPP exchanges within 16-lane rows, then the
// four row sums; no LDS traffic) and accumulated, cluster j in lane j, in wave order; for at most
// four clusters of at most 8 columns every lane instead keeps its own rows' statistics in registers
// (in row order) and the wave reduces them once at the end.  The four waves of a workgroup are added
// in order into one partial per workgroup, and the kDenseBlocks partials are added by the fixed
// two-level tree of the dense kernels.  The statistics are therefore bit-reproducible from run to run.  The work is one read of
// the block (plus the optional label and distance writes): HBM bound for the d and c of clustering U.
#include "common.hpp"
#include "dense.hpp"

namespace pspec {
namespace {

constexpr int kKmMax = PSPEC_KMEANS_MAX;

// Squared distance from the row x (zero-padded to D) to the centroid cj (zero-padded to D), summed in
// coordinate order.  Contraction is off: e * e is rounded before it is added.  The padding adds exact
// zeros after the last real coordinate, which leaves the sum unchanged.
template <int D>
__device__ __forceinline__ double sqdist(const double (&x)[D], const double *cj) {
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const double e = x[t] - cj[t];
        s = s + e * e;
    }
    return s;
}

// Per-lane statistics are used when they fit in registers: at most kLocalC clusters of at most 8
// columns (the clustering of U for small k).
constexpr int kLocalC = 4;

template <typename T, int D, bool VEC, bool LOCAL>
__global__ __launch_bounds__(kBlock) void kmeans_partial(int64_t n, int d, const T *__restrict__ X, int64_t ldx,
                                                       int c, const double *__restrict__ C,
                                                       int32_t *__restrict__ labels, double *__restrict__ dist,
                                                       double *__restrict__ part) {
    constexpr int NW = kBlock / 64;
    constexpr int A = D + 2;  // accumulator slots: D coordinate sums, the count, the distance sum
    __shared__ double s_c[kKmMax][D];
    __shared__ double s_red[NW][kKmMax][A];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int e = tid; e < kKmMax * D; e += kBlock) {
        const int j = e / D, t = e % D;
        s_c[j][t] = (j < c && t < d) ? C[j * d + t] : 0.0;
    }
    __syncthreads();

    double acc[A];  // lane j < c: the statistics of cluster j over this wave's rows
#pragma unroll
    for (int t = 0; t < A; ++t) acc[t] = 0.0;
    // LOCAL: every lane's own statistics per cluster, reduced across the wave once at the end
    constexpr int LC = LOCAL ? kLocalC : 1;
    double la[LC][A];
#pragma unroll
    for (int j = 0; j < LC; ++j)
#pragma unroll
        for (int t = 0; t < A; ++t) la[j][t] = 0.0;

    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
        const int64_t i = base + tid;
        const bool valid = i < n;
        const int64_t row = valid ? i : n - 1;  // past-the-end lanes load the last row and own no cluster
        T xr[D];
        load_row<T, D, VEC>(X + row * ldx, d, xr);
        double x[D];
#pragma unroll
        for (int t = 0; t < D; ++t) x[t] = (double)xr[t];
        double best = sqdist<D>(x, s_c[0]);
        int lab = 0;
        for (int j = 1; j < c; ++j) {
            const double s = sqdist<D>(x, s_c[j]);
            if (s < best) {
                best = s;
                lab = j;
            }
        }
        if (valid) {
            if (labels) labels[i] = lab;
            if (dist) dist[i] = best;
        }
        if (!valid) lab = -1;
        if constexpr (LOCAL) {
#pragma unroll
            for (int j = 0; j < LC; ++j) {
                const bool mine = lab == j;
#pragma unroll
                for (int t = 0; t < D; ++t) la[j][t] += mine ? x[t] : 0.0;
                la[j][D] += mine ? 1.0 : 0.0;
                la[j][D + 1] += mine ? best : 0.0;
            }
            continue;
        }
        for (int j = 0; j < c; ++j) {
            const bool mine = lab == j;
            const uint64_t ball = __ballot(mine);
            if (ball == 0) continue;  // wave-uniform: no row of this batch is in cluster j
            const bool owner = lane == j;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                if (t < d) {
                    const double tot = wave_sum_f64(mine ? x[t] : 0.0);
                    acc[t] += owner ? tot : 0.0;
                }
            }
            acc[D] += owner ? (double)__popcll(ball) : 0.0;
            const double tot = wave_sum_f64(mine ? best : 0.0);
            acc[D + 1] += owner ? tot : 0.0;
        }
    }

    if constexpr (LOCAL) {
#pragma unroll
        for (int j = 0; j < LC; ++j)
#pragma unroll
            for (int t = 0; t < A; ++t) {
                const double tot = wave_sum_f64(la[j][t]);
                if (lane == 0 && j < c) s_red[w][j][t] = tot;
            }
    } else if (lane < c) {
#pragma unroll
        for (int t = 0; t < A; ++t) s_red[w][lane][t] = acc[t];
    }
    __syncthreads();
    // partial layout: part[j * (d + 2) + t], t < d the coordinate sums, t = d the count, t = d + 1
    // the distance sum
    const int P = c * (d + 2);
    for (int e = tid; e < P; e += kBlock) {
        const int j = e / (d + 2), t = e % (d + 2);
        const int slot = t < d ? t : D + (t - d);
        double v = s_red[0][j][slot];
#pragma unroll
        for (int q = 1; q < NW; ++q) v += s_red[q][j][slot];
        part[(int64_t)blockIdx.x * P + e] = v;
    }
}

template <typename T, int D>
pspec_status kmeans_impl(int64_t n, int d, const T *X, int64_t ldx, int c, const double *C, int32_t *labels,
                         double *dist, double *stats, double *ws, hipStream_t s) {
    const bool vec = rows_vectorisable<T, D>(d, {{X, ldx}});
    if constexpr (D <= 8) {
        if (c <= kLocalC) {
            if (vec)
                kmeans_partial<T, D, true, true><<<kDenseBlocks, kBlock, 0, s>>>(n, d, X, ldx, c, C, labels, dist, ws);
            else
                kmeans_partial<T, D, false, true><<<kDenseBlocks, kBlock, 0, s>>>(n, d, X, ldx, c, C, labels, dist, ws);
            const int P = c * (d + 2);
            sum_partials(ws, P, ws + (size_t)kDenseBlocks * P, stats, nullptr, s);
            PSPEC_HIP(hipGetLastError());
            return PSPEC_OK;
        }
    }
    if (vec)
        kmeans_partial<T, D, true, false><<<kDenseBlocks, kBlock, 0, s>>>(n, d, X, ldx, c, C, labels, dist, ws);
    else
        kmeans_partial<T, D, false, false><<<kDenseBlocks, kBlock, 0, s>>>(n, d, X, ldx, c, C, labels, dist, ws);
    const int P = c * (d + 2);
    sum_partials(ws, P, ws + (size_t)kDenseBlocks * P, stats, nullptr, s);
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

size_t kmeans_ws_doubles(int c, int d) {
    return (size_t)(kDenseBlocks + kDenseBlocks / kTreeFan) * (size_t)c * (size_t)(d + 2);
}

}  // namespace
}  // namespace pspec

using namespace pspec;

extern "C" size_t pspec_kmeans_workspace_bytes(int c, int d) {
    if (c < 1) c = 1;
    if (c > kKmMax) c = kKmMax;
    if (d < 1) d = 1;
    if (d > kKmMax) d = kKmMax;
    return kmeans_ws_doubles(c, d) * sizeof(double);
}

extern "C" pspec_status pspec_kmeans_step(int64_t n, int d, pspec_dtype dt, const void *X, int64_t ldx, int c,
                                          const double *C, int32_t *labels, double *dist, double *stats, void *ws,
                                          size_t ws_bytes, pspec_stream stream) {
    clear_error();
    PSPEC_ARG(n >= 0, "kmeans_step: n = %lld < 0", (long long)n);
    PSPEC_ARG(d >= 1, "kmeans_step: d = %d < 1", d);
    PSPEC_UNSUP(d <= kKmMax, "kmeans_step: d = %d > %d", d, kKmMax);
    PSPEC_ARG(c >= 1, "kmeans_step: c = %d < 1", c);
    PSPEC_UNSUP(c <= kKmMax, "kmeans_step: c = %d > %d", c, kKmMax);
    PSPEC_ARG(dt == PSPEC_F32 || dt == PSPEC_F64, "kmeans_step: bad dtype %d", (int)dt);
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    PSPEC_ARG(n == 0 || X != nullptr, "kmeans_step: X is NULL");
    PSPEC_ARG(ldx >= d, "kmeans_step: ldx = %lld < d", (long long)ldx);
    PSPEC_ARG(((uintptr_t)X % es) == 0, "kmeans_step: X is not aligned to its element size");
    PSPEC_ARG(C != nullptr, "kmeans_step: C is NULL");
    PSPEC_ARG(stats != nullptr, "kmeans_step: stats is NULL");
    PSPEC_ARG(((uintptr_t)C % 8) == 0 && ((uintptr_t)stats % 8) == 0 && ((uintptr_t)dist % 8) == 0 &&
                  ((uintptr_t)labels % 4) == 0,
              "kmeans_step: C, stats, dist or labels is misaligned");
    PSPEC_ARG(ws != nullptr, "kmeans_step: workspace is NULL");
    PSPEC_ARG(((uintptr_t)ws % 256) == 0, "kmeans_step: workspace must be 256-byte aligned");
    if (ws_bytes < kmeans_ws_doubles(c, d) * sizeof(double)) {
        set_error("kmeans_step: workspace of %zu bytes < %zu needed", ws_bytes, kmeans_ws_doubles(c, d) * sizeof(double));
        return PSPEC_ERR_WORKSPACE;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *w = static_cast<double *>(ws);
#define PSPEC_KM(T)                                                                                        \
    switch (pad_k(d)) {                                                                                    \
        case 4: return kmeans_impl<T, 4>(n, d, (const T *)X, ldx, c, C, labels, dist, stats, w, s);        \
        case 8: return kmeans_impl<T, 8>(n, d, (const T *)X, ldx, c, C, labels, dist, stats, w, s);        \
        case 16: return kmeans_impl<T, 16>(n, d, (const T *)X, ldx, c, C, labels, dist, stats, w, s);      \
        default: return kmeans_impl<T, 32>(n, d, (const T *)X, ldx, c, C, labels, dist, stats, w, s);     \
    }
    if (dt == PSPEC_F32) PSPEC_KM(float)
    PSPEC_KM(double)
#undef PSPEC_KM
}
