// k-means (Lloyd) step on the rows of an n x d block: the discretisation that turns the rows of the
// minimiser U into cluster labels (Section 1; the paper names k-means but not its variant).
//
// One pass over the rows.  A thread owns a row: it computes the squared Euclidean distance to every
// centroid as sum_t (x_t - c_t)^2 in t order with no fused multiply-add, and keeps the first
// centroid of smallest distance, so labels and distances are a plain function of the inputs (no
// summation order to choose).  The per-cluster statistics (coordinate sums, count, distance sum)
// are gathered per wave in one of two ways (see Stat below): in each lane's registers (at most 4
// clusters of at most 8 columns), or as one-hot products on the FP64 matrix cores (the rows staged
// as [x | 1 | dist] in LDS, in two halves above 16 columns).  Both add in a fixed order;
// the four waves of a workgroup are added in order into one partial per workgroup, and the
// kDenseBlocks partials by the fixed two-level tree of the dense kernels, so the statistics are
// bit-reproducible from run to run.  The work is one read of the block plus the optional label and
// distance writes.
#include <type_traits>

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

// How the per-cluster statistics of a wave's rows are gathered:
//   kStatLane  every lane keeps its own rows' statistics (at most kLocalC clusters of at most 8
//              columns: the clustering of U for small k), one wave reduction at the end;
//   kStatMfma  otherwise: per 64-row batch the wave stages its rows as [x | 1 | dist] in LDS (all
//              64 at once up to 16 columns, in two halves of 32 above) and adds
//              indicator(cluster)^T rows on the FP64 matrix cores, one MFMA step per 4 rows.
// The staging area shares its LDS with the per-wave results that are added at the end.
constexpr int kLocalC = 4;
enum Stat { kStatLane = 1, kStatMfma = 2 };

template <typename T, int D, bool VEC, int STAT>
__global__ __launch_bounds__(kBlock) void kmeans_partial(int64_t n, int d, const T *__restrict__ X,
                                                       int64_t ldx, int c, const double *__restrict__ C,
                                                       int32_t *__restrict__ labels,
                                                       double *__restrict__ dist, double *__restrict__ part) {
    constexpr int NW = kBlock / 64;
    constexpr int A = D + 2;  // accumulator slots: D coordinate sums, the count, the distance sum
    constexpr bool LOCAL = STAT == kStatLane, MF = STAT == kStatMfma;
    constexpr int RB = MF ? (D > 16 ? 32 : 64) : 1;  // rows of a batch staged at a time
    constexpr int RED = NW * kKmMax * A, STG = MF ? NW * RB * A : 0;
    __shared__ double s_c[kKmMax][D];
    __shared__ double s_big[RED > STG ? RED : STG];
    auto s_red = reinterpret_cast<double (*)[kKmMax][A]>(s_big);  // [wave][cluster][slot], at the end
    auto s_v = reinterpret_cast<double (*)[RB][A]>(s_big);         // [wave][row][column], MF batches
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int e = tid; e < kKmMax * D; e += kBlock) {
        const int j = e / D, t = e % D;
        s_c[j][t] = (j < c && t < d) ? C[j * d + t] : 0.0;
    }
    __syncthreads();

    // LOCAL: every lane's own statistics per cluster, reduced across the wave once at the end
    constexpr int LC = LOCAL ? kLocalC : 1;
    // MF: the wave's staged rows, their labels and the 16 x 16 tiles (clusters x columns)
    constexpr int CTT = MF ? (A + 15) / 16 : 1;
    constexpr int CTC = MF ? kKmMax / 16 : 1;
    __shared__ int s_l[MF ? kBlock / 64 : 1][MF ? 64 : 1];
    dbl4 mf[CTC][CTT];
#pragma unroll
    for (int ct = 0; ct < CTC; ++ct)
#pragma unroll
        for (int tt = 0; tt < CTT; ++tt) mf[ct][tt] = dbl4{0.0, 0.0, 0.0, 0.0};
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
        if constexpr (MF) {
            s_l[w][lane] = lab;
            const int q = lane >> 4, cc = lane & 15;
            for (int h = 0; h < 64 / RB; ++h) {
                if (lane / RB == h) {
                    // this lane's row: columns < d the coordinates, d the count 1, d + 1 the distance
                    const int r = lane - h * RB;
                    s_v[w][r][D] = 0.0;
                    s_v[w][r][D + 1] = 0.0;
#pragma unroll
                    for (int t = 0; t < D; ++t) s_v[w][r][t] = x[t];
                    s_v[w][r][d] = 1.0;
                    s_v[w][r][d + 1] = best;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // lane (q, cc) supplies A[cc][q] = [label of staged row 4 st + q is 16 ct + cc] and
                // B[q][cc] = column 16 tt + cc of that row
                for (int st = 0; st < RB / 4; ++st) {
                    const int rr = 4 * st + q;
                    const int lj = s_l[w][h * RB + rr];
                    double bv[CTT];
#pragma unroll
                    for (int tt = 0; tt < CTT; ++tt) {
                        const int col = 16 * tt + cc;
                        const double v = s_v[w][rr][col < A ? col : A - 1];
                        bv[tt] = col < A ? v : 0.0;
                    }
#pragma unroll
                    for (int ct = 0; ct < CTC; ++ct) {
                        if (16 * ct >= c) continue;  // wave-uniform
                        const double av = lj == 16 * ct + cc ? 1.0 : 0.0;
#pragma unroll
                        for (int tt = 0; tt < CTT; ++tt) mf[ct][tt] = mfma_f64(av, bv[tt], mf[ct][tt]);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }

    if constexpr (MF) {
        __syncthreads();  // every wave is done with its staging area, which s_red reuses
        // element i of lane (q, cc) in tile (ct, tt): cluster 16 ct + 4 i + q, column 16 tt + cc
        const int q = lane >> 4, cc = lane & 15;
#pragma unroll
        for (int ct = 0; ct < CTC; ++ct)
#pragma unroll
            for (int tt = 0; tt < CTT; ++tt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = 16 * ct + 4 * i + q, col = 16 * tt + cc;
                    if (j < c && col < d + 2)
                        s_red[w][j][col < d ? col : D + (col - d)] = mf[ct][tt][i];
                }
    } else {
#pragma unroll
        for (int j = 0; j < LC; ++j)
#pragma unroll
            for (int t = 0; t < A; ++t) {
                const double tot = wave_sum_f64(la[j][t]);
                if (lane == 0 && j < c) s_red[w][j][t] = tot;
            }
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
    auto launch = [&](auto stat) {
        constexpr int ST = decltype(stat)::value;
        if (vec)
            kmeans_partial<T, D, true, ST><<<kDenseBlocks, kBlock, 0, s>>>(n, d, X, ldx, c, C, labels, dist, ws);
        else
            kmeans_partial<T, D, false, ST><<<kDenseBlocks, kBlock, 0, s>>>(n, d, X, ldx, c, C, labels, dist, ws);
    };
    if (D <= 8 && c <= kLocalC)
        launch(std::integral_constant<int, D <= 8 ? kStatLane : kStatMfma>{});
    else
        launch(std::integral_constant<int, kStatMfma>{});
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
        set_error("kmeans_step: workspace of %zu bytes < %zu needed", ws_bytes,
                  kmeans_ws_doubles(c, d) * sizeof(double));
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
