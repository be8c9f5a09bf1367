// Shared pieces of the dense n x k kernels: 16-byte row access, the tile geometry and the FP64
// accumulation order of tall-skinny Gram matrices, and the fixed-order reduction of per-block
// partials.  The Gram accumulation is used both by the stand-alone Gram kernel and by the fused
// epilogue of the Riemannian Hessian-vector product, so the two produce identical bits.
#pragma once

#include <initializer_list>
#include <utility>

#include "common.hpp"

namespace pspec {
namespace {


constexpr int kDenseBlocks = 1024;  // first-level partials of Gram matrices and dot products
constexpr int kTreeFan = 32;         // partials summed per thread at each further level

// Workspace (doubles) of the dense operations: room for two k x k matrices at every level, i.e.
// level-1 partials [kDenseBlocks][2][k*k], level-2 partials [kDenseBlocks / kTreeFan][2][k*k] and
// two reduced matrices (M, R^-1 or U^T G, U^T HV), plus slack.
inline size_t dense_ws_doubles(int k) {
    const size_t kk2 = 2 * (size_t)k * k;
    return kDenseBlocks * kk2 + (kDenseBlocks / kTreeFan) * kk2 + kk2 + 64;
}

// 16-byte vectors of each element type.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int W = 4;
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int W = 2;
};

// True when every (pointer, leading dimension) pair allows 16-byte row accesses and k fills the
// padded width K, so rows move as whole vectors with no column guard.
template <typename T, int K>
bool rows_vectorisable(int k, std::initializer_list<std::pair<const void *, int64_t>> blocks) {
    if (k != K) return false;
    for (const auto &b : blocks)
        if (b.first && (((uintptr_t)b.first % 16) != 0 || ((size_t)b.second * sizeof(T)) % 16 != 0)) return false;
    return true;
}

// One row of K values: VEC rows are whole 16-byte vectors; otherwise element by element, with the
// columns >= k read as zero and never stored.
template <typename T, int K, bool VEC>
__device__ __forceinline__ void load_row(const T *p, int k, T (&r)[K]) {
    if constexpr (VEC) {
        using V = typename Vec16<T>::type;
        constexpr int W = Vec16<T>::W;
#pragma unroll
        for (int m = 0; m < K / W; ++m) {
            const V v = reinterpret_cast<const V *>(p)[m];
            __builtin_memcpy(&r[m * W], &v, sizeof(V));
        }
    } else {
#pragma unroll
        for (int c = 0; c < K; ++c) r[c] = c < k ? p[c] : T(0);
    }
}

template <typename T, int K, bool VEC>
__device__ __forceinline__ void store_row(T *p, int k, const T (&r)[K]) {
    if constexpr (VEC) {
        using V = typename Vec16<T>::type;
        constexpr int W = Vec16<T>::W;
#pragma unroll
        for (int m = 0; m < K / W; ++m) {
            V v;
            __builtin_memcpy(&v, &r[m * W], sizeof(V));
            reinterpret_cast<V *>(p)[m] = v;
        }
    } else {
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (c < k) p[c] = r[c];
    }
}

// Rows per Gram tile: 3072 values (FP32) or 1536 (FP64) per matrix, 12 or 6 per thread, so each
// thread keeps 48 bytes of every input in flight while the previous tile is consumed.
template <typename T, int K>
constexpr int gram_tile_rows() {
    return (sizeof(T) == 4 ? 3072 : 1536) / K;
}

// Rows of the per-wave reduction buffer of a Gram accumulation (one per sub-block held by a wave).
template <int K>
constexpr int gram_red() {
    return (K / 4) * (K / 4) <= 64 ? (K / 4) * (K / 4) : 64;
}

// Geometry of a Gram accumulation: thread (rg, sub) owns the 4 x 4 sub-block `sub` of the k x k
// result and the tile rows rg, rg + RG, ...; each thread fetches PER vectors of W values per tile.
template <typename T, int K, bool VEC>
struct GramGeom {
    static constexpr int NS = K / 4;
    static constexpr int TPR = NS * NS;
    static constexpr int RG = kBlock / TPR;
    static constexpr int TR = gram_tile_rows<T, K>();
    static constexpr int W = VEC ? Vec16<T>::W : 1;
    static constexpr int CV = K / W;  // vectors per row
    static constexpr int PER = TR * CV / kBlock;
    static_assert(PER * kBlock == TR * CV, "tile must split evenly over the threads");
    static_assert(kBlock % CV == 0, "a thread's columns must not change between its vectors");
    static constexpr int NW = kBlock / 64;
    static constexpr int RED = gram_red<K>();
    static constexpr size_t RED_BYTES = (size_t)NW * RED * 16 * sizeof(double);
};

// Contiguous row range [r0, r1) of workgroup blockIdx.x when n rows are split over the grid.
__device__ __forceinline__ void block_rows(int64_t n, int64_t &r0, int64_t &r1) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    r0 = (int64_t)blockIdx.x * per;
    r1 = (r0 + per < n) ? r0 + per : n;
}

// W values of one row starting at column c: one 16-byte vector when VEC, else column c alone
// (zero when c >= k).
template <typename T, int W, bool VEC>
__device__ __forceinline__ void load_cols(const T *row, int c, int k, T (&x)[W]) {
    if constexpr (VEC) {
        using V = typename Vec16<T>::type;
        static_assert(W == Vec16<T>::W, "vector width");
        const V v = *reinterpret_cast<const V *>(row + c);
        __builtin_memcpy(x, &v, sizeof(V));
    } else {
        static_assert(W == 1, "scalar width");
        x[0] = c < k ? row[c] : T(0);
    }
}

// acc[m] += A^T B_m over the rows rg, rg + RG, ... of one LDS tile of TR rows (NB = 1 or 2 right
// factors sharing the left one).  Each matrix is accumulated in the same order whatever NB is.
template <typename T, int K, int TR, int NB>
__device__ __forceinline__ void gram_tile(const T (*sA)[K], const T (*sB0)[K], const T (*sB1)[K], int rg, int a0,
                                          int b0, double (&acc)[NB][4][4]) {
    constexpr int RG = kBlock / ((K / 4) * (K / 4));
    for (int r = rg; r < TR; r += RG) {
        double av[4], bv[NB][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            av[q] = (double)sA[r][a0 + q];
            bv[0][q] = (double)sB0[r][b0 + q];
            if constexpr (NB > 1) bv[1][q] = (double)sB1[r][b0 + q];
        }
#pragma unroll
        for (int m = 0; m < NB; ++m)
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[m][p][q] = fma(av[p], bv[m][q], acc[m][p][q]);
    }
}

// Sum the row groups of acc[m] (inside a wave with shuffles, across waves through LDS, in a fixed
// order) and write the block's partials part[m][a][b] (a, b < k).  s_red may alias the tiles: the
// caller has passed a barrier after its last tile.
template <int K, int NB>
__device__ __forceinline__ void gram_block_reduce(double (&acc)[NB][4][4], double (*s_red)[gram_red<K>()][16], int k, double *__restrict__ part) {
    constexpr int TPR = (K / 4) * (K / 4);
    constexpr int NW = kBlock / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int sub = tid % TPR, a0 = (sub / (K / 4)) * 4, b0 = (sub % (K / 4)) * 4;
    const size_t kk = (size_t)k * k;
#pragma unroll
    for (int m = 0; m < NB; ++m) {
#pragma unroll
        for (int o = TPR; o < 64; o <<= 1)
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[m][p][q] += __shfl_xor(acc[m][p][q], o);
        if (lane < (TPR <= 64 ? TPR : 64))
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) s_red[wave][lane][p * 4 + q] = acc[m][p][q];
        __syncthreads();
        if (tid < TPR) {
            const int wl = TPR <= 64 ? tid : tid % 64;
            for (int e = 0; e < 16; ++e) {
                double v = 0.0;
                if (TPR <= 64) {  // every wave holds all TPR sub-blocks: add the waves in order
                    for (int w = 0; w < NW; ++w) v += s_red[w][wl][e];
                } else {  // one row group: sub-block tid lives in wave tid / 64
                    v = s_red[tid / 64][wl][e];
                }
                const int a = a0 + e / 4, b = b0 + e % 4;
                if (a < k && b < k) part[m * kk + a * k + b] = v;
            }
        }
        __syncthreads();
    }
}

// One level of a fixed-order reduction over the partials part[q][e] (row stride `stride`):
// out[g][e] = sum_{q < kTreeFan} part[g*kTreeFan + q][e] for e < len, out rows of stride len.
__global__ __launch_bounds__(kBlock) void sum_level(const double *__restrict__ part, int nparts, int len,
                                                  int64_t stride, double *__restrict__ out,
                                                  double *__restrict__ out2) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= len) return;
    const int g = blockIdx.y;
    const int q1 = (g + 1) * kTreeFan < nparts ? (g + 1) * kTreeFan : nparts;
    double v[kTreeFan];
#pragma unroll
    for (int q = 0; q < kTreeFan; ++q) {
        const int qq = g * kTreeFan + q;
        v[q] = qq < q1 ? part[(int64_t)qq * stride + e] : 0.0;
    }
    double sacc = 0.0;
#pragma unroll
    for (int q = 0; q < kTreeFan; ++q) sacc += v[q];
    out[(int64_t)g * len + e] = sacc;
    if (out2) out2[(int64_t)g * len + e] = sacc;
}

// Sum kDenseBlocks partials of `len` doubles (row stride `stride` >= len) into out (and out2): two
// fixed-order levels through `mid` ([kDenseBlocks / kTreeFan][len]).
inline void sum_partials(const double *part, int len, double *mid, double *out, double *out2, hipStream_t s,
                         int64_t stride = 0) {
    constexpr int ngroups = kDenseBlocks / kTreeFan;
    const unsigned gx = (unsigned)((len + kBlock - 1) / kBlock);
    sum_level<<<dim3(gx, ngroups), kBlock, 0, s>>>(part, kDenseBlocks, len, stride > 0 ? stride : len, mid, nullptr);
    sum_level<<<dim3(gx, 1), kBlock, 0, s>>>(mid, ngroups, len, len, out, out2);
}

// Entry (a, c) of a k x k row-major matrix held in global memory, read at a wave-uniform address.
// With VEC (k == K) the offset is a compile-time constant after unrolling, so the load is a scalar
// load into SGPRs; otherwise entries outside k x k read as zero.
template <int K, bool VEC>
__device__ __forceinline__ double mat_at(const double *__restrict__ M, int k, int a, int c) {
    if constexpr (VEC) return M[a * K + c];
    return (a < k && c < k) ? M[a * k + c] : 0.0;
}

// Per-block partial of M = A^T B over a contiguous row range.  A = A1 + t A2 (rounded to T) when
// AXPY; B = A when SAME.  Tiles of rows are staged in LDS with coalesced (16-byte when VEC) loads, the
// next tile being fetched into registers while the current one is consumed.  The LDS of the tiles
// is reused for the final reduction over row groups.
template <typename T, int K, bool VEC, bool AXPY, bool SAME>
__global__ __launch_bounds__(kBlock) void gram_partial(int64_t n, int k, const T *__restrict__ A1, int64_t lda1,
                                                     const T *__restrict__ A2, int64_t lda2, double t,
                                                     const T *__restrict__ B, int64_t ldb, double *__restrict__ part) {
    using Geo = GramGeom<T, K, VEC>;
    constexpr int TR = Geo::TR, W = Geo::W, CV = Geo::CV, PER = Geo::PER;
    constexpr size_t TILE_BYTES = (size_t)TR * K * sizeof(T) * (SAME ? 1 : 2);
    __shared__ __align__(16) unsigned char smem[TILE_BYTES > Geo::RED_BYTES ? TILE_BYTES : Geo::RED_BYTES];
    T(*sA)[K] = reinterpret_cast<T(*)[K]>(smem);
    T(*sB)[K] = SAME ? sA : reinterpret_cast<T(*)[K]>(smem + (size_t)TR * K * sizeof(T));
    const int tid = threadIdx.x, sub = tid % Geo::TPR, rg = tid / Geo::TPR;
    const int a0 = (sub / Geo::NS) * 4, b0 = (sub % Geo::NS) * 4;
    const int c = (tid % CV) * W;  // this thread's columns, the same for all its vectors
    int64_t r0, r1;
    block_rows(n, r0, r1);
    double acc[1][4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[0][p][q] = 0.0;
    T xa[PER][W], xb[SAME ? 1 : PER][W];
    auto fetch = [&](int64_t t0) {
#pragma unroll
        for (int v = 0; v < PER; ++v) {
            const int64_t i = t0 + (tid + v * kBlock) / CV;
            T x[W], x2[W], y[W];
#pragma unroll
            for (int q = 0; q < W; ++q) x[q] = x2[q] = y[q] = T(0);
            if (i < r1) {
                load_cols<T, W, VEC>(A1 + i * lda1, c, k, x);
                if constexpr (AXPY) load_cols<T, W, VEC>(A2 + i * lda2, c, k, x2);
                if constexpr (!SAME) load_cols<T, W, VEC>(B + i * ldb, c, k, y);
            }
#pragma unroll
            for (int q = 0; q < W; ++q) {
                xa[v][q] = AXPY ? (T)((double)x[q] + t * (double)x2[q]) : x[q];
                if constexpr (!SAME) xb[v][q] = y[q];
            }
        }
    };
    if (r0 < r1) fetch(r0);
    for (int64_t t0 = r0; t0 < r1; t0 += TR) {
#pragma unroll
        for (int v = 0; v < PER; ++v) {
            const int r = (tid + v * kBlock) / CV;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                sA[r][c + q] = xa[v][q];
                if constexpr (!SAME) sB[r][c + q] = xb[v][q];
            }
        }
        __syncthreads();
        if (t0 + TR < r1) fetch(t0 + TR);
        gram_tile<T, K, TR, 1>(sA, sB, nullptr, rg, a0, b0, acc);
        __syncthreads();
    }
    gram_block_reduce<K, 1>(acc, reinterpret_cast<double(*)[gram_red<K>()][16]>(smem), k,
                            part + (int64_t)blockIdx.x * k * k);
}

// out[i, :] = beta Z[i, :] + (s1 (A1[i, :] + t A2[i, :])) M1 + (s2 X[i, :]) M2, with A1 + t A2
// rounded to T first.  One lane per row: the row's k outputs are accumulated in FP64 registers; the
// row-vector terms are added in the order A, X, Z so that the products can start while the later
// loads are still in flight.  s1 and s2 scale the row values (exact for the +-1 the library uses).
template <typename T, int K, bool VEC, bool AXPY, bool HAS_X, bool HAS_Z>
__global__ __launch_bounds__(kBlock) void apply_rows(int64_t n, int k, double beta, const T *__restrict__ Z,
                                                   int64_t ldz, const T *__restrict__ A1, int64_t lda1,
                                                   const T *__restrict__ A2, int64_t lda2, double t,
                                                   const double *__restrict__ M1, double s1,
                                                   const T *__restrict__ X, int64_t ldx,
                                                   const double *__restrict__ M2, double s2, T *__restrict__ out,
                                                   int64_t ldo) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    T a[K], a2[AXPY ? K : 1], x[HAS_X ? K : 1], z[HAS_Z ? K : 1];
    load_row<T, K, VEC>(A1 + i * lda1, k, a);
    if constexpr (AXPY) load_row<T, K, VEC>(A2 + i * lda2, k, a2);
    if constexpr (HAS_X) load_row<T, K, VEC>(X + i * ldx, k, x);
    if constexpr (HAS_Z) load_row<T, K, VEC>(Z + i * ldz, k, z);
    __builtin_amdgcn_sched_barrier(0);  // every row load is issued before the first product
    double o[K];
#pragma unroll
    for (int c = 0; c < K; ++c) o[c] = 0.0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const double av = s1 * (AXPY ? (double)(T)((double)a[r] + t * (double)a2[r]) : (double)a[r]);
#pragma unroll
        for (int c = 0; c < K; ++c) o[c] = fma(av, mat_at<K, VEC>(M1, k, r, c), o[c]);
    }
    if constexpr (HAS_X) {
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const double xv = s2 * (double)x[r];
#pragma unroll
            for (int c = 0; c < K; ++c) o[c] = fma(xv, mat_at<K, VEC>(M2, k, r, c), o[c]);
        }
    }
    T res[K];
#pragma unroll
    for (int c = 0; c < K; ++c) res[c] = (T)(HAS_Z ? fma(beta, (double)z[c], o[c]) : o[c]);
    store_row<T, K, VEC>(out + i * ldo, k, res);
}

}  // namespace
}  // namespace pspec
