// Shared pieces of the dense n x k kernels: 16-byte row access, the FP64 matrix-core (MFMA)
// accumulation of tall-skinny Gram matrices and of the row-block products X M, and the fixed-order
// reduction of per-block partials.  The Gram accumulation and the row-block products are used both
// by the stand-alone kernels and by the fused epilogue of the Riemannian Hessian-vector product;
// both follow the same instruction sequence, so the two produce identical bits.
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
constexpr size_t dense_ws_doubles(int k) {
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

// Contiguous row range [r0, r1) of workgroup blockIdx.x when n rows are split over the grid.
__device__ __forceinline__ void block_rows(int64_t n, int64_t &r0, int64_t &r1) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    r0 = (int64_t)blockIdx.x * per;
    r1 = (r0 + per < n) ? r0 + per : n;
}

// Guarded loads read an in-range element (row and column clamped) and are masked only after every
// load of the batch has been issued: a load whose value is selected right away is turned into a
// load under a branch and waited for on the spot, which serialises the loads of a wave.  pin()
// marks the point where the batch's values are first needed (an empty asm statement that reads
// and writes the register, so the loads cannot be moved below it); it emits no instruction.
__device__ __forceinline__ int64_t clamp_index(int64_t i, int64_t n) { return i < n ? i : n - 1; }

template <typename T>
__device__ __forceinline__ T clamped_load(const T *base, int64_t ld, int64_t row, int64_t n, int col, int k) {
    return base[clamp_index(row, n) * ld + (col < k ? col : k - 1)];
}

template <typename T>
__device__ __forceinline__ void pin(T &x) {
    __asm__ volatile("" : "+v"(x));
}

template <typename T, int N>
__device__ __forceinline__ void pin_all(T (&x)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) pin(x[i]);
}

// ---- wave reductions ---------------------------------------------------------------------------
// One DPP lane exchange of a double (two 32-bit moves, VALU only).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over the 64 lanes in a fixed order, the same value in every lane: within each 16-lane row,
// partners exchanged by DPP (lanes i and i^1, then i^2, then i and 7-i within each half row, then i
// and 15-i; each step adds two equal-sized partial sums, and since addition commutes both partners
// hold the same result), then the four row sums read from lanes 0, 16, 32, 48.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// ---- FP64 matrix cores ------------------------------------------------------------------------
// v_mfma_f64_16x16x4f64 computes D = A B + C for A 16 x 4, B 4 x 16 and C, D 16 x 16.  Lane l
// (l = 16 q + c, q < 4, c < 16) supplies A[c][q] and B[q][c] and holds D[4 i + q][c] in element i of
// its accumulator.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma_f64(double a, double b, dbl4 acc) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// Columns are handled in 16-wide tiles; k < 16 is padded with zero columns.
template <int K>
constexpr int mf_tiles() {
    return K < 16 ? 1 : K / 16;
}

// ---- Gram matrices M = A^T B -----------------------------------------------------------------
// The rows [r0, r1) of a workgroup are taken in groups of four; wave w takes the groups w, w + 4,
// w + 8, ... in that order and feeds group g to one MFMA per pair of column tiles, lane (q, c)
// supplying row 4 g + q, column 16 t + c of both factors.  For UG groups at a time,
// load(row, c, raw) issues the clamped loads of one group into raw, raw.pin() follows all of them,
// and finish(row, c, raw, a, b) forms the left factor a[t] and the NB right factors b[m][t] at
// (row, 16 t + c), zero outside the range or past column k.
template <typename T, int K, int NB, int UG, typename Raw, typename Load, typename Finish>
__device__ __forceinline__ void gram_mfma_rows(int64_t r0, int64_t r1, Load &&load, Finish &&finish,
                                               dbl4 (&acc)[NB][mf_tiles<K>()][mf_tiles<K>()]) {
    constexpr int CT = mf_tiles<K>();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane >> 4, c = lane & 15;
    for (int64_t base = r0 + 4 * w; base < r1; base += (int64_t)16 * UG) {
        Raw raw[UG];
#pragma unroll
        for (int u = 0; u < UG; ++u) load(base + 16 * u + q, c, raw[u]);
#pragma unroll
        for (int u = 0; u < UG; ++u) raw[u].pin();
        T a[UG][CT], b[UG][NB][CT];
#pragma unroll
        for (int u = 0; u < UG; ++u) finish(base + 16 * u + q, c, raw[u], a[u], b[u]);
#pragma unroll
        for (int u = 0; u < UG; ++u)
#pragma unroll
            for (int m = 0; m < NB; ++m)
#pragma unroll
                for (int ta = 0; ta < CT; ++ta)
#pragma unroll
                    for (int tb = 0; tb < CT; ++tb)
                        acc[m][ta][tb] = mfma_f64((double)a[u][ta], (double)b[u][m][tb], acc[m][ta][tb]);
    }
}

// Add the four waves' tiles in wave order and write the block's partials part[m][a][b] (a, b < k).
template <int K, int NB>
__device__ __forceinline__ void gram_mfma_reduce(dbl4 (&acc)[NB][mf_tiles<K>()][mf_tiles<K>()],
                                                 double (*s_red)[4][64], int k, double *__restrict__ part) {
    constexpr int CT = mf_tiles<K>();
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const size_t kk = (size_t)k * k;
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int ta = 0; ta < CT; ++ta)
#pragma unroll
            for (int tb = 0; tb < CT; ++tb) {
#pragma unroll
                for (int i = 0; i < 4; ++i) s_red[w][i][lane] = acc[m][ta][tb][i];
                __syncthreads();
                const int i = tid >> 6;  // element i of lane `lane` of every wave
                const double v = ((s_red[0][i][lane] + s_red[1][i][lane]) + s_red[2][i][lane]) + s_red[3][i][lane];
                const int a = 16 * ta + 4 * i + (lane >> 4), b = 16 * tb + (lane & 15);
                if (a < k && b < k) part[m * kk + (size_t)a * k + b] = v;
                __syncthreads();
            }
}

// Rows gathered per wave before their products are issued.
template <int NB>
constexpr int gram_groups() {
    return 8;
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

// The k x k matrix operands of the lane-per-row kernels are read as M[r * K + c] at compile-time
// offsets and wave-uniform addresses.  With VEC (k == K) M is the caller's matrix in global memory,
// so the reads become scalar loads into SGPR operands; otherwise it is first copied, zero-padded to
// K x K, into LDS (runtime offsets k * r + c would defeat the scalar path) and read as broadcasts.
template <int K>
__device__ __forceinline__ void stage_matrix(const double *__restrict__ M, int k, double *sM) {
    for (int e = threadIdx.x; e < K * K; e += kBlock) {
        const int a = e / K, c = e % K;
        sM[e] = (a < k && c < k) ? M[a * k + c] : 0.0;
    }
}

// Gram rows of a workgroup for k <= 4 on the FP64 VALU, one lane per row (the matrix-core tile would
// pad the rows to 16 columns and leave three quarters of its lanes idle; at k = 8 the 64 FP64
// accumulators per lane would cost more occupancy than the padding does): lane l takes the rows r0 + l,
// r0 + l + 256, ... in order (R at a time, clamped loads masked after the batch) and accumulates
// acc[p][q] += a_p b_q by FMA.
template <typename T, int K, bool AXPY, bool SAME, bool VEC>
__device__ __forceinline__ void gram_rows_lane(int64_t r0, int64_t r1, int k, const T *__restrict__ A1, int64_t lda1,
                                               const T *__restrict__ A2, int64_t lda2, double t,
                                               const T *__restrict__ B, int64_t ldb, double (&acc)[K][K]) {
    constexpr int R = (int)(K * sizeof(T)) >= 32 ? 1 : 32 / (int)(K * sizeof(T));  // rows per lane per batch
    for (int64_t i0 = r0 + threadIdx.x; i0 < r1; i0 += (int64_t)R * kBlock) {
        T a[R][K], a2[R][AXPY ? K : 1], b[R][SAME ? 1 : K];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int64_t i = clamp_index(i0 + (int64_t)u * kBlock, r1);
            load_row<T, K, VEC>(A1 + i * lda1, k, a[u]);
            if constexpr (AXPY) load_row<T, K, VEC>(A2 + i * lda2, k, a2[u]);
            if constexpr (!SAME) load_row<T, K, VEC>(B + i * ldb, k, b[u]);
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            pin_all(a[u]);
            if constexpr (AXPY) pin_all(a2[u]);
            if constexpr (!SAME) pin_all(b[u]);
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const bool ok = i0 + (int64_t)u * kBlock < r1;
            double x[K], y[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                T v = a[u][c];
                if constexpr (AXPY) v = (T)((double)v + t * (double)a2[u][c]);
                x[c] = ok ? (double)v : 0.0;
            }
#pragma unroll
            for (int c = 0; c < K; ++c) {
                if constexpr (SAME) y[c] = x[c];
                else y[c] = ok ? (double)b[u][c] : 0.0;
            }
#pragma unroll
            for (int pa = 0; pa < K; ++pa)
#pragma unroll
                for (int qb = 0; qb < K; ++qb) acc[pa][qb] = fma(x[pa], y[qb], acc[pa][qb]);
        }
    }
}

// Per-block partial of M = A^T B over a contiguous row range: on the FP64 matrix cores for k > 4,
// lane per row on the FP64 VALU up to 4.  A = A1 + t A2 (rounded to T) when AXPY; B = A when SAME.
template <typename T, int K, bool AXPY, bool SAME>
__global__ __launch_bounds__(kBlock) void gram_partial(int64_t n, int k, const T *__restrict__ A1, int64_t lda1,
                                                     const T *__restrict__ A2, int64_t lda2, double t,
                                                     const T *__restrict__ B, int64_t ldb, double *__restrict__ part) {
    if constexpr (K <= 4) {
        __shared__ double s_g[kBlock / 64][K * K];
        int64_t r0, r1;
        block_rows(n, r0, r1);
        double acc[K][K];
#pragma unroll
        for (int pa = 0; pa < K; ++pa)
#pragma unroll
            for (int qb = 0; qb < K; ++qb) acc[pa][qb] = 0.0;
        auto aligned = [](const void *ptr, int64_t ld) {
            return ptr == nullptr || (((uintptr_t)ptr % 16) == 0 && ((size_t)ld * sizeof(T)) % 16 == 0);
        };
        const bool vec = k == K && aligned(A1, lda1) && (!AXPY || aligned(A2, lda2)) && (SAME || aligned(B, ldb));
        if (vec)
            gram_rows_lane<T, K, AXPY, SAME, true>(r0, r1, k, A1, lda1, A2, lda2, t, B, ldb, acc);
        else
            gram_rows_lane<T, K, AXPY, SAME, false>(r0, r1, k, A1, lda1, A2, lda2, t, B, ldb, acc);
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int pa = 0; pa < K; ++pa)
#pragma unroll
            for (int qb = 0; qb < K; ++qb) {
                const double v = wave_sum_f64(acc[pa][qb]);
                if (lane == 0) s_g[w][pa * K + qb] = v;
            }
        __syncthreads();
        for (int e = threadIdx.x; e < k * k; e += kBlock) {
            const int idx = (e / k) * K + e % k;
            part[(int64_t)blockIdx.x * k * k + e] = ((s_g[0][idx] + s_g[1][idx]) + s_g[2][idx]) + s_g[3][idx];
        }
        return;
    }
    constexpr int CT = mf_tiles<K>();
    __shared__ double s_red[4][4][64];
    int64_t r0, r1;
    block_rows(n, r0, r1);
    dbl4 acc[1][CT][CT];
#pragma unroll
    for (int ta = 0; ta < CT; ++ta)
#pragma unroll
        for (int tb = 0; tb < CT; ++tb) acc[0][ta][tb] = dbl4{0.0, 0.0, 0.0, 0.0};
    struct Raw {
        T x[CT], x2[AXPY ? CT : 1], y[SAME ? 1 : CT];
        __device__ void pin() {
            pin_all(x);
            if constexpr (AXPY) pin_all(x2);
            if constexpr (!SAME) pin_all(y);
        }
    };
    auto load = [&](int64_t row, int c, Raw &raw) {
#pragma unroll
        for (int ti = 0; ti < CT; ++ti) {
            raw.x[ti] = clamped_load(A1, lda1, row, r1, 16 * ti + c, k);
            if constexpr (AXPY) raw.x2[ti] = clamped_load(A2, lda2, row, r1, 16 * ti + c, k);
            if constexpr (!SAME) raw.y[ti] = clamped_load(B, ldb, row, r1, 16 * ti + c, k);
        }
    };
    auto finish = [&](int64_t row, int c, const Raw &raw, T(&a)[CT], T(&b)[1][CT]) {
#pragma unroll
        for (int ti = 0; ti < CT; ++ti) {
            const bool ok = row < r1 && 16 * ti + c < k;
            T x = raw.x[ti];
            if constexpr (AXPY) x = (T)((double)x + t * (double)raw.x2[ti]);
            a[ti] = ok ? x : T(0);
            if constexpr (SAME) b[0][ti] = a[ti];
            else b[0][ti] = ok ? raw.y[ti] : T(0);
        }
    };
    gram_mfma_rows<T, K, 1, gram_groups<1>(), Raw>(r0, r1, load, finish, acc);
    gram_mfma_reduce<K, 1>(acc, s_red, k, part + (int64_t)blockIdx.x * k * k);
}

// ---- Row-block products out = beta Z + (s1 A) M1 + (s2 X) M2 ------------------------------------
// Each wave computes 16-row tiles, one 16-column tile of the output per MFMA chain.  The k index of
// the products is permuted so that lane (q, c) needs the contiguous chunk k/4 q .. k/4 q + k/4 - 1 of
// row c of the tile (one or two 16-byte loads): step s of a chain takes k-index kperm(s, q) =
// KS q + s from every lane.  Lane (q, c) then holds output row 4 i + q, column 16 t + c.
template <int K>
constexpr int mf_steps() {
    return (K < 16 ? 16 : K) / 4;  // KS: MFMA steps per chain (padded width / 4)
}

// The M operand of lane (q, c): M[KS q + s][16 t + c] for every tile t and step s (zero past k).
template <int K>
__device__ __forceinline__ void load_mf_operand(const double *__restrict__ M, int k, double (&mb)[mf_tiles<K>()][mf_steps<K>()]) {
    constexpr int KS = mf_steps<K>();
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
#pragma unroll
    for (int t = 0; t < mf_tiles<K>(); ++t)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int r = KS * q + s, col = 16 * t + c;
            mb[t][s] = (r < k && col < k) ? M[r * k + col] : 0.0;
        }
}

// The A-operand chunk of lane (q, c): row `row`, columns KS q .. KS q + KS - 1, loaded clamped into
// the valid range (one or two 16-byte loads when VEC); mask_mf_chunk zeroes it past k or n once the
// batch's loads are issued and pinned.
template <typename T, int K, bool VEC>
__device__ __forceinline__ void load_mf_chunk(const T *base, int64_t ld, int64_t row, int64_t n, int k,
                                              T (&x)[mf_steps<K>()]) {
    constexpr int KS = mf_steps<K>();
    const int c0 = KS * ((threadIdx.x & 63) >> 4);
    if constexpr (VEC) {
        using V = typename Vec16<T>::type;
        constexpr int W = Vec16<T>::W;
        const T *src = base + clamp_index(row, n) * ld + (c0 < K ? c0 : 0);
#pragma unroll
        for (int m = 0; m < KS / W; ++m) {
            const V v = *reinterpret_cast<const V *>(src + m * W);
            __builtin_memcpy(&x[m * W], &v, sizeof(V));
        }
    } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) x[s] = clamped_load(base, ld, row, n, c0 + s, k);
    }
}

template <typename T, int K>
__device__ __forceinline__ void mask_mf_chunk(int64_t row, int64_t n, int k, T (&x)[mf_steps<K>()]) {
    constexpr int KS = mf_steps<K>();
    const int c0 = KS * ((threadIdx.x & 63) >> 4);
#pragma unroll
    for (int s = 0; s < KS; ++s) x[s] = (row < n && c0 + s < k) ? x[s] : T(0);
}

// acc[t] += (sc x) M for the chunk x of this lane's row (one chain of KS MFMAs per column tile).
template <typename T, int K>
__device__ __forceinline__ void mf_products(const T (&x)[mf_steps<K>()], double sc,
                                            const double (&mb)[mf_tiles<K>()][mf_steps<K>()],
                                            dbl4 (&acc)[mf_tiles<K>()]) {
#pragma unroll
    for (int t = 0; t < mf_tiles<K>(); ++t)
#pragma unroll
        for (int s = 0; s < mf_steps<K>(); ++s) acc[t] = mfma_f64(sc * (double)x[s], mb[t][s], acc[t]);
}

// Tiles of 16 rows handed to the waves of the grid in turn, MF_TPI per wave and iteration.
constexpr int MF_TPI = 2;
__device__ __forceinline__ int64_t mf_first_tile() { return (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); }
__device__ __forceinline__ int64_t mf_tile_stride() { return (int64_t)gridDim.x * (kBlock / 64); }
inline unsigned mf_grid(int64_t n) {
    const int64_t tiles = (n + 15) / 16, blocks = (tiles + kBlock / 64 - 1) / (kBlock / 64);
    return (unsigned)(blocks < 4096 ? (blocks < 1 ? 1 : blocks) : 4096);
}

// out = beta Z + (s1 (A1 + t A2)) M1 + (s2 X) M2 with A1 + t A2 rounded to T first, on the FP64
// matrix cores (k <= 32; wider blocks use apply_rows_wide).  s1 and s2 scale the row values (exact for
// the +-1 the library uses).  VEC: 16-byte chunk loads (k == K and aligned rows).
template <typename T, int K, bool VEC, bool AXPY, bool HAS_X, bool HAS_Z>
__global__ __launch_bounds__(kBlock) void apply_rows(int64_t n, int k, double beta, const T *__restrict__ Z,
                                                   int64_t ldz, const T *__restrict__ A1, int64_t lda1,
                                                   const T *__restrict__ A2, int64_t lda2, double t,
                                                   const double *__restrict__ M1, double s1,
                                                   const T *__restrict__ X, int64_t ldx,
                                                   const double *__restrict__ M2, double s2, T *__restrict__ out,
                                                   int64_t ldo) {
    constexpr int CT = mf_tiles<K>(), KS = mf_steps<K>();
    static_assert(K <= 32, "wide blocks use apply_rows_wide");
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    double m1[CT][KS], m2[HAS_X ? CT : 1][HAS_X ? KS : 1];
    load_mf_operand<K>(M1, k, m1);
    if constexpr (HAS_X) load_mf_operand<K>(M2, k, m2);
    // each wave takes MF_TPI tiles per iteration (tile, tile + stride, ...) to keep more loads in flight
    const int64_t stride = mf_tile_stride();
    for (int64_t tile0 = mf_first_tile(); tile0 * 16 < n; tile0 += MF_TPI * stride) {
        T a[MF_TPI][KS], a2[MF_TPI][AXPY ? KS : 1], x[MF_TPI][HAS_X ? KS : 1], z[MF_TPI][HAS_Z ? CT : 1][4];
#pragma unroll
        for (int j = 0; j < MF_TPI; ++j) {
            const int64_t row0 = (tile0 + j * stride) * 16;
            load_mf_chunk<T, K, VEC>(A1, lda1, row0 + c, n, k, a[j]);
            if constexpr (AXPY) load_mf_chunk<T, K, VEC>(A2, lda2, row0 + c, n, k, a2[j]);
            if constexpr (HAS_X) load_mf_chunk<T, K, VEC>(X, ldx, row0 + c, n, k, x[j]);
            if constexpr (HAS_Z)
#pragma unroll
                for (int ti = 0; ti < CT; ++ti)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        z[j][ti][i] = clamped_load(Z, ldz, row0 + 4 * i + q, n, 16 * ti + c, k);
        }
#pragma unroll
        for (int j = 0; j < MF_TPI; ++j) {
            pin_all(a[j]);
            if constexpr (AXPY) pin_all(a2[j]);
            if constexpr (HAS_X) pin_all(x[j]);
            if constexpr (HAS_Z)
#pragma unroll
                for (int ti = 0; ti < CT; ++ti) pin_all(z[j][ti]);
        }
#pragma unroll
        for (int j = 0; j < MF_TPI; ++j) {
            const int64_t row0 = (tile0 + j * stride) * 16;
            mask_mf_chunk<T, K>(row0 + c, n, k, a[j]);
            if constexpr (AXPY) mask_mf_chunk<T, K>(row0 + c, n, k, a2[j]);
            if constexpr (HAS_X) mask_mf_chunk<T, K>(row0 + c, n, k, x[j]);
            if constexpr (AXPY)
#pragma unroll
                for (int s = 0; s < KS; ++s) a[j][s] = (T)((double)a[j][s] + t * (double)a2[j][s]);
            dbl4 acc[CT];
#pragma unroll
            for (int ti = 0; ti < CT; ++ti) acc[ti] = dbl4{0.0, 0.0, 0.0, 0.0};
            mf_products<T, K>(a[j], s1, m1, acc);
            if constexpr (HAS_X) mf_products<T, K>(x[j], s2, m2, acc);
#pragma unroll
            for (int ti = 0; ti < CT; ++ti)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t r = row0 + 4 * i + q;
                    const int col = 16 * ti + c;
                    // z is only used where (r, col) is in range, so it needs no mask
                    if (r < n && col < k)
                        out[r * ldo + col] = (T)(HAS_Z ? fma(beta, (double)z[j][ti][i], acc[ti][i]) : acc[ti][i]);
                }
        }
    }
}

// Apply for k > 32 (see apply_rows): one lane per row on the FP64 VALU; the row's k outputs are
// accumulated in registers in the order A, X, Z so that the products can start while the later
// loads are still in flight.
template <typename T, int K, bool VEC, bool AXPY, bool HAS_X, bool HAS_Z>
__global__ __launch_bounds__(kBlock) void apply_rows_wide(int64_t n, int k, double beta, const T *__restrict__ Z,
                                                   int64_t ldz, const T *__restrict__ A1, int64_t lda1,
                                                   const T *__restrict__ A2, int64_t lda2, double t,
                                                   const double *__restrict__ M1, double s1,
                                                   const T *__restrict__ X, int64_t ldx,
                                                   const double *__restrict__ M2, double s2, T *__restrict__ out,
                                                   int64_t ldo) {
    constexpr int RU = VEC ? K : 1;  // products fully unrolled only with compile-time operand offsets
    __shared__ double sM1[VEC ? 1 : K * K], sM2[VEC || !HAS_X ? 1 : K * K];
    if constexpr (!VEC) {
        stage_matrix<K>(M1, k, sM1);
        if constexpr (HAS_X) stage_matrix<K>(M2, k, sM2);
        __syncthreads();
        M1 = sM1;
        M2 = sM2;
    }
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
#pragma unroll RU
    for (int r = 0; r < K; ++r) {
        const double av = s1 * (AXPY ? (double)(T)((double)a[r] + t * (double)a2[r]) : (double)a[r]);
#pragma unroll
        for (int c = 0; c < K; ++c) o[c] = fma(av, M1[r * K + c], o[c]);
    }
    if constexpr (HAS_X) {
#pragma unroll RU
        for (int r = 0; r < K; ++r) {
            const double xv = s2 * (double)x[r];
#pragma unroll
            for (int c = 0; c < K; ++c) o[c] = fma(xv, M2[r * K + c], o[c]);
        }
    }
    T res[K];
#pragma unroll
    for (int c = 0; c < K; ++c) res[c] = (T)(HAS_Z ? fma(beta, (double)z[c], o[c]) : o[c]);
    store_row<T, K, VEC>(out + i * ldo, k, res);
}

// Launch of the row-block product on stream s (matrix cores for k <= 32, apply_rows_wide above).
template <typename T, int K, bool VEC, bool AXPY, bool HAS_X, bool HAS_Z>
void launch_apply(hipStream_t s, int64_t n, int k, double beta, const T *Z, int64_t ldz, const T *A1, int64_t lda1,
                  const T *A2, int64_t lda2, double t, const double *M1, double s1, const T *X, int64_t ldx,
                  const double *M2, double s2, T *out, int64_t ldo) {
    if constexpr (K <= 32) {
        apply_rows<T, K, VEC, AXPY, HAS_X, HAS_Z><<<mf_grid(n), kBlock, 0, s>>>(n, k, beta, Z, ldz, A1, lda1, A2, lda2, t,
                                                                            M1, s1, X, ldx, M2, s2, out, ldo);
    } else {
        const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
        apply_rows_wide<T, K, VEC, AXPY, HAS_X, HAS_Z><<<blocks, kBlock, 0, s>>>(n, k, beta, Z, ldz, A1, lda1, A2, lda2,
                                                                               t, M1, s1, X, ldx, M2, s2, out, ldo);
    }
}

}  // namespace
}  // namespace pspec
