// Dense n x k operations of the Grassmann geometry: tall-skinny Gram matrices, the tangent
// projection Z - U (U^T Z) (- X MX), the Cholesky-QR retraction qf(U + t eta), and the FP64 inner
// product / axpby used by the truncated-CG driver.
//
// Every sum over the n rows is FP64 and deterministic: a fixed grid of kDenseBlocks workgroups, each
// owning a contiguous row range, writes one partial, and a single workgroup adds the partials in
// order.  Gram: each thread owns a 4 x 4 block of the k x k result and streams the rows of its
// workgroup's range (the FP64 VALU work, 2 k^2 flops per row, stays below the HBM time of reading
// the two n x k inputs for k <= 32; FP64 matrix cores run at the same rate as the FP64 VALU on this
// GPU, so they would not shorten it).  Apply: one lane per row keeps the row's k outputs in
// registers while the k x k matrix is read from LDS with broadcast reads.
#include <cmath>

#include "common.hpp"

namespace pspec {
namespace {

constexpr int kDenseBlocks = 1024;  // first-level partials of Gram matrices and dot products
constexpr int kTreeFan = 32;         // partials summed per thread at each further level

// Workspace layout (doubles): level-1 partials [kDenseBlocks][k*k], level-2 partials
// [kDenseBlocks / kTreeFan][k*k], then M, R^-1 (k*k each), plus slack.
size_t dense_ws_doubles(int k) {
    const size_t kk = (size_t)k * k;
    return kDenseBlocks * kk + (kDenseBlocks / kTreeFan) * kk + 2 * kk + 64;
}

// Rows per LDS tile: 1024 values per matrix for FP32 (4 per thread), 512 for FP64.
template <typename T, int K>
constexpr int gram_tile_rows() {
    return (sizeof(T) == 4 ? 1024 : 512) / K;
}

// Per-block partial of M = A^T B over a contiguous row range.  A = A1 + t A2 when AXPY; B = A when
// SAME.  Tiles of rows are staged in LDS with coalesced loads (the next tile is fetched into
// registers while the current one is consumed); thread (rg, sub) owns the 4 x 4 sub-block `sub` of M
// and accumulates the tile rows rg, rg + RG, ... in FP64.
template <typename T, int K, bool AXPY, bool SAME>
__global__ __launch_bounds__(kBlock) void gram_partial(int64_t n, int k, const T *__restrict__ A1, int64_t lda1,
                                                     const T *__restrict__ A2, int64_t lda2, double t,
                                                     const T *__restrict__ B, int64_t ldb, double *__restrict__ part) {
    constexpr int NS = K / 4;
    constexpr int TPR = NS * NS;
    constexpr int RG = kBlock / TPR;
    constexpr int TR = gram_tile_rows<T, K>();
    constexpr int KP = K + 4;  // padded LDS row (keeps 16-byte alignment of each 4-wide read)
    constexpr int PER = TR * K / kBlock;  // tile values per thread per matrix
    constexpr int NW = kBlock / 64;
    __shared__ T sA[TR][KP];
    __shared__ T sB[SAME ? 1 : TR][KP];
    __shared__ double s_red[NW][TPR <= 64 ? TPR : 64][16];
    const int tid = threadIdx.x, sub = tid % TPR, rg = tid / TPR;
    const int a0 = (sub / NS) * 4, b0 = (sub % NS) * 4;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = (r0 + per < n) ? r0 + per : n;
    double acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
    T xa[PER], xb[PER];
    auto fetch = [&](int64_t t0) {
#pragma unroll
        for (int v = 0; v < PER; ++v) {
            const int e = tid + v * kBlock;
            const int r = e / K, c = e % K;
            const int64_t i = t0 + r;
            T x = 0, y = 0;
            if (i < r1 && c < k) {
                x = A1[i * lda1 + c];
                if (AXPY) x = (T)((double)x + t * (double)A2[i * lda2 + c]);
                if (!SAME) y = B[i * ldb + c];
            }
            xa[v] = x;
            xb[v] = y;
        }
    };
    if (r0 < r1) fetch(r0);
    for (int64_t t0 = r0; t0 < r1; t0 += TR) {
#pragma unroll
        for (int v = 0; v < PER; ++v) {
            const int e = tid + v * kBlock;
            sA[e / K][e % K] = xa[v];
            if (!SAME) sB[e / K][e % K] = xb[v];
        }
        __syncthreads();
        if (t0 + TR < r1) fetch(t0 + TR);
        for (int r = rg; r < TR; r += RG) {
            double av[4], bv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                av[q] = (double)sA[r][a0 + q];
                bv[q] = SAME ? (double)sA[r][b0 + q] : (double)sB[r][b0 + q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fma(av[p], bv[q], acc[p][q]);
        }
        __syncthreads();
    }
    // sum the row groups: inside a wave with shuffles, across waves in LDS, in a fixed order
#pragma unroll
    for (int o = TPR; o < 64; o <<= 1)
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p][q] += __shfl_xor(acc[p][q], o);
    const int lane = tid & 63, wave = tid >> 6;
    if (lane < (TPR <= 64 ? TPR : 64))
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) s_red[wave][lane][p * 4 + q] = acc[p][q];
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
            if (a < k && b < k) part[(int64_t)blockIdx.x * k * k + a * k + b] = v;
        }
    }
}

// One level of a fixed-order reduction: out[g][e] = sum_{q < kTreeFan} part[g*kTreeFan + q][e].
__global__ __launch_bounds__(kBlock) void sum_level(const double *__restrict__ part, int nparts, int len,
                                                  double *__restrict__ out, double *__restrict__ out2) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= len) return;
    const int g = blockIdx.y;
    const int q1 = (g + 1) * kTreeFan < nparts ? (g + 1) * kTreeFan : nparts;
    double v[kTreeFan];
#pragma unroll
    for (int q = 0; q < kTreeFan; ++q) {
        const int qq = g * kTreeFan + q;
        v[q] = qq < q1 ? part[(int64_t)qq * len + e] : 0.0;
    }
    double sacc = 0.0;
#pragma unroll
    for (int q = 0; q < kTreeFan; ++q) sacc += v[q];
    out[(int64_t)g * len + e] = sacc;
    if (out2) out2[(int64_t)g * len + e] = sacc;
}

// Sum kDenseBlocks partials of `len` doubles into out (and out2): two fixed-order levels.
void sum_partials(const double *part, int len, double *mid, double *out, double *out2, hipStream_t s) {
    constexpr int ngroups = kDenseBlocks / kTreeFan;
    const unsigned gx = (unsigned)((len + kBlock - 1) / kBlock);
    sum_level<<<dim3(gx, ngroups), kBlock, 0, s>>>(part, kDenseBlocks, len, mid, nullptr);
    sum_level<<<dim3(gx, 1), kBlock, 0, s>>>(mid, ngroups, len, out, out2);
}

// Cholesky factor R (upper, positive diagonal) of the SPD k x k matrix M, and R^-1.  One workgroup;
// thread c owns column c (of R during the factorisation, of R^-1 during the back substitution, which
// each thread carries out in its own column of the output array).
__global__ __launch_bounds__(64) void chol_inv(int k, const double *__restrict__ M, double *__restrict__ R_out,
                                               double *__restrict__ Rinv) {
    __shared__ double R[PSPEC_K_MAX][PSPEC_K_MAX + 1];
    const int c = threadIdx.x;
    if (c < k)
        for (int r = 0; r < k; ++r) R[r][c] = M[r * k + c];
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (c == j) R[j][j] = sqrt(R[j][j]);
        __syncthreads();
        if (c > j && c < k) R[j][c] /= R[j][j];
        __syncthreads();
        if (c > j && c < k)
            for (int r = j + 1; r <= c; ++r) R[r][c] -= R[j][r] * R[j][c];
        __syncthreads();
    }
    if (c < k) {
        for (int r = k - 1; r >= 0; --r) {
            double v = 0.0;
            if (r <= c) {
                v = (r == c) ? 1.0 : 0.0;
                for (int q = r + 1; q <= c; ++q) v -= R[r][q] * Rinv[q * k + c];
                v /= R[r][r];
            }
            Rinv[r * k + c] = v;
        }
        if (R_out)
            for (int r = 0; r < k; ++r) R_out[r * k + c] = r <= c ? R[r][c] : 0.0;
    }
}

// out[i, :] = beta Z[i, :] + (A1[i, :] + t A2[i, :]) (s1 M1) + X[i, :] (s2 M2).
// One lane per row: a tile of TR rows of each input is staged in LDS with coalesced loads, each lane
// keeps its row's k outputs in FP64 registers, the k x k matrices are read with wave-uniform
// addresses, and the outputs go back through LDS for a coalesced store.
// Rows per apply tile: at most 256 (one lane each) and about 12 KB of LDS per staged matrix.
template <typename T, int K>
constexpr int apply_tile_rows() {
    return (12288 / (K * (int)sizeof(T))) < 256 ? 12288 / (K * (int)sizeof(T)) : 256;
}

template <typename T, int K, bool AXPY, bool HAS_X, bool HAS_Z>
__global__ __launch_bounds__(256) void apply_rows(int64_t n, int k, double beta, const T *Z, int64_t ldz,
                                                const T *A1, int64_t lda1, const T *A2, int64_t lda2, double t,
                                                const double *__restrict__ M1, double s1, const T *X, int64_t ldx,
                                                const double *__restrict__ M2, double s2, T *out, int64_t ldo) {
    constexpr int TR = apply_tile_rows<T, K>();
    constexpr int KP = K + 1;
    __shared__ T sA[TR][KP];
    __shared__ T sX[HAS_X ? TR : 1][KP];
    __shared__ T sZ[TR][KP];  // Z tile on the way in, the output tile on the way out
    __shared__ double sM1[K][K];
    __shared__ double sM2[HAS_X ? K : 1][K];
    const int tid = threadIdx.x;
    for (int e = tid; e < K * K; e += TR) {
        const int a = e / K, c = e % K;
        sM1[a][c] = (a < k && c < k) ? s1 * M1[a * k + c] : 0.0;
        if (HAS_X) sM2[a][c] = (a < k && c < k) ? s2 * M2[a * k + c] : 0.0;
    }
    const int64_t t0 = (int64_t)blockIdx.x * TR;
#pragma unroll
    for (int v = 0; v < K; ++v) {
        const int e = tid + v * TR;
        const int r = e / K, c = e % K;
        const int64_t i = t0 + r;
        const bool ok = i < n && c < k;
        T x = 0;
        if (ok) {
            x = A1[i * lda1 + c];
            if (AXPY) x = (T)((double)x + t * (double)A2[i * lda2 + c]);
        }
        sA[r][c] = x;
        if (HAS_X) sX[r][c] = ok ? X[i * ldx + c] : (T)0;
        if (HAS_Z) sZ[r][c] = ok ? Z[i * ldz + c] : (T)0;
    }
    __syncthreads();
    double o[K];
#pragma unroll
    for (int c = 0; c < K; ++c) o[c] = HAS_Z ? beta * (double)sZ[tid][c] : 0.0;
    for (int a = 0; a < k; ++a) {
        const double av = (double)sA[tid][a];
#pragma unroll
        for (int c = 0; c < K; ++c) o[c] = fma(av, sM1[a][c], o[c]);
    }
    if (HAS_X) {
        for (int a = 0; a < k; ++a) {
            const double xv = (double)sX[tid][a];
#pragma unroll
            for (int c = 0; c < K; ++c) o[c] = fma(xv, sM2[a][c], o[c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < K; ++c) sZ[tid][c] = (T)o[c];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < K; ++v) {
        const int e = tid + v * TR;
        const int r = e / K, c = e % K;
        const int64_t i = t0 + r;
        if (i < n && c < k) out[i * ldo + c] = sZ[r][c];
    }
}

template <typename T, int K>
__global__ __launch_bounds__(kBlock) void dot_partial(int64_t n, int k, const T *__restrict__ A, int64_t lda,
                                                    const T *__restrict__ B, int64_t ldb, double *__restrict__ part) {
    __shared__ double s[kBlock];
    constexpr int RG = kBlock / K;
    const int tid = threadIdx.x, c = tid % K, rg = tid / K;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = (r0 + per < n) ? r0 + per : n;
    double acc = 0.0;
    if (c < k)
        for (int64_t i = r0 + rg; i < r1; i += RG) acc = fma((double)A[i * lda + c], (double)B[i * ldb + c], acc);
    s[tid] = acc;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = s[0];
}

template <typename T, int K>
__global__ __launch_bounds__(kBlock) void axpby_k(int64_t n, int k, double alpha, const T *__restrict__ X, int64_t ldx,
                                                double beta, T *__restrict__ Y, int64_t ldy) {
    const int c = threadIdx.x % K;
    if (c >= k) return;
    const int64_t stride = (int64_t)gridDim.x * (kBlock / K);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / K) + threadIdx.x / K; i < n; i += stride) {
        const double y = beta == 0.0 ? 0.0 : beta * (double)Y[i * ldy + c];
        Y[i * ldy + c] = (T)(alpha * (double)X[i * ldx + c] + y);
    }
}

unsigned rows_grid(int64_t n, int per_block) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

unsigned apply_grid(int64_t n, int tile) { return (unsigned)((n + tile - 1) / tile); }

template <typename T, int K>
pspec_status project_impl(int64_t n, int k, const T *U, int64_t ldu, const T *Z, int64_t ldz, const T *X, int64_t ldx,
                          const double *MX, T *out, int64_t ldo, double *M, double *ws, hipStream_t s) {
    const size_t kk = (size_t)k * k;
    double *part = ws;
    double *mid = part + kDenseBlocks * kk;
    double *Mw = mid + (kDenseBlocks / kTreeFan) * kk;
    constexpr int TR = apply_tile_rows<T, K>();
    gram_partial<T, K, false, false><<<kDenseBlocks, kBlock, 0, s>>>(n, k, U, ldu, nullptr, 0, 0.0, Z, ldz, part);
    sum_partials(part, (int)kk, mid, Mw, M, s);
    if (X)
        apply_rows<T, K, false, true, true><<<apply_grid(n, TR), TR, 0, s>>>(n, k, 1.0, Z, ldz, U, ldu, nullptr, 0,
                                                                             0.0, Mw, -1.0, X, ldx, MX, -1.0, out, ldo);
    else
        apply_rows<T, K, false, false, true><<<apply_grid(n, TR), TR, 0, s>>>(
            n, k, 1.0, Z, ldz, U, ldu, nullptr, 0, 0.0, Mw, -1.0, nullptr, 0, nullptr, 0.0, out, ldo);
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

template <typename T, int K>
pspec_status retract_impl(int64_t n, int k, const T *U, int64_t ldu, const T *eta, int64_t lde, double t, T *out,
                          int64_t ldo, double *R, double *ws, hipStream_t s) {
    const size_t kk = (size_t)k * k;
    double *part = ws;
    double *mid = part + kDenseBlocks * kk;
    double *Mw = mid + (kDenseBlocks / kTreeFan) * kk;
    double *Rinv = Mw + kk;
    constexpr int TR = apply_tile_rows<T, K>();
    gram_partial<T, K, true, true><<<kDenseBlocks, kBlock, 0, s>>>(n, k, U, ldu, eta, lde, t, nullptr, 0, part);
    sum_partials(part, (int)kk, mid, Mw, nullptr, s);
    chol_inv<<<1, 64, 0, s>>>(k, Mw, R, Rinv);
    apply_rows<T, K, true, false, false><<<apply_grid(n, TR), TR, 0, s>>>(n, k, 0.0, nullptr, 0, U, ldu, eta, lde, t,
                                                                          Rinv, 1.0, nullptr, 0, nullptr, 0.0, out,
                                                                          ldo);
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

template <typename T, int K>
pspec_status dot_impl(int64_t n, int k, const T *A, int64_t lda, const T *B, int64_t ldb, double *out, double *ws,
                      hipStream_t s) {
    dot_partial<T, K><<<kDenseBlocks, kBlock, 0, s>>>(n, k, A, lda, B, ldb, ws);
    sum_partials(ws, 1, ws + kDenseBlocks, out, nullptr, s);
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

template <typename T, int K>
pspec_status axpby_impl(int64_t n, int k, double alpha, const T *X, int64_t ldx, double beta, T *Y, int64_t ldy,
                        hipStream_t s) {
    axpby_k<T, K><<<rows_grid(n, kBlock / K), kBlock, 0, s>>>(n, k, alpha, X, ldx, beta, Y, ldy);
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

#define PSPEC_DISPATCH_K(k, CALL)                                       \
    switch (pad_k(k)) {                                                 \
        case 4: { constexpr int KK = 4; return CALL; }                  \
        case 8: { constexpr int KK = 8; return CALL; }                  \
        case 16: { constexpr int KK = 16; return CALL; }                \
        case 32: { constexpr int KK = 32; return CALL; }                \
        case 64: { constexpr int KK = 64; return CALL; }                \
        default: set_error("unsupported k = %d", k); return PSPEC_ERR_UNSUPPORTED; \
    }

pspec_status check_block(int64_t n, int k, pspec_dtype dt, const void *A, int64_t ld, const char *name,
                         const char *who) {
    PSPEC_ARG(A != nullptr, "%s: %s is NULL", who, name);
    PSPEC_ARG(ld >= k, "%s: ld of %s = %lld < k", who, name, (long long)ld);
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    PSPEC_ARG(((uintptr_t)A % es) == 0, "%s: %s is not aligned to its element size", who, name);
    return PSPEC_OK;
}

pspec_status check_dims(int64_t n, int k, pspec_dtype dt, const char *who) {
    PSPEC_ARG(n >= 1, "%s: n = %lld < 1", who, (long long)n);
    PSPEC_ARG(k >= 1, "%s: k = %d < 1", who, k);
    PSPEC_UNSUP(k <= PSPEC_K_MAX, "%s: k = %d > %d", who, k, PSPEC_K_MAX);
    PSPEC_ARG(dt == PSPEC_F32 || dt == PSPEC_F64, "%s: bad dtype %d", who, (int)dt);
    return PSPEC_OK;
}

pspec_status check_ws(int k, void *ws, size_t ws_bytes, const char *who) {
    PSPEC_ARG(ws != nullptr, "%s: workspace is NULL", who);
    PSPEC_ARG(((uintptr_t)ws % 256) == 0, "%s: workspace must be 256-byte aligned", who);
    if (ws_bytes < dense_ws_doubles(k) * sizeof(double)) {
        set_error("%s: workspace of %zu bytes < %zu needed", who, ws_bytes, dense_ws_doubles(k) * sizeof(double));
        return PSPEC_ERR_WORKSPACE;
    }
    return PSPEC_OK;
}

}  // namespace

}  // namespace pspec

using namespace pspec;

extern "C" size_t pspec_dense_workspace_bytes(int k) {
    if (k < 1) k = 1;
    if (k > PSPEC_K_MAX) k = PSPEC_K_MAX;
    return dense_ws_doubles(k) * sizeof(double);
}

extern "C" pspec_status pspec_project(int64_t n, int k, pspec_dtype dt, const void *U, int64_t ldu, const void *Z,
                                      int64_t ldz, const void *X, int64_t ldx, const double *MX, void *out, int64_t ldo,
                                      double *M, void *ws, size_t ws_bytes, pspec_stream stream) {
    clear_error();
    pspec_status st;
    if ((st = check_dims(n, k, dt, "project")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, U, ldu, "U", "project")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, Z, ldz, "Z", "project")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, out, ldo, "out", "project")) != PSPEC_OK) return st;
    if (X) {
        if ((st = check_block(n, k, dt, X, ldx, "X", "project")) != PSPEC_OK) return st;
        PSPEC_ARG(MX != nullptr, "project: MX is NULL while X is given");
    }
    if ((st = check_ws(k, ws, ws_bytes, "project")) != PSPEC_OK) return st;
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    PSPEC_ARG(!blocks_overlap(out, ldo, U, ldu, n, k, es), "project: out overlaps U");
    PSPEC_ARG(!(X && blocks_overlap(out, ldo, X, ldx, n, k, es)), "project: out overlaps X");
    PSPEC_ARG(out == Z || !blocks_overlap(out, ldo, Z, ldz, n, k, es), "project: out partially overlaps Z");
    PSPEC_ARG(out != Z || ldo == ldz, "project: in-place needs ldo == ldz");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *w = static_cast<double *>(ws);
    if (dt == PSPEC_F32) {
        PSPEC_DISPATCH_K(k, (project_impl<float, KK>(n, k, (const float *)U, ldu, (const float *)Z, ldz,
                                                     (const float *)X, ldx, MX, (float *)out, ldo, M, w, s)))
    }
    PSPEC_DISPATCH_K(k, (project_impl<double, KK>(n, k, (const double *)U, ldu, (const double *)Z, ldz,
                                                  (const double *)X, ldx, MX, (double *)out, ldo, M, w, s)))
}

extern "C" pspec_status pspec_retract(int64_t n, int k, pspec_dtype dt, const void *U, int64_t ldu, const void *eta,
                                      int64_t lde, double t, void *Uout, int64_t ldo, double *R, void *ws,
                                      size_t ws_bytes, pspec_stream stream) {
    clear_error();
    pspec_status st;
    if ((st = check_dims(n, k, dt, "retract")) != PSPEC_OK) return st;
    PSPEC_ARG(n >= k, "retract: n = %lld < k = %d", (long long)n, k);
    if ((st = check_block(n, k, dt, U, ldu, "U", "retract")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, eta, lde, "eta", "retract")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, Uout, ldo, "Uout", "retract")) != PSPEC_OK) return st;
    PSPEC_ARG(std::isfinite(t), "retract: t is not finite");
    if ((st = check_ws(k, ws, ws_bytes, "retract")) != PSPEC_OK) return st;
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    PSPEC_ARG(!blocks_overlap(Uout, ldo, eta, lde, n, k, es), "retract: Uout overlaps eta");
    PSPEC_ARG(Uout == U || !blocks_overlap(Uout, ldo, U, ldu, n, k, es), "retract: Uout partially overlaps U");
    PSPEC_ARG(Uout != U || ldo == ldu, "retract: in-place needs ldo == ldu");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *w = static_cast<double *>(ws);
    if (dt == PSPEC_F32) {
        PSPEC_DISPATCH_K(k, (retract_impl<float, KK>(n, k, (const float *)U, ldu, (const float *)eta, lde, t,
                                                     (float *)Uout, ldo, R, w, s)))
    }
    PSPEC_DISPATCH_K(k, (retract_impl<double, KK>(n, k, (const double *)U, ldu, (const double *)eta, lde, t,
                                                  (double *)Uout, ldo, R, w, s)))
}

extern "C" pspec_status pspec_dot(int64_t n, int k, pspec_dtype dt, const void *A, int64_t lda, const void *B,
                                  int64_t ldb, double *out, void *ws, size_t ws_bytes, pspec_stream stream) {
    clear_error();
    pspec_status st;
    if ((st = check_dims(n, k, dt, "dot")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, A, lda, "A", "dot")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, B, ldb, "B", "dot")) != PSPEC_OK) return st;
    PSPEC_ARG(out != nullptr, "dot: out is NULL");
    if ((st = check_ws(k, ws, ws_bytes, "dot")) != PSPEC_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *w = static_cast<double *>(ws);
    if (dt == PSPEC_F32) {
        PSPEC_DISPATCH_K(k, (dot_impl<float, KK>(n, k, (const float *)A, lda, (const float *)B, ldb, out, w, s)))
    }
    PSPEC_DISPATCH_K(k, (dot_impl<double, KK>(n, k, (const double *)A, lda, (const double *)B, ldb, out, w, s)))
}

extern "C" pspec_status pspec_axpby(int64_t n, int k, pspec_dtype dt, double alpha, const void *X, int64_t ldx,
                                    double beta, void *Y, int64_t ldy, pspec_stream stream) {
    clear_error();
    pspec_status st;
    if ((st = check_dims(n, k, dt, "axpby")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, X, ldx, "X", "axpby")) != PSPEC_OK) return st;
    if ((st = check_block(n, k, dt, Y, ldy, "Y", "axpby")) != PSPEC_OK) return st;
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    PSPEC_ARG(X == Y ? ldx == ldy : !blocks_overlap(X, ldx, Y, ldy, n, k, es), "axpby: X partially overlaps Y");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dt == PSPEC_F32) {
        PSPEC_DISPATCH_K(k, (axpby_impl<float, KK>(n, k, alpha, (const float *)X, ldx, beta, (float *)Y, ldy, s)))
    }
    PSPEC_DISPATCH_K(k, (axpby_impl<double, KK>(n, k, alpha, (const double *)X, ldx, beta, (double *)Y, ldy, s)))
}
