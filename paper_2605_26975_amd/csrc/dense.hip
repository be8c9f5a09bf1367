// Dense n x k operations of the Grassmann geometry: tall-skinny Gram matrices, the tangent
// projection Z - U (U^T Z) (- X MX), the Cholesky-QR retraction qf(U + t eta), and the FP64 inner
// product / axpby used by the truncated-CG driver.
//
// Every sum over the n rows is FP64 and deterministic: a fixed grid of kDenseBlocks workgroups, each
// owning a contiguous row range, writes one partial, and the partials are added by a fixed two-level
// tree.  Gram matrices (k > 4) and the row-block products X M of the projection and retraction run on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64, four rows per instruction; dense.hpp), which keeps
// them below the HBM time of their passes at k = 32, where the FP64 VALU was bound by operand
// delivery; for k <= 4 each lane accumulates its rows' k x k products by FP64 FMA and the wave adds
// them by DPP (a 16-column matrix tile would leave three quarters of its lanes idle).  Dot and axpby:
// one lane per row, the row moved with 16-byte loads and stores.
#include <cmath>

#include "common.hpp"
#include "dense.hpp"

namespace pspec {
namespace {
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

// Rows loaded together by one lane of the dot product: enough for 64 bytes of each input.
template <typename T, int K>
constexpr int dot_unroll() {
    return (int)(K * sizeof(T)) >= 64 ? 1 : 64 / (int)(K * sizeof(T));
}

// Per-block partial of sum_{i, c} A[i, c] B[i, c] over a contiguous row range: lane per row, FP64
// accumulation in row order per lane, then a fixed-order reduction over the lanes.
template <typename T, int K, bool VEC>
__global__ __launch_bounds__(kBlock) void dot_partial(int64_t n, int k, const T *__restrict__ A, int64_t lda,
                                                    const T *__restrict__ B, int64_t ldb, double *__restrict__ part) {
    constexpr int R = dot_unroll<T, K>();
    constexpr int NW = kBlock / 64;
    __shared__ double s[NW];
    const int tid = threadIdx.x;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = (r0 + per < n) ? r0 + per : n;
    double acc = 0.0;
    for (int64_t i0 = r0 + tid; i0 < r1; i0 += (int64_t)R * kBlock) {
        T a[R][K], b[R][K];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            if (i < r1) {
                load_row<T, K, VEC>(A + i * lda, k, a[u]);
                load_row<T, K, VEC>(B + i * ldb, k, b[u]);
            } else {
#pragma unroll
                for (int c = 0; c < K; ++c) a[u][c] = b[u][c] = T(0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
            for (int c = 0; c < K; ++c) acc = fma((double)a[u][c], (double)b[u][c], acc);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((tid & 63) == 0) s[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double v = 0.0;
        for (int w = 0; w < NW; ++w) v += s[w];
        part[blockIdx.x] = v;
    }
}

// Y = alpha X + beta Y (Y is not read when beta == 0).  Lane per row; X may be Y.
template <typename T, int K, bool VEC>
__global__ __launch_bounds__(kBlock) void axpby_k(int64_t n, int k, double alpha, const T *X, int64_t ldx,
                                                double beta, T *Y, int64_t ldy) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    T x[K], y[K];
    load_row<T, K, VEC>(X + i * ldx, k, x);
    if (beta != 0.0) {
        load_row<T, K, VEC>(Y + i * ldy, k, y);
#pragma unroll
        for (int c = 0; c < K; ++c) y[c] = (T)fma(alpha, (double)x[c], beta * (double)y[c]);
    } else {
#pragma unroll
        for (int c = 0; c < K; ++c) y[c] = (T)(alpha * (double)x[c]);
    }
    store_row<T, K, VEC>(Y + i * ldy, k, y);
}

unsigned row_blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename T, int K, bool VEC>
void launch_project(int64_t n, int k, const T *U, int64_t ldu, const T *Z, int64_t ldz, const T *X, int64_t ldx,
                    const double *MX, T *out, int64_t ldo, double *M, double *ws, hipStream_t s) {
    const size_t kk = (size_t)k * k;
    double *part = ws;
    double *mid = part + kDenseBlocks * kk;
    double *Mw = mid + (kDenseBlocks / kTreeFan) * kk;
    gram_partial<T, K, false, false><<<kDenseBlocks, kBlock, 0, s>>>(n, k, U, ldu, nullptr, 0, 0.0, Z, ldz, part);
    sum_partials(part, (int)kk, mid, Mw, M, s);
    if (X)
        launch_apply<T, K, VEC, false, true, true>(s, n, k, 1.0, Z, ldz, U, ldu, nullptr, 0, 0.0, Mw, -1.0, X, ldx, MX,
                                                   -1.0, out, ldo);
    else
        launch_apply<T, K, VEC, false, false, true>(s, n, k, 1.0, Z, ldz, U, ldu, nullptr, 0, 0.0, Mw, -1.0, nullptr, 0,
                                                    nullptr, 0.0, out, ldo);
}

template <typename T, int K>
pspec_status project_impl(int64_t n, int k, const T *U, int64_t ldu, const T *Z, int64_t ldz, const T *X, int64_t ldx,
                          const double *MX, T *out, int64_t ldo, double *M, double *ws, hipStream_t s) {
    if (rows_vectorisable<T, K>(k, {{U, ldu}, {Z, ldz}, {X, ldx}, {out, ldo}}))
        launch_project<T, K, true>(n, k, U, ldu, Z, ldz, X, ldx, MX, out, ldo, M, ws, s);
    else
        launch_project<T, K, false>(n, k, U, ldu, Z, ldz, X, ldx, MX, out, ldo, M, ws, s);
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

template <typename T, int K, bool VEC>
void launch_retract(int64_t n, int k, const T *U, int64_t ldu, const T *eta, int64_t lde, double t, T *out,
                    int64_t ldo, double *R, double *ws, hipStream_t s) {
    const size_t kk = (size_t)k * k;
    double *part = ws;
    double *mid = part + kDenseBlocks * kk;
    double *Mw = mid + (kDenseBlocks / kTreeFan) * kk;
    double *Rinv = Mw + kk;
    gram_partial<T, K, true, true><<<kDenseBlocks, kBlock, 0, s>>>(n, k, U, ldu, eta, lde, t, nullptr, 0, part);
    sum_partials(part, (int)kk, mid, Mw, nullptr, s);
    chol_inv<<<1, 64, 0, s>>>(k, Mw, R, Rinv);
    launch_apply<T, K, VEC, true, false, false>(s, n, k, 0.0, nullptr, 0, U, ldu, eta, lde, t, Rinv, 1.0, nullptr, 0,
                                                nullptr, 0.0, out, ldo);
}

template <typename T, int K>
pspec_status retract_impl(int64_t n, int k, const T *U, int64_t ldu, const T *eta, int64_t lde, double t, T *out,
                          int64_t ldo, double *R, double *ws, hipStream_t s) {
    if (rows_vectorisable<T, K>(k, {{U, ldu}, {eta, lde}, {out, ldo}}))
        launch_retract<T, K, true>(n, k, U, ldu, eta, lde, t, out, ldo, R, ws, s);
    else
        launch_retract<T, K, false>(n, k, U, ldu, eta, lde, t, out, ldo, R, ws, s);
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

template <typename T, int K>
pspec_status dot_impl(int64_t n, int k, const T *A, int64_t lda, const T *B, int64_t ldb, double *out, double *ws,
                      hipStream_t s) {
    if (rows_vectorisable<T, K>(k, {{A, lda}, {B, ldb}}))
        dot_partial<T, K, true><<<kDenseBlocks, kBlock, 0, s>>>(n, k, A, lda, B, ldb, ws);
    else
        dot_partial<T, K, false><<<kDenseBlocks, kBlock, 0, s>>>(n, k, A, lda, B, ldb, ws);
    sum_partials(ws, 1, ws + kDenseBlocks, out, nullptr, s);
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

template <typename T, int K>
pspec_status axpby_impl(int64_t n, int k, double alpha, const T *X, int64_t ldx, double beta, T *Y, int64_t ldy,
                        hipStream_t s) {
    if (rows_vectorisable<T, K>(k, {{X, ldx}, {Y, ldy}}))
        axpby_k<T, K, true><<<row_blocks(n), kBlock, 0, s>>>(n, k, alpha, X, ldx, beta, Y, ldy);
    else
        axpby_k<T, K, false><<<row_blocks(n), kBlock, 0, s>>>(n, k, alpha, X, ldx, beta, Y, ldy);
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
