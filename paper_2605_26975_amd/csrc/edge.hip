// Fused edge pass of the graph p-Laplacian (objective, gradient, Hessian-vector product).
//
// For every column l, with x = u_i - u_j over the stored edges (i, j) of row i (Section 2):
//   N_l   = 1/2 sum w |x|^p                 numerator of Eq. (1)
//   L_i   = sum_j w phi_p(x)                (Delta_p u)_i
//   J_i   = sum_j w psi(x) (v_i - v_j)      (Hessian edge part / (p-1)), psi(x) = max(|x|, eps)^(p-2)
// and per row: D_l += |u_i|^p, a_l += phi_p(u_i) v_i, S_l += L_i v_i.  One pass reads the CSR once
// and gathers the k contiguous values of u_j (and v_j) per edge from the row-major block; |x|^(p-2)
// is formed once per edge-column as exp2((p-2) log2|x|) and gives phi = |x|^(p-2) x,
// |x|^p = phi x and psi = min(|x|^(p-2), eps^(p-2)).
//
// Edge values are accumulated per row in the working precision T; every sum over rows is FP64:
// each light workgroup (kTileRows rows) and each heavy chunk writes one FP64 partial row
// [kQ][k], and a two-stage reduction sums them in a fixed order.  The epilogue (finalize) turns
// the raw rows L, J (stored in the G and HV outputs) into
//   G_i  = (p/D) (L_i - F phi_p(u_i))
//   HV_i = (p/D) ((p-1) J_i - F (p-1) psi(u_i) v_i - G_i a - phi_p(u_i) b),  b = (p/D)(S - F a) = g^T v.
#include <cmath>
#include <type_traits>
#include <utility>

#include "common.hpp"

namespace pspec {
namespace {

enum Mode { OBJ = 0, GRAD = 1, HVP = 2 };

// |x|^(p-2) for x >= 0.  FP32: hardware exp2/log2 on max(x, 2^-64), so an exact zero gives a finite
// value (2^(64 (2-p))) whose product with x is exactly 0.  FP64: the device-library pow().
template <typename T>
struct PowM2;
template <>
struct PowM2<float> {
    float pm2;
    __device__ __forceinline__ float operator()(float ax) const {
        ax = fmaxf(ax, 0x1p-64f);
        return __builtin_amdgcn_exp2f(pm2 * __builtin_amdgcn_logf(ax));
    }
};
template <>
struct PowM2<double> {
    double pm2;
    __device__ __forceinline__ double operator()(double ax) const { return pow(fmax(ax, 0x1p-512), pm2); }
};

template <typename T, typename WT>
struct EdgeArgs {
    const int64_t *rowptr;
    const int32_t *col;
    const WT *w;
    int64_t n;
    int k;
    const T *U;
    const T *V;
    uint32_t ldu_b, ldv_b, U_bytes, V_bytes;  // leading dimensions and extents in bytes
    T *L;                                     // raw (Delta_p u) rows  (the G output)
    T *J;                                     // raw Hessian edge rows (the HV output)
    int64_t ldl, ldj;
    PowM2<T> pw;
    T epsc;          // eps^(p-2)
    int light_max;
    double *partials;  // [(tiles + chunks)][kQ][k]
    const Chunk *chunks;
    double *scratch;   // [chunks][2][k_max]
    int k_max;
    int64_t part_base; // first partial row of the chunks (= tiles)
};

// One edge-column term.  wv is the weight (0 for padding lanes, whose gather is the row itself).
template <typename T, int MODE>
struct Term {
    __device__ __forceinline__ static void apply(const PowM2<T> &pw, T epsc, T ui, T uj, T vi, T vj, T wv, T &Ls,
                                                 T &Js, T &Ns) {
        const T x = ui - uj;
        const T h = pw(fabs(x));
        const T wh = wv * h;
        const T wphi = wh * x;  // w phi_p(x)
        Ns = fma(wphi, x, Ns);  // w |x|^p
        if (MODE != OBJ) Ls += wphi;
        if (MODE == HVP) {
            const T wpsi = fmin(wh, wv * epsc);  // w psi(x)
            Js = fma(wpsi, vi - vj, Js);
        }
    }
};

// Sum the FP64 per-lane accumulators over the lanes of one column and write the block's partial row.
template <int K>
__device__ __forceinline__ void write_partials(double q[kQ], double (*s_red)[kQ][K], double *prow, int k) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int o = K; o < 64; o <<= 1)
#pragma unroll
        for (int i = 0; i < kQ; ++i) q[i] += __shfl_xor(q[i], o);
    if (lane < K)
#pragma unroll
        for (int i = 0; i < kQ; ++i) s_red[wave][i][lane] = q[i];
    __syncthreads();
    if (tid < kQ * K) {
        const int i = tid / K, c = tid % K;
        double s = 0.0;
#pragma unroll
        for (int wv = 0; wv < kBlock / 64; ++wv) s += s_red[wv][i][c];
        if (c < k) prow[i * k + c] = s;
    }
}

// ---- cross-lane helpers (VALU only: DPP broadcasts, readlane, permlane swaps) ---------------
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Value of lane IDX of this lane's group of G lanes (G in {16, 32, 64}), for 32-bit payloads.
template <int G, int IDX>
__device__ __forceinline__ int32_t group_bcast(int32_t v, int lane) {
    static_assert(IDX >= 0 && IDX < G, "lane index outside the group");
    if constexpr (G == 16) {
        return __builtin_amdgcn_update_dpp(0, v, 0x150 + IDX, 0xf, 0xf, false);  // DPP row_newbcast
    } else if constexpr (G == 32) {
        const int32_t lo = __builtin_amdgcn_readlane(v, IDX);
        const int32_t hi = __builtin_amdgcn_readlane(v, 32 + IDX);
        return lane < 32 ? lo : hi;
    } else {
        return __builtin_amdgcn_readlane(v, IDX);
    }
}

// Value of edge slot `e` at step U: lane U * EPR + e of the group (EPR edge slots per step).
template <int G, int EPR, int U>
__device__ __forceinline__ int32_t edge_bcast(int32_t v, int e, int lane) {
    int32_t r = group_bcast<G, U * EPR>(v, lane);
    static_for<1, EPR>([&](auto ec) {
        constexpr int E = decltype(ec)::value;
        const int32_t t = group_bcast<G, U * EPR + E>(v, lane);
        r = e == E ? t : r;
    });
    return r;
}

template <typename T, int G, int EPR, int U>
__device__ __forceinline__ T edge_bcast_val(T v, int e, int lane) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, edge_bcast<G, EPR, U>(__builtin_bit_cast(int32_t, v), e, lane));
    } else {
        const int64_t b = __builtin_bit_cast(int64_t, v);
        const int32_t lo = edge_bcast<G, EPR, U>((int32_t)(b & 0xffffffff), e, lane);
        const int32_t hi = edge_bcast<G, EPR, U>((int32_t)(b >> 32), e, lane);
        return __builtin_bit_cast(T, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
    }
}

// Light rows: a group of G lanes per row (K column lanes x G/K edge slots), kTileRows rows per
// workgroup, rows of a group interleaved so that neighbouring groups stream adjacent CSR ranges.
// A row is walked in chunks of G edges: the group loads the chunk's neighbour ids and weights with
// one coalesced load (lane l of the group takes edge l), hands them to the lanes that need them with
// VALU broadcasts (DPP row broadcast for 16-lane groups, readlane for 32- and 64-lane groups), and
// issues every gather of the chunk before using any.  The ids of the group's next row are loaded
// before the current row's gathers, so a row costs one memory latency, not two.  The gather rate of
// random neighbour rows, not HBM bandwidth, bounds this kernel on random graphs: keeping 4 rows per
// wave (16-lane groups for k <= 16) in flight matters more than the width of each load.

template <typename T, typename WT, int K, int G, int MODE>
__global__ __launch_bounds__(kBlock) void edge_light(EdgeArgs<T, WT> a) {
    constexpr int EPR = G / K;   // edge slots per row
    constexpr int NU = G / EPR;  // shuffle steps per chunk of G edges (= K)
    constexpr int NGRP = kBlock / G;
    constexpr int RS = kTileRows / NGRP;
    static_assert(kTileRows % NGRP == 0, "tile rows must split evenly over groups");
    __shared__ int64_t s_rp[kTileRows + 1];
    __shared__ double s_red[kBlock / 64][kQ][K];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int grp = tid / G, gl = tid % G;
    const int gbase = lane - gl;  // first lane of this group within the wave
    const int c = gl % K, e = gl / K;
    const int cl = c < a.k ? c : a.k - 1;
    const uint32_t cb = (uint32_t)cl * (uint32_t)sizeof(T);
    const int64_t row0 = (int64_t)blockIdx.x * kTileRows;
    for (int t = tid; t <= kTileRows; t += kBlock) {
        const int64_t r = row0 + t;
        s_rp[t] = a.rowptr[r < a.n ? r : a.n];
    }
    __syncthreads();

    const auto rU = make_rsrc(a.U, a.U_bytes);
    const auto rV = make_rsrc(a.V, a.V_bytes);
    // ids and weights of the first chunk of local row rl (padding: the row itself, weight 0)
    auto first_chunk = [&](int rl, int32_t &jl, T &wl) {
        const int64_t row = row0 + rl;
        jl = row < a.n ? (int32_t)row : 0;
        wl = (T)0;
        if (row < a.n) {
            const int64_t b = s_rp[rl], d = s_rp[rl + 1] - b;
            if (d <= a.light_max && gl < d) {
                jl = a.col[b + gl];
                wl = (T)a.w[b + gl];
            }
        }
    };
    int32_t jl;
    T wl;
    first_chunk(grp, jl, wl);
    double q[kQ] = {0.0, 0.0, 0.0, 0.0};  // N, D, a, S
    for (int s = 0; s < RS; ++s) {
        const int rl = grp + s * NGRP;
        const int64_t row = row0 + rl;
        const bool valid = row < a.n;
        const int64_t beg = valid ? s_rp[rl] : 0, end = valid ? s_rp[rl + 1] : 0;
        const bool light = valid && (end - beg) <= a.light_max;
        const int64_t len = light ? end - beg : 0;
        const uint32_t own = valid ? (uint32_t)row : 0u;
        const T ui = bload<T>(rU, own * a.ldu_b + cb);
        T vi = 0;
        if (MODE == HVP) vi = bload<T>(rV, own * a.ldv_b + cb);
        int32_t jn = 0;
        T wn = (T)0;
        if (s + 1 < RS) first_chunk(rl + NGRP, jn, wn);  // prefetch the next row's ids
        const int nch = (int)((len + G - 1) / G);
        T Ls = 0, Js = 0, Ns = 0;
        for (int ch = 0; ch < nch; ++ch) {
            const int64_t c0 = beg + (int64_t)ch * G;
            const int64_t rem = len - (int64_t)ch * G;
            const int cnt = rem <= 0 ? 0 : (rem < G ? (int)rem : G);
            if (ch > 0) {
                jl = gl < cnt ? a.col[c0 + gl] : (int32_t)own;
                wl = gl < cnt ? (T)a.w[c0 + gl] : (T)0;
            }
            T uj[NU], vj[NU];
            static_for<0, NU>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                uj[u] = ui;
                vj[u] = vi;
                if (u * EPR < cnt) {
                    const int32_t j = edge_bcast<G, EPR, u>(jl, e, lane);
                    uj[u] = bload<T>(rU, (uint32_t)j * a.ldu_b + cb);
                    if (MODE == HVP) vj[u] = bload<T>(rV, (uint32_t)j * a.ldv_b + cb);
                }
            });
            // every gather of the chunk is in flight before the first one is used
            static_for<0, NU>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                if (u * EPR < cnt) {
                    const T wv = edge_bcast_val<T, G, EPR, u>(wl, e, lane);
                    Term<T, MODE>::apply(a.pw, a.epsc, ui, uj[u], vi, vj[u], wv, Ls, Js, Ns);
                }
            });
        }
        jl = jn;
        wl = wn;
        if (EPR > 1) {
#pragma unroll
            for (int o = K; o < G; o <<= 1) {
                if (MODE != OBJ) Ls += __shfl_xor(Ls, o);
                if (MODE == HVP) Js += __shfl_xor(Js, o);
            }
        }
        q[0] += (double)Ns;
        if (valid && e == 0) {
            const T hi = a.pw(fabs(ui));
            const T phi = hi * ui;  // phi_p(u_i)
            q[1] += (double)(phi * ui);
            if (MODE == HVP) {
                q[2] += (double)phi * (double)vi;
                if (light) q[3] += (double)Ls * (double)vi;
            }
            if (light && c < a.k) {
                if (MODE != OBJ) a.L[row * a.ldl + c] = Ls;
                if (MODE == HVP) a.J[row * a.ldj + c] = Js;
            }
        }
    }
    write_partials<K>(q, s_red, a.partials + (int64_t)blockIdx.x * kQ * a.k, a.k);
}

// Heavy rows: one workgroup per chunk of at most PSPEC_CHUNK edges.  The chunk's neighbour ids and
// weights are staged in LDS with coalesced loads; the workgroup's 256/K edge slots then stream them.
template <typename T, typename WT, int K, int MODE, int UNR>
__global__ __launch_bounds__(kBlock) void edge_heavy(EdgeArgs<T, WT> a) {
    constexpr int EPB = kBlock / K;
    __shared__ int32_t s_col[PSPEC_CHUNK];
    __shared__ T s_w[PSPEC_CHUNK];
    __shared__ double s_r[3][kBlock];
    const Chunk ch = a.chunks[blockIdx.x];
    const int len = (int)(ch.end - ch.beg);
    const int tid = threadIdx.x;
    for (int t = tid; t < len; t += kBlock) {
        s_col[t] = a.col[ch.beg + t];
        s_w[t] = (T)a.w[ch.beg + t];
    }
    __syncthreads();
    const int c = tid % K, e = tid / K;
    const int cl = c < a.k ? c : a.k - 1;
    const uint32_t cb = (uint32_t)cl * (uint32_t)sizeof(T);
    const auto rU = make_rsrc(a.U, a.U_bytes);
    const auto rV = make_rsrc(a.V, a.V_bytes);
    const uint32_t row = (uint32_t)ch.row;
    const T ui = bload<T>(rU, row * a.ldu_b + cb);
    T vi = 0;
    if (MODE == HVP) vi = bload<T>(rV, row * a.ldv_b + cb);
    T Ls = 0, Js = 0, Ns = 0;
    for (int base = 0; base < len; base += EPB * UNR) {
        int32_t j[UNR];
        T wv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int idx = base + u * EPB + e;
            const bool ok = idx < len;
            j[u] = ok ? s_col[idx] : (int32_t)row;
            wv[u] = ok ? s_w[idx] : (T)0;
        }
        T uj[UNR], vj[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uj[u] = bload<T>(rU, (uint32_t)j[u] * a.ldu_b + cb);
            vj[u] = (MODE == HVP) ? bload<T>(rV, (uint32_t)j[u] * a.ldv_b + cb) : (T)0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) Term<T, MODE>::apply(a.pw, a.epsc, ui, uj[u], vi, vj[u], wv[u], Ls, Js, Ns);
    }
    s_r[0][tid] = (double)Ls;
    s_r[1][tid] = (double)Js;
    s_r[2][tid] = (double)Ns;
    __syncthreads();
    if (tid < K && tid < a.k) {
        double L = 0.0, J = 0.0, N = 0.0;
        for (int q = 0; q < EPB; ++q) {
            L += s_r[0][q * K + tid];
            J += s_r[1][q * K + tid];
            N += s_r[2][q * K + tid];
        }
        if (ch.slot < 0) {
            if (MODE != OBJ) a.L[(int64_t)row * a.ldl + tid] = (T)L;
            if (MODE == HVP) a.J[(int64_t)row * a.ldj + tid] = (T)J;
        } else {
            a.scratch[((int64_t)ch.slot * 2 + 0) * a.k_max + tid] = L;
            a.scratch[((int64_t)ch.slot * 2 + 1) * a.k_max + tid] = J;
        }
        double *prow = a.partials + (a.part_base + blockIdx.x) * kQ * a.k;
        prow[0 * a.k + tid] = N;
        prow[1 * a.k + tid] = 0.0;
        prow[2 * a.k + tid] = 0.0;
        prow[3 * a.k + tid] = (MODE == HVP) ? L * (double)vi : 0.0;
    }
}

// Rows spanning several chunks: sum the chunk rows in chunk order.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void combine_split(const Split *__restrict__ splits, int64_t n_split,
                                                      const double *__restrict__ scratch, int k, int k_max,
                                                      T *__restrict__ L, int64_t ldl, T *__restrict__ J,
                                                      int64_t ldj) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_split * k) return;
    const int64_t s = t / k;
    const int c = (int)(t - s * k);
    const Split sp = splits[s];
    double Ls = 0.0, Js = 0.0;
    for (int q = 0; q < sp.count; ++q) {
        Ls += scratch[((int64_t)(sp.first + q) * 2 + 0) * k_max + c];
        Js += scratch[((int64_t)(sp.first + q) * 2 + 1) * k_max + c];
    }
    L[(int64_t)sp.row * ldl + c] = (T)Ls;
    if (MODE == HVP) J[(int64_t)sp.row * ldj + c] = (T)Js;
}

// Stage 1: workgroup b sums a contiguous range of partial rows, R rows in parallel per quantity.
__global__ __launch_bounds__(kBlock) void reduce_stage1(const double *__restrict__ part, int64_t P, int W,
                                                      double *__restrict__ red1) {
    __shared__ double s[kBlock];
    const int tid = threadIdx.x;
    const int R = kBlock / W;
    const int qi = tid % W, r = tid / W;
    const int64_t per = (P + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = (r0 + per < P) ? r0 + per : P;
    double acc = 0.0;
    if (r < R)
        for (int64_t row = r0 + r; row < r1; row += R) acc += part[row * W + qi];
    s[tid] = acc;
    __syncthreads();
    if (tid < W) {
        double t = 0.0;
        for (int i = 0; i < R; ++i) t += s[i * W + tid];
        red1[(int64_t)blockIdx.x * W + tid] = t;
    }
}

// Stage 2 (one workgroup): totals and the per-column scalars.
__global__ __launch_bounds__(kBlock) void reduce_stage2(const double *__restrict__ red1, int W, int k, double p,
                                                      double *__restrict__ sc, int k_max, double *__restrict__ F_col,
                                                      double *__restrict__ F) {
    __shared__ double s[kBlock];
    __shared__ double sf[PSPEC_K_MAX];
    const int tid = threadIdx.x;
    if (tid < W) {
        double acc = 0.0;
        for (int b = 0; b < kReduceSlices; ++b) acc += red1[b * W + tid];
        s[tid] = acc;
    }
    __syncthreads();
    if (tid < k) {
        const double N = 0.5 * s[0 * k + tid], D = s[1 * k + tid], av = s[2 * k + tid], S = s[3 * k + tid];
        const double Fl = N / D, pD = p / D;
        sc[SC_N * k_max + tid] = N;
        sc[SC_D * k_max + tid] = D;
        sc[SC_F * k_max + tid] = Fl;
        sc[SC_PD * k_max + tid] = pD;
        sc[SC_A * k_max + tid] = av;
        sc[SC_B * k_max + tid] = pD * (S - Fl * av);
        sf[tid] = Fl;
        if (F_col) F_col[tid] = Fl;
    }
    __syncthreads();
    if (tid == 0 && F) {
        double t = 0.0;
        for (int c = 0; c < k; ++c) t += sf[c];
        *F = t;
    }
}

// Epilogue: G (and HV) from the raw rows and the per-column scalars; K lanes per row.
template <typename T, int K, int MODE>
__global__ __launch_bounds__(kBlock) void finalize(int64_t n, int k, const T *__restrict__ U, int64_t ldu,
                                                 const T *__restrict__ V, int64_t ldv, T *__restrict__ G, int64_t ldg,
                                                 T *__restrict__ HV, int64_t ldh, PowM2<T> pw, T epsc, double p,
                                                 const double *__restrict__ sc, int k_max) {
    const int64_t stride = (int64_t)gridDim.x * (kBlock / K);
    const int c = threadIdx.x % K;
    if (c >= k) return;
    const double pD = sc[SC_PD * k_max + c], F = sc[SC_F * k_max + c];
    const double av = sc[SC_A * k_max + c], bv = sc[SC_B * k_max + c];
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / K) + threadIdx.x / K; i < n; i += stride) {
        const T u = U[i * ldu + c];
        const T h = pw(fabs(u));
        const T phi = h * u;
        const double g = pD * ((double)G[i * ldg + c] - F * (double)phi);
        G[i * ldg + c] = (T)g;
        if (MODE == HVP) {
            const T v = V[i * ldv + c];
            const T psi = fmin(h, epsc);
            const double hv =
                pD * ((p - 1.0) * (double)HV[i * ldh + c] - F * (p - 1.0) * (double)psi * (double)v - g * av -
                      (double)phi * bv);
            HV[i * ldh + c] = (T)hv;
        }
    }
}

template <int K>
constexpr int light_group() {
    return K <= 16 ? 16 : K;
}
constexpr int kUnroll = 4;

unsigned grid_for(int64_t items, int64_t per_block, int64_t cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

template <typename T, typename WT, int K, int MODE>
pspec_status launch_edges(Graph *g, int k, const T *U, int64_t ldu, const T *V, int64_t ldv, T *L, int64_t ldl, T *J,
                          int64_t ldj, double p, double eps, double *F_col, double *F, hipStream_t s) {
    EdgeArgs<T, WT> a;
    a.rowptr = g->rowptr;
    a.col = g->col;
    a.w = static_cast<const WT *>(g->w);
    a.n = g->n;
    a.k = k;
    a.U = U;
    a.V = V;
    a.ldu_b = (uint32_t)(ldu * (int64_t)sizeof(T));
    a.ldv_b = (uint32_t)(ldv * (int64_t)sizeof(T));
    a.U_bytes = (uint32_t)block_extent(g->n, k, ldu, sizeof(T));
    a.V_bytes = V ? (uint32_t)block_extent(g->n, k, ldv, sizeof(T)) : 0u;
    a.L = L;
    a.J = J;
    a.ldl = ldl;
    a.ldj = ldj;
    a.pw.pm2 = (T)(p - 2.0);
    a.epsc = (T)std::pow(eps, p - 2.0);
    a.light_max = PSPEC_LIGHT_MAX;
    a.partials = g->partials;
    a.chunks = g->chunks;
    a.scratch = g->chunk_scratch;
    a.k_max = g->k_max;
    a.part_base = g->tiles;
    if (g->ev_before) PSPEC_HIP(hipEventRecord(g->ev_before, s));
    edge_light<T, WT, K, light_group<K>(), MODE><<<(unsigned)g->tiles, kBlock, 0, s>>>(a);
    if (g->n_chunks > 0) edge_heavy<T, WT, K, MODE, kUnroll><<<(unsigned)g->n_chunks, kBlock, 0, s>>>(a);
    if (g->n_split > 0 && MODE != OBJ)
        combine_split<T, MODE><<<grid_for(g->n_split * k, kBlock, 1 << 30), kBlock, 0, s>>>(
            g->splits, g->n_split, g->chunk_scratch, k, g->k_max, L, ldl, J, ldj);
    if (g->ev_after) PSPEC_HIP(hipEventRecord(g->ev_after, s));
    const int W = kQ * k;
    reduce_stage1<<<kReduceSlices, kBlock, 0, s>>>(g->partials, g->tiles + g->n_chunks, W, g->red1);
    reduce_stage2<<<1, kBlock, 0, s>>>(g->red1, W, k, p, g->scalars, g->k_max, F_col, F);
    if (MODE != OBJ) {
        PowM2<T> pw;
        pw.pm2 = (T)(p - 2.0);
        const T epsc = (T)std::pow(eps, p - 2.0);
        finalize<T, K, MODE><<<grid_for(g->n, kBlock / K, 65536), kBlock, 0, s>>>(
            g->n, k, U, ldu, V, ldv, L, ldl, J, ldj, pw, epsc, p, g->scalars, g->k_max);
    }
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

template <typename T, typename WT, int MODE>
pspec_status dispatch_k(Graph *g, int k, const T *U, int64_t ldu, const T *V, int64_t ldv, T *L, int64_t ldl, T *J,
                        int64_t ldj, double p, double eps, double *F_col, double *F, hipStream_t s) {
    switch (pad_k(k)) {
        case 4: return launch_edges<T, WT, 4, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s);
        case 8: return launch_edges<T, WT, 8, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s);
        case 16: return launch_edges<T, WT, 16, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s);
        case 32: return launch_edges<T, WT, 32, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s);
        case 64: return launch_edges<T, WT, 64, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s);
        default: set_error("unsupported k = %d", k); return PSPEC_ERR_UNSUPPORTED;
    }
}

template <int MODE>
pspec_status dispatch(Graph *g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V, int64_t ldv,
                      void *L, int64_t ldl, void *J, int64_t ldj, double p, double eps, double *F_col, double *F,
                      hipStream_t s) {
    if (dt == PSPEC_F32)
        return dispatch_k<float, float, MODE>(g, k, (const float *)U, ldu, (const float *)V, ldv, (float *)L, ldl,
                                              (float *)J, ldj, p, eps, F_col, F, s);
    if (g->wtype == PSPEC_F32)
        return dispatch_k<double, float, MODE>(g, k, (const double *)U, ldu, (const double *)V, ldv, (double *)L,
                                               ldl, (double *)J, ldj, p, eps, F_col, F, s);
    return dispatch_k<double, double, MODE>(g, k, (const double *)U, ldu, (const double *)V, ldv, (double *)L, ldl,
                                            (double *)J, ldj, p, eps, F_col, F, s);
}

// Host-side argument checks shared by the three entry points.
pspec_status check_common(Graph *g, pspec_dtype dt, int k, const void *U, int64_t ldu, double p, const char *who) {
    PSPEC_ARG(g != nullptr, "%s: NULL graph", who);
    PSPEC_ARG(dt == PSPEC_F32 || dt == PSPEC_F64, "%s: bad dtype %d", who, (int)dt);
    PSPEC_UNSUP(!(dt == PSPEC_F32 && g->wtype == PSPEC_F64), "%s: F32 arithmetic needs F32 weights", who);
    PSPEC_ARG(k >= 1, "%s: k = %d < 1", who, k);
    PSPEC_ARG(k <= g->k_max, "%s: k = %d exceeds the graph's k_max = %d", who, k, g->k_max);
    PSPEC_ARG(U != nullptr, "%s: U is NULL", who);
    PSPEC_ARG(ldu >= k, "%s: ldu = %lld < k", who, (long long)ldu);
    PSPEC_ARG(p > 1.0 && p <= 2.0, "%s: p = %g outside (1, 2]", who, p);
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    PSPEC_UNSUP(block_extent(g->n, k, ldu, es) < (1ull << 32), "%s: U spans 4 GiB or more", who);
    PSPEC_ARG(((uintptr_t)U % es) == 0, "%s: U is not aligned to its element size", who);
    return PSPEC_OK;
}

pspec_status check_out(Graph *g, pspec_dtype dt, int k, const void *X, int64_t ld, const char *name, const char *who) {
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    PSPEC_ARG(X != nullptr, "%s: %s is NULL", who, name);
    PSPEC_ARG(ld >= k, "%s: ld of %s = %lld < k", who, name, (long long)ld);
    PSPEC_ARG(((uintptr_t)X % es) == 0, "%s: %s is not aligned to its element size", who, name);
    PSPEC_UNSUP(block_extent(g->n, k, ld, es) < (1ull << 32), "%s: %s spans 4 GiB or more", who, name);
    return PSPEC_OK;
}

}  // namespace
}  // namespace pspec

using namespace pspec;

extern "C" pspec_status pspec_objective(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, double p,
                                        double *F_col, double *F, pspec_stream stream) {
    clear_error();
    pspec_status st = check_common(g, dt, k, U, ldu, p, "objective");
    if (st != PSPEC_OK) return st;
    return dispatch<OBJ>(g, dt, k, U, ldu, nullptr, 0, nullptr, 0, nullptr, 0, p, 1.0, F_col, F,
                         reinterpret_cast<hipStream_t>(stream));
}

extern "C" pspec_status pspec_grad(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, double p, void *G,
                                   int64_t ldg, double *F_col, pspec_stream stream) {
    clear_error();
    pspec_status st = check_common(g, dt, k, U, ldu, p, "grad");
    if (st != PSPEC_OK) return st;
    if ((st = check_out(g, dt, k, G, ldg, "G", "grad")) != PSPEC_OK) return st;
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    PSPEC_ARG(!blocks_overlap(U, ldu, G, ldg, g->n, k, es), "grad: G overlaps U");
    return dispatch<GRAD>(g, dt, k, U, ldu, nullptr, 0, G, ldg, nullptr, 0, p, 1.0, F_col, nullptr,
                          reinterpret_cast<hipStream_t>(stream));
}

extern "C" pspec_status pspec_hvp(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                                  int64_t ldv, double p, double eps, void *HV, int64_t ldh, void *G, int64_t ldg,
                                  double *F_col, pspec_stream stream) {
    clear_error();
    pspec_status st = check_common(g, dt, k, U, ldu, p, "hvp");
    if (st != PSPEC_OK) return st;
    PSPEC_ARG(eps > 0.0 && std::isfinite(eps), "hvp: eps = %g must be positive", eps);
    if ((st = check_out(g, dt, k, V, ldv, "V", "hvp")) != PSPEC_OK) return st;
    if ((st = check_out(g, dt, k, HV, ldh, "HV", "hvp")) != PSPEC_OK) return st;
    if ((st = check_out(g, dt, k, G, ldg, "G", "hvp")) != PSPEC_OK) return st;
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    const int64_t n = g->n;
    PSPEC_ARG(!blocks_overlap(HV, ldh, U, ldu, n, k, es) && !blocks_overlap(HV, ldh, V, ldv, n, k, es) &&
                  !blocks_overlap(G, ldg, U, ldu, n, k, es) && !blocks_overlap(G, ldg, V, ldv, n, k, es) &&
                  !blocks_overlap(G, ldg, HV, ldh, n, k, es),
              "hvp: HV and G must not overlap U, V or each other");
    return dispatch<HVP>(g, dt, k, U, ldu, V, ldv, G, ldg, HV, ldh, p, eps, F_col, nullptr,
                         reinterpret_cast<hipStream_t>(stream));
}
