// Fused edge pass of the graph p-Laplacian (objective, gradient, Hessian-vector product).
//
// For every column l, with x = u_i - u_j over the stored edges (i, j) of row i (Section 2):
//   N_l   = 1/2 sum w |x|^p                 numerator of Eq. (1)
//   L_i   = sum_j w phi_p(x)                (Delta_p u)_i
//   J_i   = sum_j w psi(x) (v_i - v_j)      (Hessian edge part / (p-1)), psi(x) = max(|x|, eps)^(p-2)
// and per row: D_l += |u_i|^p, a_l += phi_p(u_i) v_i, S_l += L_i v_i.  The objective alone (OBJ) needs
// no row output, so when every row's columns ascend it visits each undirected edge once: w and |x|^p
// are symmetric in (i, j), hence N_l = sum over the entries j > i, half the gathers.  One pass reads the CSR once
// and gathers the k contiguous values of u_j (and v_j) per edge from the row-major block; |x|^(p-2)
// is formed once per edge-column as exp2((p-2) log2|x|) and gives phi = |x|^(p-2) x,
// |x|^p = phi x and psi = min(|x|^(p-2), eps^(p-2)).
//
// Edge values are accumulated per row in the working precision T; every sum over rows is FP64:
// each light workgroup (kTileRows rows) and each workgroup of the persistent heavy-chunk kernel
// writes one FP64 partial row [kQ][k], and a two-stage reduction sums them in a fixed order.  The
// epilogue (finalize) turns the raw rows L, J (stored in the G and HV outputs) into
//   G_i  = (p/D) (L_i - F phi_p(u_i))
//   HV_i = (p/D) ((p-1) J_i - F (p-1) psi(u_i) v_i - G_i a - phi_p(u_i) b),  b = (p/D)(S - F a) = g^T v;
// the sparse-only Hessian (pspec_hvp_sparse) sets a = b = 0, dropping the rank-2 term.  The
// Riemannian call (pspec_rhvp) fuses the epilogue with both projections for 16 <= k <= 32.
#include <cmath>
#include <mutex>
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "dense.hpp"

namespace pspec {
namespace {

// OBJ: N and D only.  GRAD: also L = Delta_p u.  HVP: also J (needs V) and the scalars of the
// rank-2 term.  HESS: the Hessian at a fixed U whose gradient G is given: J and the rank-2 scalars,
// with b = g^T v summed from G, no L.
enum Mode { OBJ = 0, GRAD = 1, HVP = 2, HESS = 3 };
constexpr bool mode_l(int m) { return m == GRAD || m == HVP; }  // forms L
constexpr bool mode_v(int m) { return m == HVP || m == HESS; }  // reads V, forms J

// |x|^(p-2) for x >= 0.  FP32: hardware exp2/log2 on max(x, 2^-64), so an exact zero gives a finite
// value (2^(64 (2-p))) whose product with x is exactly 0.  FP64: exp(q ln x) for x clamped to
// [2^-512, inf), q = p - 2, table-driven after Tang (ACM TOMS 1989 and 1990), written out for this one
// use (the general pow() handles cases that cannot occur here and costs several times as many
// instructions, which bounds the FP64 edge pass):
//   x = 2^e m, m in [1, 2); j = the top 7 bits of m's fraction; r = m C_j - 1 (|r| <= 2^-8, one FMA),
//   C_j ~ 1 / (1 + (j + 1/2) / 128);  ln x = e ln 2 + (-ln C_j) + ln(1 + r), the series of ln(1 + r) to
//   r^8 (truncation below 2^-67), -ln C_j a double-double from the table, e ln 2 with ln 2 split so
//   that e ln2_hi is exact;  t = q ln x as a double-double;
//   exp(t) = 2^(n / 128) exp(s), n = rint(128 t / ln 2), |s| <= ln 2 / 256, exp(s) by its Taylor series
//   to s^6 (truncation below 2^-72), 2^(k / 128) (k = n mod 128) a double-double from the table.
// A transcription on the CPU is within 0.52 units in the last place of pow over x in [1e-150, 1e3],
// q in [-0.95, 0.5].  q = 0 gives exactly 1 (and is returned at once: p = 2 is the first level of every
// continuation); x = inf gives pow()'s limits.  The tables (pow_tables.inc, from gen_pow_tables.py) are
// staged into LDS by every kernel that evaluates the FP64 power (stage_pow).
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

constexpr int kPowTabLen = 5 * 128;  // C, LH, LL (logarithm), TH, TL (exponential)
__device__ const double kPowTab[kPowTabLen] = {
#include "pow_tables.inc"
};

// FP64 fused multiply-add whose addend (vvs) or multiplier (vsv) is wave-uniform, taken from an SGPR
// pair: one v_fma_f64.  Left to itself the compiler keeps series coefficients in VGPRs and copies one
// into the destination before every step (v_mov_b64 + v_fmac_f64), which doubles the instruction
// count of the FP64 power.  Same operation, same rounding as fma().
__device__ __forceinline__ double fma_vvs(double a, double b, double c) {
    double r;
    __asm__("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}
__device__ __forceinline__ double fma_vsv(double a, double b, double c) {
    double r;
    __asm__("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}
__device__ __forceinline__ double fma_neg_vsv(double a, double b, double c) {  // -a b + c
    double r;
    __asm__("v_fma_f64 %0, -%1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

template <>
struct PowM2<double> {
    double pm2;
    const double *tab = nullptr;  // the kernel's LDS copy of kPowTab (set by stage_pow)
    __device__ __forceinline__ double operator()(double ax) const {
        constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;  // ln 2 to 42 bits: e * kLn2Hi is exact
        constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
        constexpr double k128Log2e = 0x1.71547652b82fep0 * 128.0;
        if (pm2 == 0.0) return 1.0;  // p = 2 (uniform branch): the routine below gives exactly 1 too
        const double x = fmax(ax, 0x1p-512);
        int e;
        const double m = frexp(x, &e);  // [1/2, 1): the same fraction bits as 2m in [1, 2)
        const int j = (int)((uint32_t)__double2hiint(m) >> 13) & 127;
        const double C = tab[j], LH = tab[128 + j], LL = tab[256 + j];
        const double r = fma(m + m, C, -1.0);  // exact scaling of m, one rounding
        const double r2 = r * r;
        double P = fma_vsv(r, -1.0 / 8.0, 1.0 / 7.0);
        P = fma_vvs(P, r, -1.0 / 6.0);
        P = fma_vvs(P, r, 1.0 / 5.0);
        P = fma_vvs(P, r, -1.0 / 4.0);
        P = fma_vvs(P, r, 1.0 / 3.0);
        P = fma(P, r, -0.5);
        const double lp = fma(r2, P, r);  // ln(1 + r)
        const double de = (double)(e - 1);
        const double a = de * kLn2Hi;  // exact; |a| >= ln 2 >= |LH| unless e = 1
        const double hi = a + LH;
        const double lo = ((a - hi) + LH) + (fma_vsv(de, kLn2Lo, LL) + lp);
        const double th = pm2 * hi;
        const double tl = fma(pm2, hi, -th) + pm2 * lo;
        const double n = rint(th * k128Log2e);
        double s = fma_neg_vsv(n, kLn2Hi / 128.0, th);
        s = fma_neg_vsv(n, kLn2Lo / 128.0, s) + tl;
        double E = fma_vsv(s, 1.0 / 720.0, 1.0 / 120.0);
        E = fma_vvs(E, s, 1.0 / 24.0);
        E = fma_vvs(E, s, 1.0 / 6.0);
        E = fma(E, s, 0.5);
        E = fma(E * s, s, s);  // exp(s) - 1
        const int ni = (int)n;
        const int k = ni & 127;
        const double TH = tab[384 + k], TL = tab[512 + k];
        const double y = ldexp(fma(TH, E, fma(TL, E, TL)) + TH, ni >> 7);  // 2^(n/128) (1 + E)
        // x = inf (a non-finite U): the limits of pow (0, 1 or inf by the sign of q); NaN stays NaN
        return x < __builtin_inf() ? y : (pm2 < 0.0 ? 0.0 : (pm2 == 0.0 ? 1.0 : x));
    }
};

// Stage the FP64 power's tables into the kernel's LDS array s (kPowTabLen doubles) and point pw at
// it; a no-op for FP32.  Every thread of the workgroup must call it before its first power.
template <typename T>
__device__ __forceinline__ void stage_pow(PowM2<T> &pw, double *s) {
    if constexpr (sizeof(T) == 8) {
        for (int i = threadIdx.x; i < kPowTabLen; i += blockDim.x) s[i] = kPowTab[i];
        __syncthreads();
        pw.tab = s;
    }
}

template <typename T, typename WT>
struct EdgeArgs {
    const int64_t *rowptr;
    const int32_t *col;
    const WT *w;
    int64_t n;
    int k;
    const T *U;
    const T *V;
    const T *Gc;                              // HESS: the gradient at U (n x k), else NULL
    uint32_t ldu_b, ldv_b, U_bytes, V_bytes;  // leading dimensions and extents in bytes
    uint32_t ldg_b, G_bytes;
    T *L;                                     // raw (Delta_p u) rows  (the G output)
    T *J;                                     // raw Hessian edge rows (the HV output)
    int64_t ldl, ldj;
    PowM2<T> pw;
    T epsc;          // eps^(p-2)
    int light_max;
    double *partials;  // [(tiles + heavy workgroups)][kQ][k]
    const Chunk *chunks;
    double *scratch;   // [split chunks][2][k_max]
    int k_max;
    int64_t part_base; // first partial row of the chunks (= tiles)
    int64_t seg_base[kSegs + 1];  // chunks of column segment s: [seg_base[s], seg_base[s + 1])
    int64_t n_chunks;             // the shared list: [seg_base[kSegs], n_chunks)
    const int64_t *ustart;        // OBJ over rows with ascending columns: the first entry j > i of each
                                  // row (each undirected edge visited once); otherwise NULL
    double *gpart;                // light kernel with Gram products: [tiles][kGramQ][k][k]
    const int32_t *lperm;         // light tiles' rows in degree order, or NULL (node order)
};

// One edge-column term.  wv is the weight (0 for padding lanes, whose gather is the row itself).
// FLOOR: the gather-floor reference of the benchmark -- the same loads and stores with the
// arithmetic replaced by a plain sum of the gathered values (the results are not the method's).
template <typename T, int MODE, bool FLOOR = false>
struct Term {
    __device__ __forceinline__ static void apply(const PowM2<T> &pw, T epsc, T ui, T uj, T vi, T vj, T wv, T &Ls,
                                                 T &Js, T &Ns) {
        if constexpr (FLOOR) {
            Ns += uj;
            Ls += wv;
            Js += vj;
            return;
        }
        const T x = ui - uj;
        const T h = pw(fabs(x));
        const T wh = wv * h;
        const T wphi = wh * x;  // w phi_p(x)
        Ns = fma(wphi, x, Ns);  // w |x|^p
        if (mode_l(MODE)) Ls += wphi;
        if (mode_v(MODE)) {
            const T wpsi = fmin(wh, wv * epsc);  // w psi(x)
            Js = fma(wpsi, vi - vj, Js);
        }
    }
};

// ---- cross-lane helpers (VALU only: DPP broadcasts, readlane, permlane swaps) ---------------
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Value of lane IDX of this lane's group of G lanes (G in {4, 8, 16, 32, 64}), for 32-bit payloads.
template <int G, int IDX>
__device__ __forceinline__ int32_t group_bcast(int32_t v, int lane) {
    static_assert(IDX >= 0 && IDX < G, "lane index outside the group");
    if constexpr (G == 4) {
        return __builtin_amdgcn_update_dpp(0, v, IDX * 0x55, 0xf, 0xf, false);  // DPP quad_perm [IDX x 4]
    } else if constexpr (G == 8) {
        // lane IDX % 4 of each quad, then the other quad's copy by row_half_mirror (lane j of each
        // 8 takes lane 7 - j); each lane keeps the copy from the quad that holds lane IDX
        const int32_t y = __builtin_amdgcn_update_dpp(0, v, (IDX & 3) * 0x55, 0xf, 0xf, false);
        const int32_t z = __builtin_amdgcn_update_dpp(0, y, 0x141, 0xf, 0xf, false);
        return (lane & 4) == (IDX & 4) ? y : z;
    } else if constexpr (G == 16) {
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

// Light rows: a group of G = 16 lanes (one DPP row) per row, four rows per wave, or for k <= 8 a
// group of G = K lanes (K = 4 or 8, k padded) per row, 16 or 8 rows per wave; kTileRows rows per
// workgroup, rows of a group interleaved so that neighbouring groups stream adjacent CSR ranges.
// For k <= 16 the group is KL = K column lanes x G/KL edge slots; for k > 16 each lane owns
// CPL = K/16 columns at stride 16, so every load is a coalesced 64-byte segment and four rows per
// wave stay in flight.  A row is walked in chunks of G edges: the group loads
// the chunk's neighbour ids and weights with one coalesced load (lane l takes edge l), the loading
// lane turns each id into byte offsets into U and V once, DPP broadcasts hand offsets and
// weights to the lanes that need them, and every gather of the chunk is issued before any is
// used (in FP32; FP64 issues them in batches, see light_batches).  The group's next row (its own
// u_i, v_i and first-chunk ids) is loaded before the current row's gathers.  A tile's rows are taken
// in degree order (lperm), so that the rows of a wave are about equally long, in every FP64 call
// and in FP32 calls on graphs whose light rows' degrees vary widely; else in node order.  The
// gather rate of random neighbour rows, not HBM bandwidth, bounds this kernel in FP32 on random
// graphs: rows in flight per wave matter more than the width of each load.
template <int K>
constexpr int light_cpl() {
    return K > 16 ? K / 16 : 1;
}

// Lanes per row group: 16, or K for K = 4 and 8, where a 16-lane group would hold 16 / K edge slots
// of K columns and repeat the row's own power and sums in every slot; K-lane groups take one edge at
// a time and keep 64 / K rows per wave in flight.
template <int K>
constexpr int light_group() {
    return K <= 4 ? 4 : (K == 8 ? 8 : 16);
}

// Batches in which the light kernel issues and consumes the gathers of one chunk of G edges: all at
// once in FP32, whose pass is bound by the gathers; in several batches in FP64, whose pass is bound
// by the arithmetic of the power and gains resident waves from the registers this frees.  Measured
// per mode and width: the objective 4 at k >= 16 (k = 16: 6 -> 7 waves per SIMD) and 2 below (4
// measured slower on a 100k-node kNN graph, k = 8, whose few waves gain nothing from occupancy); the
// gradient passes 2 at k <= 16 (4 waves either way, fewer waits), 8 at k = 32 (3 -> 4 waves) and 4
// above.
template <typename T, int K, int MODE>
constexpr int light_batches() {
    if constexpr (sizeof(T) == 4) return 1;
    else if constexpr (MODE == OBJ) return K >= 16 ? 4 : 2;
    else return K == 32 ? 8 : (K > 32 ? 4 : 2);
}

// Waves per SIMD the light kernel is compiled for (k = 32 in FP32 sits just above 128 VGPRs).
template <typename T, int K, bool GRAM = false>
constexpr int light_waves() {
    return GRAM ? 4 : (sizeof(T) == 4 && K == 32) ? 4 : 1;
}

template <typename T, typename WT, int K, int MODE, bool FLOOR = false, bool GRAM = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(light_waves<T, K, GRAM>()))) void edge_light(EdgeArgs<T, WT> a) {
    constexpr int G = light_group<K>();  // lanes per row group
    constexpr int CPL = light_cpl<K>();  // columns per lane
    constexpr int KL = K / CPL;          // column lanes per edge slot
    constexpr int EPR = G / KL;          // edge slots per row
    constexpr int NU = G / EPR;          // broadcast steps per chunk of G edges
    constexpr int NGRP = kBlock / G;
    constexpr int RS = kTileRows / NGRP;
    static_assert(kTileRows % NGRP == 0, "tile rows must split evenly over groups");
    __shared__ int64_t s_b[kTileRows], s_e[kTileRows];  // each slot's row: first and past-the-last entry
    __shared__ int32_t s_row[kTileRows];
    __shared__ int64_t s_up[MODE == OBJ ? kTileRows : 1];
    __shared__ double s_red[kBlock / 64][kQ][K];
    __shared__ double s_gred[GRAM ? kBlock / 64 : 1][4][64];
    __shared__ double s_pow[sizeof(T) == 8 ? kPowTabLen : 1];
    static_assert(!GRAM || (K == 16 && (MODE == HVP || MODE == HESS) && !FLOOR), "Gram products: k = 16, HVP or HESS");
    PowM2<T> pw = a.pw;  // a local copy (taking the address of the argument block would move it to scratch)
    stage_pow(pw, s_pow);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int grp = tid / G, gl = tid % G;
    const int c = gl % KL, e = gl / KL;
    uint32_t cb[CPL];  // byte offsets of this lane's columns (clamped to k - 1)
#pragma unroll
    for (int m = 0; m < CPL; ++m) {
        const int cm = c + m * KL;
        cb[m] = (uint32_t)(cm < a.k ? cm : a.k - 1) * (uint32_t)sizeof(T);
    }
    // slot t of the tile takes row row0 + t, or the tile's t-th row in degree order (lperm); slots past
    // the last row are empty
    const int64_t row0 = (int64_t)blockIdx.x * kTileRows;
    for (int t = tid; t < kTileRows; t += kBlock) {
        const int64_t slot = row0 + t;
        const int64_t r = slot < a.n ? (a.lperm != nullptr ? (int64_t)a.lperm[slot] : slot) : a.n;
        s_row[t] = (int32_t)(slot < a.n ? r : 0);
        s_b[t] = a.rowptr[r];
        s_e[t] = slot < a.n ? a.rowptr[r + 1] : s_b[t];
        if (MODE == OBJ && a.ustart != nullptr && slot < a.n) s_up[t] = a.ustart[r];
    }
    __syncthreads();
    // first entry of slot rl's row this pass visits: the whole row, or its entries j > i (OBJ, ascending)
    auto first = [&](int rl) -> int64_t {
        if constexpr (MODE == OBJ) {
            if (a.ustart != nullptr) return s_up[rl];
        }
        return s_b[rl];
    };

    const auto rU = make_rsrc(a.U, a.U_bytes);
    const auto rV = make_rsrc(a.V, a.V_bytes);
    const auto rG = make_rsrc(a.Gc, a.G_bytes);
    // What row rl needs before its gathers: own u_i, v_i, and the first chunk's neighbour offsets
    // (padding: the row itself, weight 0).  Loaded one row ahead.
    struct RowPre {
        T ui[CPL], vi[CPL];
        T wl;
        uint32_t ou, ov;
    };
    auto prefetch = [&](int rl) {
        RowPre r;
        const bool valid = row0 + rl < a.n;
        const int64_t row = s_row[rl];
        uint32_t j = valid ? (uint32_t)row : 0u;
#pragma unroll
        for (int m = 0; m < CPL; ++m) {
            r.ui[m] = bload<T>(rU, j * a.ldu_b + cb[m]);
            r.vi[m] = mode_v(MODE) ? bload<T>(rV, j * a.ldv_b + cb[m]) : (T)0;
        }
        r.wl = (T)0;
        if (valid) {
            const int64_t b = first(rl), d = s_e[rl] - s_b[rl];
            if (d <= a.light_max && gl < s_e[rl] - b) {
                j = (uint32_t)a.col[b + gl];
                r.wl = (T)a.w[b + gl];
            }
        }
        r.ou = j * a.ldu_b;
        r.ov = j * a.ldv_b;
        return r;
    };
    RowPre nxt = prefetch(grp);
    double q[kQ][CPL];  // N, D, a, S per owned column
#pragma unroll
    for (int i = 0; i < kQ; ++i)
#pragma unroll
        for (int m = 0; m < CPL; ++m) q[i][m] = 0.0;
    // GRAM: the four products U^T X of this wave's rows on the matrix cores, X = L (HVP) or the given
    // gradient (HESS), J, phi_p(u), psi(u) v.  Lane 16 q + c holds column c of row q of the wave's four
    // rows, which is the operand layout of v_mfma_f64_16x16x4f64 (A[c][q] = u, B[q][c] = x).
    dbl4 gacc[GRAM ? kGramQ : 1];
#pragma unroll
    for (int i = 0; i < (GRAM ? kGramQ : 1); ++i) gacc[i] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < RS; ++s) {
        const int rl = grp + s * NGRP;
        const bool valid = row0 + rl < a.n;
        const int64_t row = s_row[rl];
        const int64_t beg = valid ? first(rl) : 0, end = valid ? s_e[rl] : 0;
        const bool light = valid && (end - s_b[rl]) <= a.light_max;
        const int64_t len = light ? end - beg : 0;
        const uint32_t own = valid ? (uint32_t)row : 0u;
        const RowPre cur = nxt;
        if (s + 1 < RS) nxt = prefetch(rl + NGRP);
        uint32_t ou = cur.ou, ov = cur.ov;
        T wl = cur.wl;
        const int nch = (int)((len + G - 1) / G);
        T Ls[CPL], Js[CPL], Ns[CPL];
#pragma unroll
        for (int m = 0; m < CPL; ++m) Ls[m] = Js[m] = Ns[m] = 0;
        for (int ch = 0; ch < nch; ++ch) {
            const int64_t rem = len - (int64_t)ch * G;
            const int cnt = rem <= 0 ? 0 : (rem < G ? (int)rem : G);
            // offsets of the row's next chunk, loaded while this chunk's gathers are in flight
            uint32_t ou2 = own * a.ldu_b, ov2 = own * a.ldv_b;
            T wl2 = (T)0;
            if (ch + 1 < nch) {
                const int64_t c1 = beg + (int64_t)(ch + 1) * G;
                if (c1 + gl < end) {
                    const uint32_t j2 = (uint32_t)a.col[c1 + gl];
                    ou2 = j2 * a.ldu_b;
                    ov2 = j2 * a.ldv_b;
                    wl2 = (T)a.w[c1 + gl];
                }
            }
            constexpr int NBAT = light_batches<T, K, MODE>();
            constexpr int BU = NU / NBAT;
            static_for<0, NBAT>([&](auto bc) {
                constexpr int b0 = decltype(bc)::value * BU;
                T uj[BU][CPL], vj[BU][CPL];
                static_for<0, BU>([&](auto uc) {
                    constexpr int r = decltype(uc)::value;
                    constexpr int u = b0 + r;
#pragma unroll
                    for (int m = 0; m < CPL; ++m) {
                        uj[r][m] = cur.ui[m];
                        vj[r][m] = cur.vi[m];
                    }
                    if (u * EPR < cnt) {
                        const uint32_t bu = (uint32_t)edge_bcast<G, EPR, u>((int32_t)ou, e, lane);
                        const uint32_t bv = mode_v(MODE) ? (uint32_t)edge_bcast<G, EPR, u>((int32_t)ov, e, lane) : 0u;
#pragma unroll
                        for (int m = 0; m < CPL; ++m) {
                            uj[r][m] = bload<T>(rU, bu + cb[m]);
                            if (mode_v(MODE)) vj[r][m] = bload<T>(rV, bv + cb[m]);
                        }
                    }
                });
                static_for<0, BU>([&](auto uc) {
                    constexpr int r = decltype(uc)::value;
                    constexpr int u = b0 + r;
                    if (u * EPR < cnt) {
                        const T wv = edge_bcast_val<T, G, EPR, u>(wl, e, lane);
#pragma unroll
                        for (int m = 0; m < CPL; ++m)
                            Term<T, MODE, FLOOR>::apply(pw, a.epsc, cur.ui[m], uj[r][m], cur.vi[m], vj[r][m], wv,
                                                        Ls[m], Js[m], Ns[m]);
                    }
                });
            });
            ou = ou2;
            ov = ov2;
            wl = wl2;
        }
#pragma unroll
        for (int m = 0; m < CPL; ++m) {
            if (EPR > 1) {
#pragma unroll
                for (int o = KL; o < G; o <<= 1) {
                    if (mode_l(MODE)) Ls[m] += __shfl_xor(Ls[m], o);
                    if (mode_v(MODE)) Js[m] += __shfl_xor(Js[m], o);
                }
            }
            q[0][m] += (double)Ns[m];
            const T ui = cur.ui[m], vi = cur.vi[m];
            const T hi = pw(fabs(ui));
            const T phi = hi * ui;  // phi_p(u_i)
            // HESS: g_i read here (not held through the row); own is row 0 past the last row
            const T gi = MODE == HESS ? bload<T>(rG, own * a.ldg_b + cb[m]) : T(0);
            if constexpr (GRAM) {
                const double A = (light && c < a.k) ? (double)ui : 0.0;
                gacc[0] = mfma_f64(A, MODE == HESS ? (double)gi : (double)Ls[m], gacc[0]);
                gacc[1] = mfma_f64(A, (double)Js[m], gacc[1]);
                gacc[2] = mfma_f64(A, (double)phi, gacc[2]);
                gacc[3] = mfma_f64(A, (double)(fmin(hi, a.epsc) * vi), gacc[3]);
            }
            if (valid && e == 0) {
                q[1][m] += (double)(phi * ui);
                if (mode_v(MODE)) q[2][m] += (double)phi * (double)vi;
                if (MODE == HVP && light) q[3][m] += (double)Ls[m] * (double)vi;
                if (MODE == HESS) q[3][m] += (double)gi * (double)vi;  // g^T v over every row
                const int cm = c + m * KL;
                if (light && cm < a.k) {
                    if (mode_l(MODE)) a.L[row * a.ldl + cm] = Ls[m];
                    if (mode_v(MODE)) a.J[row * a.ldj + cm] = Js[m];
                }
            }
        }
    }
    // sum the FP64 accumulators over the lanes of each column and write the block's partial row
#pragma unroll
    for (int o = KL; o < 64; o <<= 1)
#pragma unroll
        for (int i = 0; i < kQ; ++i)
#pragma unroll
            for (int m = 0; m < CPL; ++m) q[i][m] += __shfl_xor(q[i][m], o);
    const int wave = tid >> 6;
    if (lane < KL)
#pragma unroll
        for (int i = 0; i < kQ; ++i)
#pragma unroll
            for (int m = 0; m < CPL; ++m) s_red[wave][i][lane + m * KL] = q[i][m];
    __syncthreads();
    double *prow = a.partials + (int64_t)blockIdx.x * kQ * a.k;
    for (int t = tid; t < kQ * K; t += kBlock) {
        const int i = t / K, cc = t % K;
        double sum = 0.0;
#pragma unroll
        for (int wv = 0; wv < kBlock / 64; ++wv) sum += s_red[wv][i][cc];
        if (cc < a.k) prow[i * a.k + cc] = sum;
    }
    if constexpr (GRAM) {  // the four waves' products added in wave order: one partial per tile
        dbl4 acc[kGramQ][1][1];
#pragma unroll
        for (int i = 0; i < kGramQ; ++i) acc[i][0][0] = gacc[i];
        gram_mfma_reduce<16, kGramQ>(acc, s_gred, a.k, a.gpart + (int64_t)blockIdx.x * kGramQ * a.k * a.k);
    }
}

// Heavy rows: chunks of at most PSPEC_CHUNK edges handed out in a fixed order to persistent waves.
// Workgroup b first serves column segment s = b % kSegs (the XCD it runs on): its waves take that
// segment's chunks in turn, so one XCD's L2 only ever holds neighbour rows of one segment; then every
// wave W of the grid takes the shared list's chunks W, W + NW, W + 2 NW, ...  (The objective walks the
// whole list that way, see below.)  A wave stages its chunk's neighbour
// byte offsets and weights in its own slice of LDS (no workgroup barrier), runs ES = 64 / K edge
// slots of K column lanes with UNR gathers in flight per lane (slots past the chunk gather the row
// itself with weight 0, so every load is unconditional), adds the slots up with cross-lane sums,
// writes the chunk's rows (or its scratch row when the row spans several chunks) and carries the
// FP64 column sums of w |x|^p and L_i v_i from chunk to chunk.  Each workgroup writes one partial
// row, its waves added in order, so the result does not depend on timing.
template <typename T, typename WT, int K, int MODE, int UNR, bool FLOOR = false>
__global__ __launch_bounds__(kBlock) void edge_heavy(EdgeArgs<T, WT> a) {
    constexpr int KW = K < 64 ? K : 64;  // column lanes of an edge slot
    constexpr int ES = 64 / KW;          // edge slots per wave
    constexpr int NWB = kBlock / 64;     // waves per workgroup
    __shared__ uint32_t s_ou[NWB][PSPEC_CHUNK], s_ov[NWB][PSPEC_CHUNK];  // neighbour byte offsets into U, V
    __shared__ T s_w[NWB][PSPEC_CHUNK];
    __shared__ double s_acc[NWB][2][KW];
    __shared__ double s_pow[sizeof(T) == 8 ? kPowTabLen : 1];
    PowM2<T> pw = a.pw;  // a local copy (taking the address of the argument block would move it to scratch)
    stage_pow(pw, s_pow);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = lane % KW, e = lane / KW;
    const int cl = c < a.k ? c : a.k - 1;
    const uint32_t cb = (uint32_t)cl * (uint32_t)sizeof(T);
    const auto rU = make_rsrc(a.U, a.U_bytes);
    const auto rV = make_rsrc(a.V, a.V_bytes);
    double Nacc = 0.0, Sacc = 0.0;
    auto chunk = [&](int64_t ci) {
        const Chunk ch = a.chunks[ci];
        int64_t cbeg = ch.beg;
        if constexpr (MODE == OBJ) {
            if (a.ustart != nullptr) {
                const int64_t us = a.ustart[ch.row];
                cbeg = us > cbeg ? us : cbeg;
            }
        }
        const int len = ch.end > cbeg ? (int)(ch.end - cbeg) : 0;
        if (MODE == OBJ && len == 0) return;  // no entry j > i in this chunk
        for (int t0 = 0; t0 < len; t0 += 4 * 64) {  // four ids per lane in flight
            uint32_t jj[4];
            WT ww[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + 64 * u + lane;
                const int64_t src = cbeg + (t < len ? t : len - 1);
                jj[u] = (uint32_t)a.col[src];
                ww[u] = a.w[src];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                pin(jj[u]);
                pin(ww[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + 64 * u + lane;
                if (t < len) {
                    s_ou[wv][t] = jj[u] * a.ldu_b;
                    s_ov[wv][t] = jj[u] * a.ldv_b;
                    s_w[wv][t] = (T)ww[u];
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t row = (uint32_t)ch.row;
        const uint32_t own_u = row * a.ldu_b + cb, own_v = row * a.ldv_b + cb;
        const T ui = bload<T>(rU, own_u);
        const T vi = mode_v(MODE) ? bload<T>(rV, own_v) : T(0);
        T Ls = 0, Js = 0, Ns = 0;
        for (int base = 0; base < len; base += ES * UNR) {
            // all staged offsets of the batch are read before any is used (see pin)
            uint32_t ou[UNR], ov[UNR];
            T uj[UNR], vj[UNR], wt[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int idx = base + u * ES + e;
                const int ix = idx < len ? idx : 0;
                ou[u] = s_ou[wv][ix];
                if (mode_v(MODE)) ov[u] = s_ov[wv][ix];
                wt[u] = s_w[wv][ix];
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                pin(ou[u]);
                if (mode_v(MODE)) pin(ov[u]);
                pin(wt[u]);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const bool ok = base + u * ES + e < len;
                wt[u] = ok ? wt[u] : T(0);
                uj[u] = bload<T>(rU, ok ? ou[u] + cb : own_u);
                if (mode_v(MODE)) vj[u] = bload<T>(rV, ok ? ov[u] + cb : own_v);
                else vj[u] = T(0);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u)
                Term<T, MODE, FLOOR>::apply(pw, a.epsc, ui, uj[u], vi, vj[u], wt[u], Ls, Js, Ns);
        }
        double L = (double)Ls, J = (double)Js, N = (double)Ns;
#pragma unroll
        for (int o = KW; o < 64; o <<= 1) {
            L += __shfl_xor(L, o);
            if (mode_v(MODE)) J += __shfl_xor(J, o);
            N += __shfl_xor(N, o);
        }
        if (e == 0 && c < a.k) {
            if (ch.slot < 0) {
                if (mode_l(MODE)) a.L[(int64_t)row * a.ldl + c] = (T)L;
                if (mode_v(MODE)) a.J[(int64_t)row * a.ldj + c] = (T)J;
            } else {
                a.scratch[((int64_t)ch.slot * 2 + 0) * a.k_max + c] = L;
                a.scratch[((int64_t)ch.slot * 2 + 1) * a.k_max + c] = J;
            }
            Nacc += N;
            if (MODE == HVP) Sacc += L * (double)vi;
        }
        // the next chunk's staging must not overtake this chunk's LDS reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    const int64_t NW = (int64_t)gridDim.x * NWB;
    if constexpr (MODE == OBJ) {
        // The objective visits only the entries above the diagonal, and the column segments hold
        // very unequal shares of those (segment s keeps an entry only when its row id is below the
        // column), so segment-bound workgroups would idle on the low segments: the whole chunk list
        // is walked with one stride instead.
        for (int64_t ci = (int64_t)blockIdx.x * NWB + wv; ci < a.n_chunks; ci += NW) chunk(ci);
    } else {
        {  // this workgroup's column segment (gridDim.x is a multiple of kSegs)
            const int sg = blockIdx.x % kSegs;
            const int64_t step = (int64_t)(gridDim.x / kSegs) * NWB;
            for (int64_t ci = a.seg_base[sg] + (int64_t)(blockIdx.x / kSegs) * NWB + wv; ci < a.seg_base[sg + 1];
                 ci += step)
                chunk(ci);
        }
        for (int64_t ci = a.seg_base[kSegs] + (int64_t)blockIdx.x * NWB + wv; ci < a.n_chunks; ci += NW) chunk(ci);
    }
    if (e == 0) {
        s_acc[wv][0][c] = Nacc;
        s_acc[wv][1][c] = Sacc;
    }
    __syncthreads();
    const int tid = threadIdx.x;
    if (tid < a.k) {
        double N = 0.0, S = 0.0;
        for (int w = 0; w < NWB; ++w) {
            N += s_acc[w][0][tid];
            S += s_acc[w][1][tid];
        }
        double *prow = a.partials + (a.part_base + blockIdx.x) * kQ * a.k;
        prow[0 * a.k + tid] = N;
        prow[1 * a.k + tid] = 0.0;
        prow[2 * a.k + tid] = 0.0;
        prow[3 * a.k + tid] = S;
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
    if (mode_l(MODE)) L[(int64_t)sp.row * ldl + c] = (T)Ls;
    if (mode_v(MODE)) J[(int64_t)sp.row * ldj + c] = (T)Js;
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
                                                      double *__restrict__ F, bool rank2, bool b_direct,
                                                      double nscale) {
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
        const double N = nscale * s[0 * k + tid], D = s[1 * k + tid], av = s[2 * k + tid], S = s[3 * k + tid];
        const double Fl = N / D, pD = p / D;
        sc[SC_N * k_max + tid] = N;
        sc[SC_D * k_max + tid] = D;
        sc[SC_F * k_max + tid] = Fl;
        sc[SC_PD * k_max + tid] = pD;
        // without the rank-2 part of the Hessian the epilogue's g a + phi b term is zero
        sc[SC_A * k_max + tid] = rank2 ? av : 0.0;
        // b = g^T v: from L^T v (HVP) or summed from the given gradient (HESS)
        sc[SC_B * k_max + tid] = rank2 ? (b_direct ? S : pD * (S - Fl * av)) : 0.0;
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

// Per-column scalars of the epilogue, read from Graph::scalars.
struct ColScalars {
    double pD, F, a, b;
};
__device__ __forceinline__ ColScalars col_scalars(const double *__restrict__ sc, int k_max, int c) {
    return {sc[SC_PD * k_max + c], sc[SC_F * k_max + c], sc[SC_A * k_max + c], sc[SC_B * k_max + c]};
}

// Epilogue of one entry: from u_i, v_i and the raw rows L_i = (Delta_p u)_i, J_i (edge part of the
// Hessian over p - 1), the gradient g = (p/D)(L - F phi_p(u)) and
// HV = (p/D)((p-1) J - F (p-1) psi(u) v - g a - phi_p(u) b), both rounded to T.  Every kernel that
// forms these entries goes through this function, so they agree bit for bit; contraction into
// FMAs is off here, since the compiler would otherwise fuse differently in different kernels.  In
// HESS mode l is the given gradient g itself (U fixed), and only HV is formed.
template <typename T, int MODE>
__device__ __forceinline__ void epilogue(const PowM2<T> &pw, T epsc, double p, const ColScalars &s, T u, T v, T l,
                                         T j, T &gout, T &hout) {
#pragma clang fp contract(off)
    const T h = pw(fabs(u));
    const T phi = h * u;
    const double g = MODE == HESS ? (double)l : s.pD * ((double)l - s.F * (double)phi);
    gout = (T)g;
    if (mode_v(MODE)) {
        const T psi = fmin(h, epsc);
        const double hv = s.pD * ((p - 1.0) * (double)j - s.F * (p - 1.0) * (double)psi * (double)v - g * s.a -
                                  (double)phi * s.b);
        hout = (T)hv;
    }
}

// Epilogue over all rows: G (and HV) in place of the raw rows; K lanes per row.
template <typename T, int K, int MODE>
__global__ __launch_bounds__(kBlock) void finalize(int64_t n, int k, const T *__restrict__ U, int64_t ldu,
                                                 const T *__restrict__ V, int64_t ldv, T *__restrict__ G, int64_t ldg,
                                                 T *__restrict__ HV, int64_t ldh, PowM2<T> pw, T epsc, double p,
                                                 const double *__restrict__ sc, int k_max) {
    __shared__ double s_pow[sizeof(T) == 8 ? kPowTabLen : 1];
    stage_pow(pw, s_pow);
    const int64_t stride = (int64_t)gridDim.x * (kBlock / K);
    const int c = threadIdx.x % K;
    if (c >= k) return;
    const ColScalars cs = col_scalars(sc, k_max, c);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / K) + threadIdx.x / K; i < n; i += stride) {
        const T v = mode_v(MODE) ? V[i * ldv + c] : T(0);
        const T j = mode_v(MODE) ? HV[i * ldh + c] : T(0);
        T g, hv;
        epilogue<T, MODE>(pw, epsc, p, cs, U[i * ldu + c], v, G[i * ldg + c], j, g, hv);
        if (MODE != HESS) G[i * ldg + c] = g;  // in HESS mode G is the given gradient, read only
        if (mode_v(MODE)) HV[i * ldh + c] = hv;
    }
}

// Fused epilogue and Gram matrices of the Riemannian Hessian-vector product: per workgroup (a fixed
// grid of kDenseBlocks, each over a contiguous row range) the FP64 partials of U^T G and U^T HV on
// the matrix cores, with G and HV formed from the raw rows L, J by the epilogue above and never
// stored.  Rows, groups and the MFMA sequence are those of the stand-alone Gram kernel, so the sums
// equal the Gram matrices of the finalized G and HV bit for bit.  In HESS mode L is the given
// gradient.
template <typename T, int K, int MODE = HVP>
__global__ __launch_bounds__(kBlock) void finalize_gram(int64_t n, int k, const T *__restrict__ U, int64_t ldu,
                                                      const T *__restrict__ V, int64_t ldv, const T *__restrict__ L,
                                                      int64_t ldl, const T *__restrict__ J, int64_t ldj, PowM2<T> pw,
                                                      T epsc, double p, const double *__restrict__ sc, int k_max,
                                                      double *__restrict__ part) {
    constexpr int CT = mf_tiles<K>();
    __shared__ double s_red[4][4][64];
    __shared__ double s_pow[sizeof(T) == 8 ? kPowTabLen : 1];
    stage_pow(pw, s_pow);
    const int c = threadIdx.x & 15;
    ColScalars cs[CT];  // this lane's columns 16 t + c
#pragma unroll
    for (int t = 0; t < CT; ++t)
        cs[t] = 16 * t + c < k ? col_scalars(sc, k_max, 16 * t + c) : ColScalars{0.0, 0.0, 0.0, 0.0};
    int64_t r0, r1;
    block_rows(n, r0, r1);
    dbl4 acc[2][CT][CT];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int ta = 0; ta < CT; ++ta)
#pragma unroll
            for (int tb = 0; tb < CT; ++tb) acc[m][ta][tb] = dbl4{0.0, 0.0, 0.0, 0.0};
    struct Raw {
        T u[CT], v[CT], l[CT], j[CT];
        __device__ void pin() {
            pin_all(u);
            pin_all(v);
            pin_all(l);
            pin_all(j);
        }
    };
    auto load = [&](int64_t row, int cl, Raw &raw) {
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int col = 16 * t + cl;
            raw.u[t] = clamped_load(U, ldu, row, r1, col, k);
            raw.v[t] = clamped_load(V, ldv, row, r1, col, k);
            raw.l[t] = clamped_load(L, ldl, row, r1, col, k);
            raw.j[t] = clamped_load(J, ldj, row, r1, col, k);
        }
    };
    auto finish = [&](int64_t row, int cl, const Raw &raw, T(&a)[CT], T(&b)[2][CT]) {
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const bool ok = row < r1 && 16 * t + cl < k;
            T g, hv;
            epilogue<T, MODE>(pw, epsc, p, cs[t], raw.u[t], raw.v[t], raw.l[t], raw.j[t], g, hv);
            a[t] = ok ? raw.u[t] : T(0);
            b[0][t] = ok ? g : T(0);
            b[1][t] = ok ? hv : T(0);
        }
    };
    gram_mfma_rows<T, K, 2, gram_groups<2>(), Raw>(r0, r1, load, finish, acc);
    gram_mfma_reduce<K, 2>(acc, s_red, k, part + (int64_t)blockIdx.x * 2 * k * k);
}

// Projection of the fused Riemannian Hessian-vector product on the matrix cores:
//   RG = G - U MG,   RH = HV - U MH - V MG,   MG = U^T G, MH = U^T HV,
// with G and HV formed again from the raw rows (held in RG and RH on entry, overwritten in place) by
// the shared epilogue.  The products follow the MFMA sequence of the stand-alone projection (U then
// V, each in k order), so the outputs equal pspec_project's bit for bit.  In HESS mode RG holds the
// given gradient (read only) and only RH is written.
template <typename T, int K, bool VEC, int MODE = HVP>
__global__ __launch_bounds__(kBlock) void apply_rhvp(int64_t n, int k, const T *__restrict__ U, int64_t ldu,
                                                   const T *__restrict__ V, int64_t ldv, T *__restrict__ RG,
                                                   int64_t ldrg, T *__restrict__ RH, int64_t ldrh, PowM2<T> pw, T epsc,
                                                   double p, const double *__restrict__ sc, int k_max,
                                                   const double *__restrict__ MG, const double *__restrict__ MH) {
    constexpr int CT = mf_tiles<K>(), KS = mf_steps<K>();
    __shared__ double s_pow[sizeof(T) == 8 ? kPowTabLen : 1];
    stage_pow(pw, s_pow);
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    double mg[CT][KS], mh[CT][KS];
    load_mf_operand<K>(MG, k, mg);
    load_mf_operand<K>(MH, k, mh);
    ColScalars cs[CT];  // this lane's output columns 16 t + c
#pragma unroll
    for (int t = 0; t < CT; ++t)
        cs[t] = 16 * t + c < k ? col_scalars(sc, k_max, 16 * t + c) : ColScalars{0.0, 0.0, 0.0, 0.0};
    constexpr int TPI = 1;  // one tile per iteration: this kernel already holds four rows per lane
    const int64_t stride = mf_tile_stride();
    for (int64_t tile0 = mf_first_tile(); tile0 * 16 < n; tile0 += TPI * stride) {
        T ua[TPI][KS], va[TPI][KS];  // operand chunks of row row0 + c
        T u[TPI][CT][4], v[TPI][CT][4], l[TPI][CT][4], j[TPI][CT][4];  // (row0 + 4 i + q, 16 t + c)
#pragma unroll
        for (int s = 0; s < TPI; ++s) {
            const int64_t row0 = (tile0 + s * stride) * 16;
            load_mf_chunk<T, K, VEC>(U, ldu, row0 + c, n, k, ua[s]);
            load_mf_chunk<T, K, VEC>(V, ldv, row0 + c, n, k, va[s]);
#pragma unroll
            for (int t = 0; t < CT; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t r = row0 + 4 * i + q;
                    const int col = 16 * t + c;
                    u[s][t][i] = clamped_load(U, ldu, r, n, col, k);
                    v[s][t][i] = clamped_load(V, ldv, r, n, col, k);
                    l[s][t][i] = clamped_load<T>(RG, ldrg, r, n, col, k);
                    j[s][t][i] = clamped_load<T>(RH, ldrh, r, n, col, k);
                }
        }
#pragma unroll
        for (int s = 0; s < TPI; ++s) {
            pin_all(ua[s]);
            pin_all(va[s]);
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                pin_all(u[s][t]);
                pin_all(v[s][t]);
                pin_all(l[s][t]);
                pin_all(j[s][t]);
            }
        }
#pragma unroll
        for (int s = 0; s < TPI; ++s) {
            const int64_t row0 = (tile0 + s * stride) * 16;
            mask_mf_chunk<T, K>(row0 + c, n, k, ua[s]);
            mask_mf_chunk<T, K>(row0 + c, n, k, va[s]);
            dbl4 acc[CT];
            if constexpr (MODE == HVP) {
#pragma unroll
                for (int t = 0; t < CT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
                mf_products<T, K>(ua[s], -1.0, mg, acc);
#pragma unroll
                for (int t = 0; t < CT; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t r = row0 + 4 * i + q;
                        const int col = 16 * t + c;
                        T g, hv;
                        epilogue<T, GRAD>(pw, epsc, p, cs[t], u[s][t][i], v[s][t][i], l[s][t][i], j[s][t][i], g, hv);
                        if (r < n && col < k) RG[r * ldrg + col] = (T)fma(1.0, (double)g, acc[t][i]);
                    }
            }
#pragma unroll
            for (int t = 0; t < CT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
            mf_products<T, K>(ua[s], -1.0, mh, acc);
            mf_products<T, K>(va[s], -1.0, mg, acc);
#pragma unroll
            for (int t = 0; t < CT; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t r = row0 + 4 * i + q;
                    const int col = 16 * t + c;
                    T g, hv;
                    epilogue<T, MODE>(pw, epsc, p, cs[t], u[s][t][i], v[s][t][i], l[s][t][i], j[s][t][i], g, hv);
                    if (r < n && col < k) RH[r * ldrh + col] = (T)fma(1.0, (double)hv, acc[t][i]);
                }
        }
    }
}

// Gathers in flight per lane in the heavy-chunk kernel: 32 edges per wave (64 / K edge slots), at
// most 8 per lane (more registers per wave cost more in resident waves than they gain); at most 4 in
// FP64, whose pass is bound by the arithmetic of the power, not by the gathers.
template <typename T, int K>
constexpr int heavy_unroll() {
    constexpr int slots = K < 64 ? 64 / K : 1;
    constexpr int cap = sizeof(T) == 8 ? 4 : 8;
    return 32 / slots > cap ? cap : (32 / slots < 2 ? 2 : 32 / slots);
}

// Workgroups of the persistent heavy-chunk kernel for this element type and k: as many as stay
// resident together (from the occupancy of the HVP variant, the hungriest, so every mode shares
// the partition of the chunks and the per-column sums agree bit for bit across entry points), at
// most kHeavyPerCUMax per CU and one per four chunks.
template <typename T, typename WT, int K>
int64_t heavy_grid(const Graph *g) {
    static int per_cu = 0;  // per instantiation; every thread computes the same value
    if (per_cu == 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, edge_heavy<T, WT, K, HVP, heavy_unroll<T, K>()>,
                                                         kBlock, 0) != hipSuccess ||
            v < 1)
            v = 1;
        per_cu = v < kHeavyPerCUMax ? v : kHeavyPerCUMax;
    }
    if (g->n_chunks == 0) return 0;
    const int64_t want = (g->n_chunks + 3) / 4, cap = (int64_t)per_cu * g->cus;
    int64_t grid = want < cap ? want : cap;
    grid = grid < g->heavy_grid_max ? grid : g->heavy_grid_max;  // the partial rows the workspace holds
    grid = grid / kSegs * kSegs;                                 // every segment served alike
    return grid > kSegs ? grid : kSegs;
}

unsigned grid_for(int64_t items, int64_t per_block, int64_t cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

// The edge pass proper: edge kernels, split-row combine and the reductions to the per-column
// scalars; L and J receive the raw rows.
template <typename T, typename WT, int K, int MODE, bool FLOOR = false, bool GRAM = false>
pspec_status edge_pass(Graph *g, int k, const T *U, int64_t ldu, const T *V, int64_t ldv, T *L, int64_t ldl, T *J, int64_t ldj,
               double p, double eps, double *F_col, double *F, hipStream_t s, bool rank2 = true,
               const T *Gc = nullptr, int64_t ldgc = 0) {
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
    a.Gc = Gc;
    a.ldg_b = (uint32_t)(ldgc * (int64_t)sizeof(T));
    a.G_bytes = Gc ? (uint32_t)block_extent(g->n, k, ldgc, sizeof(T)) : 0u;
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
    for (int sg = 0; sg <= kSegs; ++sg) a.seg_base[sg] = g->seg_chunk_base[sg];
    a.n_chunks = g->n_chunks;
    a.ustart = (MODE == OBJ && g->ascending) ? g->ustart : nullptr;
    a.gpart = GRAM ? g->gram_part : nullptr;
    a.lperm = (sizeof(T) == 8 || g->sorted_tiles) ? g->lperm : nullptr;
    if (g->ev_before) PSPEC_HIP(hipEventRecord(g->ev_before, s));
    edge_light<T, WT, K, MODE, FLOOR, GRAM><<<(unsigned)g->tiles, kBlock, 0, s>>>(a);
    const int64_t hb = heavy_grid<T, WT, K>(g);
    if (hb > 0) edge_heavy<T, WT, K, MODE, heavy_unroll<T, K>(), FLOOR><<<(unsigned)hb, kBlock, 0, s>>>(a);
    if (g->n_split > 0 && MODE != OBJ)
        combine_split<T, MODE><<<grid_for(g->n_split * k, kBlock, 1 << 30), kBlock, 0, s>>>(
            g->splits, g->n_split, g->chunk_scratch, k, g->k_max, L, ldl, J, ldj);
    if (g->ev_after) PSPEC_HIP(hipEventRecord(g->ev_after, s));
    const int W = kQ * k;
    reduce_stage1<<<kReduceSlices, kBlock, 0, s>>>(g->partials, g->tiles + hb, W, g->red1);
    // N = 1/2 sum over the stored entries, or the sum over the entries j > i
    reduce_stage2<<<1, kBlock, 0, s>>>(g->red1, W, k, p, g->scalars, g->k_max, F_col, F, rank2, MODE == HESS,
                                       a.ustart ? 1.0 : 0.5);
    return PSPEC_OK;
}

template <typename T, typename WT, int K, int MODE>
pspec_status launch_edges(Graph *g, int k, const T *U, int64_t ldu, const T *V, int64_t ldv, T *L, int64_t ldl, T *J,
                          int64_t ldj, double p, double eps, double *F_col, double *F, hipStream_t s, bool rank2) {
    const pspec_status st = edge_pass<T, WT, K, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s, rank2);
    if (st != PSPEC_OK) return st;
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

// The fused kernels run on the matrix cores for 16 <= k <= 32.  Below 16 the matrix-core layout pads
// the rows to 16 columns, so the two fused kernels would evaluate the epilogue (one power per
// entry, a long FP64 routine in the FP64 path) for the padding lanes too, and twice per entry; the
// stand-alone sequence evaluates it once per entry.  Wider blocks take the stand-alone path as well.
template <typename T, int K>
constexpr bool rhvp_fused() {
    return K >= 16 && K <= 32;
}

// Gram products of the heavy rows (more than PSPEC_LIGHT_MAX entries), which the light kernel leaves
// out: the same four products U^T X, U^T J, U^T phi_p(u), U^T (psi(u) v) over the rows of the shared
// chunk list (one chunk each) and of the split-row list, after the split rows are combined; X is L
// (HVP) or the given gradient (HESS).  Workgroup b takes a contiguous range of that row list.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void gram_heavy(const Chunk *__restrict__ glob, int64_t n_glob,
                                                   const Split *__restrict__ splits, int64_t n_split, int k,
                                                   const T *__restrict__ U, int64_t ldu, const T *__restrict__ V,
                                                   int64_t ldv, const T *__restrict__ X, int64_t ldx,
                                                   const T *__restrict__ J, int64_t ldj, PowM2<T> pw, T epsc,
                                                   double *__restrict__ part) {
    __shared__ double s_red[4][4][64];
    __shared__ double s_pow[sizeof(T) == 8 ? kPowTabLen : 1];
    stage_pow(pw, s_pow);
    int64_t r0, r1;
    block_rows(n_glob + n_split, r0, r1);
    auto row_of = [&](int64_t h) -> int64_t { return h < n_glob ? (int64_t)glob[h].row : (int64_t)splits[h - n_glob].row; };
    struct Raw {
        T u, v, x, j;
        __device__ void pin() {
            pspec::pin(u);
            pspec::pin(v);
            pspec::pin(x);
            pspec::pin(j);
        }
    };
    auto load = [&](int64_t h, int cl, Raw &raw) {
        const int64_t r = row_of(h < r1 ? h : r1 - 1);
        const int col = cl < k ? cl : k - 1;
        raw.u = U[r * ldu + col];
        raw.v = V[r * ldv + col];
        raw.x = X[r * ldx + col];
        raw.j = J[r * ldj + col];
    };
    auto finish = [&](int64_t h, int cl, const Raw &raw, T(&av)[1], T(&bv)[kGramQ][1]) {
        const T hi = pw(fabs(raw.u));
        av[0] = (h < r1 && cl < k) ? raw.u : T(0);
        bv[0][0] = raw.x;
        bv[1][0] = raw.j;
        bv[2][0] = hi * raw.u;
        bv[3][0] = fmin(hi, epsc) * raw.v;
    };
    dbl4 acc[kGramQ][1][1];
#pragma unroll
    for (int i = 0; i < kGramQ; ++i) acc[i][0][0] = dbl4{0.0, 0.0, 0.0, 0.0};
    gram_mfma_rows<T, 16, kGramQ, 4, Raw>(r0, r1, load, finish, acc);
    gram_mfma_reduce<16, kGramQ>(acc, s_red, k, part + (int64_t)blockIdx.x * kGramQ * k * k);
}

// out[g][e] = sum of part[q][e] over the contiguous range of q that group g = blockIdx.y of `groups`
// takes (rows of `len` doubles), in q order.
__global__ __launch_bounds__(kBlock) void sum_range(const double *__restrict__ part, int64_t P, int len, int groups,
                                                  double *__restrict__ out) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= len) return;
    const int64_t per = (P + groups - 1) / groups;
    const int64_t q0 = (int64_t)blockIdx.y * per, q1 = q0 + per < P ? q0 + per : P;
    double acc = 0.0;
    int64_t q = q0;
    for (; q + 8 <= q1; q += 8) {  // eight loads in flight, added in q order
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(q + u) * len + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; q < q1; ++q) acc += part[q * len + e];
    out[(int64_t)blockIdx.y * len + e] = acc;
}

// MG = U^T G and MH = U^T HV from the four Gram products (U^T X, U^T J, U^T phi, U^T (psi v)) and the
// per-column scalars, following the epilogue term by term: column l of G is (p/D)(L - F phi) (or the
// given gradient in HESS mode) and column l of HV is (p/D)((p-1) J - F (p-1) psi v - g a - phi b).
template <int MODE>
__global__ __launch_bounds__(kBlock) void gram_combine(const double *__restrict__ fin, int k, double p,
                                                     const double *__restrict__ sc, int k_max,
                                                     double *__restrict__ MG, double *__restrict__ MH,
                                                     double *__restrict__ MG_out) {
    const int kk = k * k;
    for (int t = threadIdx.x; t < kk; t += kBlock) {
        const ColScalars s = col_scalars(sc, k_max, t % k);
        const double GX = fin[t], GJ = fin[kk + t], GP = fin[2 * kk + t], GS = fin[3 * kk + t];
        const double mg = MODE == HESS ? GX : s.pD * (GX - s.F * GP);
        MG[t] = mg;
        MH[t] = s.pD * ((p - 1.0) * GJ - s.F * (p - 1.0) * GS - mg * s.a - GP * s.b);
        if (MG_out) MG_out[t] = mg;
    }
}

// Whether the Riemannian call forms its Gram products inside the edge pass (FP32, 9 <= k <= 16).
template <typename T, int K>
constexpr bool rhvp_gram_in_edge() {
    return sizeof(T) == 4 && K == kGramK;
}

// Riemannian gradient and Hessian-vector product on Gr(k, n).  Workspace: level-1 partials
// [kDenseBlocks][2][k*k], level-2 partials, then MG = U^T G and MH = U^T HV (k*k each).
// MODE = HVP: RG and RH from U and V.  MODE = HESS: RH only, at a U whose Euclidean gradient is given
// in RG (read only): the edge pass forms no L, and b = g^T v comes from the given gradient.
template <typename T, typename WT, int K, bool VEC, int MODE = HVP>
pspec_status launch_rhvp(Graph *g, int k, const T *U, int64_t ldu, const T *V, int64_t ldv, double p, double eps, T *RH,
                 int64_t ldrh, T *RG, int64_t ldrg, double *MG_out, double *F_col, double *ws, hipStream_t s) {
    const int64_t n = g->n;
    const size_t kk = (size_t)k * k;
    double *part = ws;
    double *mid = part + (size_t)kDenseBlocks * 2 * kk;
    double *Mw = mid + (size_t)(kDenseBlocks / kTreeFan) * 2 * kk;  // [MG | MH]
    PowM2<T> pw;
    pw.pm2 = (T)(p - 2.0);
    const T epsc = (T)std::pow(eps, p - 2.0);
    constexpr bool GE = rhvp_gram_in_edge<T, K>();
    if (GE && g->gram_part == nullptr) {
        set_error("rhvp: the graph handle holds no Gram area (k_max = %d)", g->k_max);
        return PSPEC_ERR_ARG;
    }
    const pspec_status st =
        MODE == HESS ? edge_pass<T, WT, K, HESS, false, GE>(g, k, U, ldu, V, ldv, nullptr, 0, RH, ldrh, p, eps, F_col,
                                                            nullptr, s, true, RG, ldrg)
                     : edge_pass<T, WT, K, HVP, false, GE>(g, k, U, ldu, V, ldv, RG, ldrg, RH, ldrh, p, eps, F_col,
                                                           nullptr, s);
    if (st != PSPEC_OK) return st;
    if constexpr (GE) {
        // light tiles' partials from the edge pass, then the heavy rows', then fixed-order sums
        const int len = kGramQ * (int)kk;
        double *gp = g->gram_part;
        const int64_t n_glob = g->n_chunks - g->seg_chunk_base[kSegs], nh = n_glob + g->n_split;
        const int64_t hb = nh == 0 ? 0 : std::min<int64_t>(kGramHeavyBlocks, (nh + 63) / 64);
        if (hb > 0)
            gram_heavy<T, MODE><<<(unsigned)hb, kBlock, 0, s>>>(g->chunks + g->seg_chunk_base[kSegs], n_glob, g->splits,
                                                                g->n_split, k, U, ldu, V, ldv, RG, ldrg, RH, ldrh, pw,
                                                                epsc, gp + g->tiles * len);
        double *mid1 = gp + (g->tiles + kGramHeavyBlocks) * len, *mid2 = mid1 + (int64_t)kGramMid * len;
        double *fin = mid2 + (int64_t)(kGramMid / kTreeFan) * len;
        const unsigned gx = (unsigned)((len + kBlock - 1) / kBlock);
        sum_range<<<dim3(gx, kGramMid), kBlock, 0, s>>>(gp, g->tiles + hb, len, kGramMid, mid1);
        sum_level<<<dim3(gx, kGramMid / kTreeFan), kBlock, 0, s>>>(mid1, kGramMid, len, len, mid2, nullptr);
        sum_level<<<dim3(gx, 1), kBlock, 0, s>>>(mid2, kGramMid / kTreeFan, len, len, fin, nullptr);
        gram_combine<MODE><<<1, kBlock, 0, s>>>(fin, k, p, g->scalars, g->k_max, Mw, Mw + kk, MG_out);
        apply_rhvp<T, K, VEC, MODE><<<mf_grid(n), kBlock, 0, s>>>(n, k, U, ldu, V, ldv, RG, ldrg, RH, ldrh, pw, epsc,
                                                                  p, g->scalars, g->k_max, Mw, Mw + kk);
    } else if constexpr (rhvp_fused<T, K>()) {
        finalize_gram<T, K, MODE><<<kDenseBlocks, kBlock, 0, s>>>(n, k, U, ldu, V, ldv, RG, ldrg, RH, ldrh, pw, epsc,
                                                                  p, g->scalars, g->k_max, part);
        sum_partials(part, (int)kk, mid, Mw, MG_out, s, 2 * (int64_t)kk);
        sum_partials(part + kk, (int)kk, mid, Mw + kk, nullptr, s, 2 * (int64_t)kk);
        apply_rhvp<T, K, VEC, MODE><<<mf_grid(n), kBlock, 0, s>>>(n, k, U, ldu, V, ldv, RG, ldrg, RH, ldrh, pw, epsc,
                                                                  p, g->scalars, g->k_max, Mw, Mw + kk);
    } else {  // wide rows: finalize, then the two projections with the stand-alone kernels, in place
        finalize<T, K, MODE><<<grid_for(n, kBlock / K, 65536), kBlock, 0, s>>>(n, k, U, ldu, V, ldv, RG, ldrg, RH,
                                                                                ldrh, pw, epsc, p, g->scalars,
                                                                                g->k_max);
        gram_partial<T, K, false, false><<<kDenseBlocks, kBlock, 0, s>>>(n, k, U, ldu, nullptr, 0, 0.0, RG, ldrg,
                                                                          part);
        sum_partials(part, (int)kk, mid, Mw, MG_out, s);
        gram_partial<T, K, false, false><<<kDenseBlocks, kBlock, 0, s>>>(n, k, U, ldu, nullptr, 0, 0.0, RH, ldrh,
                                                                          part);
        sum_partials(part, (int)kk, mid, Mw + kk, nullptr, s);
        if (MODE == HVP)
            launch_apply<T, K, VEC, false, false, true>(s, n, k, 1.0, RG, ldrg, U, ldu, nullptr, 0, 0.0, Mw, -1.0,
                                                        nullptr, 0, nullptr, 0.0, RG, ldrg);
        launch_apply<T, K, VEC, false, true, true>(s, n, k, 1.0, RH, ldrh, U, ldu, nullptr, 0, 0.0, Mw + kk, -1.0, V,
                                                   ldv, Mw, -1.0, RH, ldrh);
    }
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

template <typename T, typename WT, int MODE>
pspec_status dispatch_k(Graph *g, int k, const T *U, int64_t ldu, const T *V, int64_t ldv, T *L, int64_t ldl, T *J,
                        int64_t ldj, double p, double eps, double *F_col, double *F, hipStream_t s, bool rank2) {
    switch (pad_k(k)) {
        case 4: return launch_edges<T, WT, 4, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s, rank2);
        case 8: return launch_edges<T, WT, 8, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s, rank2);
        case 16: return launch_edges<T, WT, 16, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s, rank2);
        case 32: return launch_edges<T, WT, 32, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s, rank2);
        case 64: return launch_edges<T, WT, 64, MODE>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, p, eps, F_col, F, s, rank2);
        default: set_error("unsupported k = %d", k); return PSPEC_ERR_UNSUPPORTED;
    }
}

template <int MODE>
pspec_status dispatch(Graph *g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V, int64_t ldv,
                      void *L, int64_t ldl, void *J, int64_t ldj, double p, double eps, double *F_col, double *F,
                      hipStream_t s, bool rank2 = true) {
    if (dt == PSPEC_F32)
        return dispatch_k<float, float, MODE>(g, k, (const float *)U, ldu, (const float *)V, ldv, (float *)L, ldl,
                                              (float *)J, ldj, p, eps, F_col, F, s, rank2);
    if (g->wtype == PSPEC_F32)
        return dispatch_k<double, float, MODE>(g, k, (const double *)U, ldu, (const double *)V, ldv, (double *)L,
                                               ldl, (double *)J, ldj, p, eps, F_col, F, s, rank2);
    return dispatch_k<double, double, MODE>(g, k, (const double *)U, ldu, (const double *)V, ldv, (double *)L, ldl,
                                            (double *)J, ldj, p, eps, F_col, F, s, rank2);
}

template <typename T, typename WT, int K, int MODE>
pspec_status rhvp_layout(Graph *g, int k, const T *U, int64_t ldu, const T *V, int64_t ldv, double p, double eps,
                         T *RH, int64_t ldrh, T *RG, int64_t ldrg, double *MG, double *F_col, double *ws,
                         hipStream_t s) {
    if (rows_vectorisable<T, K>(k, {{U, ldu}, {V, ldv}, {RH, ldrh}, {RG, ldrg}}))
        return launch_rhvp<T, WT, K, true, MODE>(g, k, U, ldu, V, ldv, p, eps, RH, ldrh, RG, ldrg, MG, F_col, ws, s);
    return launch_rhvp<T, WT, K, false, MODE>(g, k, U, ldu, V, ldv, p, eps, RH, ldrh, RG, ldrg, MG, F_col, ws, s);
}

template <typename T, typename WT, int MODE>
pspec_status rhvp_k(Graph *g, int k, const void *U, int64_t ldu, const void *V, int64_t ldv, double p, double eps,
                    void *RH, int64_t ldrh, void *RG, int64_t ldrg, double *MG, double *F_col, double *ws,
                    hipStream_t s) {
#define PSPEC_RHVP_K(KK)                                                                                         \
    case KK:                                                                                                     \
        return rhvp_layout<T, WT, KK, MODE>(g, k, (const T *)U, ldu, (const T *)V, ldv, p, eps, (T *)RH, ldrh,   \
                                            (T *)RG, ldrg, MG, F_col, ws, s);
    switch (pad_k(k)) {
        PSPEC_RHVP_K(4)
        PSPEC_RHVP_K(8)
        PSPEC_RHVP_K(16)
        PSPEC_RHVP_K(32)
        PSPEC_RHVP_K(64)
        default: set_error("unsupported k = %d", k); return PSPEC_ERR_UNSUPPORTED;
    }
#undef PSPEC_RHVP_K
}

// The gather-floor reference: the HVP edge pass (FP32 data, same kernels, grid, loads and stores)
// with the arithmetic of every edge term replaced by a sum of the gathered values.
pspec_status gather_floor(Graph *g, int k, const float *U, int64_t ldu, const float *V, int64_t ldv, float *L,
                          int64_t ldl, float *J, int64_t ldj, hipStream_t s) {
#define PSPEC_FLOOR_K(KK)                                                                                        \
    case KK:                                                                                                     \
        st = edge_pass<float, float, KK, HVP, true>(g, k, U, ldu, V, ldv, L, ldl, J, ldj, 1.5, 1.0, nullptr,      \
                                                    nullptr, s);                                                 \
        break;
    pspec_status st = PSPEC_OK;
    switch (pad_k(k)) {
        PSPEC_FLOOR_K(4)
        PSPEC_FLOOR_K(8)
        PSPEC_FLOOR_K(16)
        PSPEC_FLOOR_K(32)
        PSPEC_FLOOR_K(64)
        default: set_error("unsupported k = %d", k); return PSPEC_ERR_UNSUPPORTED;
    }
#undef PSPEC_FLOOR_K
    if (st != PSPEC_OK) return st;
    PSPEC_HIP(hipGetLastError());
    return PSPEC_OK;
}

// Host-side argument checks shared by the entry points.
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

// ---- the allocation-free Riemannian call ----------------------------------------------------
// The dense workspace of pspec_rhvp_static is a file-scope device array, one copy per GPU, sized for
// k <= PSPEC_STATIC_K_MAX.  Host code never passes its name to a kernel: the device address of each
// GPU's copy comes from hipGetSymbolAddress, taken once per device with that device current.
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[dense_ws_doubles(PSPEC_STATIC_K_MAX)];
std::mutex g_scratch_mutex;
double *g_scratch_addr[kMaxDevices] = {};

pspec_status static_scratch(double **out, const char *who) {
    int dev = 0;
    PSPEC_HIP(hipGetDevice(&dev));
    PSPEC_UNSUP(dev >= 0 && dev < kMaxDevices, "%s: device %d outside 0..%d", who, dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_addr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("%s: hipGetSymbolAddress(scratch) on device %d: %s", who, dev, hipGetErrorString(e));
            return PSPEC_ERR_HIP;
        }
        g_scratch_addr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_addr[dev];
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

static pspec_status hvp_entry(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                              int64_t ldv, double p, double eps, void *HV, int64_t ldh, void *G, int64_t ldg,
                              double *F_col, pspec_stream stream, bool rank2, const char *who, bool floor = false) {
    clear_error();
    pspec_status st = check_common(g, dt, k, U, ldu, p, who);
    if (st != PSPEC_OK) return st;
    PSPEC_ARG(eps > 0.0 && std::isfinite(eps), "%s: eps = %g must be positive", who, eps);
    if ((st = check_out(g, dt, k, V, ldv, "V", who)) != PSPEC_OK) return st;
    if ((st = check_out(g, dt, k, HV, ldh, "HV", who)) != PSPEC_OK) return st;
    if ((st = check_out(g, dt, k, G, ldg, "G", who)) != PSPEC_OK) return st;
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    const int64_t n = g->n;
    PSPEC_ARG(!blocks_overlap(HV, ldh, U, ldu, n, k, es) && !blocks_overlap(HV, ldh, V, ldv, n, k, es) &&
                  !blocks_overlap(G, ldg, U, ldu, n, k, es) && !blocks_overlap(G, ldg, V, ldv, n, k, es) &&
                  !blocks_overlap(G, ldg, HV, ldh, n, k, es),
              "%s: HV and G must not overlap U, V or each other", who);
    if (floor)
        return gather_floor(g, k, (const float *)U, ldu, (const float *)V, ldv, (float *)G, ldg, (float *)HV, ldh,
                            reinterpret_cast<hipStream_t>(stream));
    return dispatch<HVP>(g, dt, k, U, ldu, V, ldv, G, ldg, HV, ldh, p, eps, F_col, nullptr,
                         reinterpret_cast<hipStream_t>(stream), rank2);
}

extern "C" pspec_status pspec_hvp(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                                  int64_t ldv, double p, double eps, void *HV, int64_t ldh, void *G, int64_t ldg,
                                  double *F_col, pspec_stream stream) {
    return hvp_entry(g, dt, k, U, ldu, V, ldv, p, eps, HV, ldh, G, ldg, F_col, stream, true, "hvp");
}

extern "C" pspec_status pspec_hvp_sparse(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu,
                                         const void *V, int64_t ldv, double p, double eps, void *HV, int64_t ldh,
                                         void *G, int64_t ldg, double *F_col, pspec_stream stream) {
    return hvp_entry(g, dt, k, U, ldu, V, ldv, p, eps, HV, ldh, G, ldg, F_col, stream, false, "hvp_sparse");
}

extern "C" pspec_status pspec_hvp_gather_floor(pspec_graph g, int k, const void *U, int64_t ldu, const void *V,
                                               int64_t ldv, void *HV, int64_t ldh, void *G, int64_t ldg,
                                               pspec_stream stream) {
    pspec_status st = hvp_entry(g, PSPEC_F32, k, U, ldu, V, ldv, 1.5, 1.0, HV, ldh, G, ldg, nullptr, stream, true,
                                "hvp_gather_floor", true);
    return st;
}

static pspec_status rhvp_entry(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                               int64_t ldv, double p, double eps, void *RH, int64_t ldrh, void *RG, int64_t ldrg,
                               double *MG, double *F_col, void *ws, size_t ws_bytes, pspec_stream stream, bool fixed_u,
                               const char *who) {
    clear_error();
    pspec_status st = check_common(g, dt, k, U, ldu, p, who);
    if (st != PSPEC_OK) return st;
    PSPEC_ARG(eps > 0.0 && std::isfinite(eps), "%s: eps = %g must be positive", who, eps);
    if ((st = check_out(g, dt, k, V, ldv, "V", who)) != PSPEC_OK) return st;
    if ((st = check_out(g, dt, k, RH, ldrh, "RH", who)) != PSPEC_OK) return st;
    if ((st = check_out(g, dt, k, RG, ldrg, fixed_u ? "G" : "RG", who)) != PSPEC_OK) return st;
    PSPEC_ARG(ws != nullptr, "%s: workspace is NULL", who);
    PSPEC_ARG(((uintptr_t)ws % 256) == 0, "%s: workspace must be 256-byte aligned", who);
    if (ws_bytes < dense_ws_doubles(k) * sizeof(double)) {
        set_error("%s: workspace of %zu bytes < %zu needed", who, ws_bytes, dense_ws_doubles(k) * sizeof(double));
        return PSPEC_ERR_WORKSPACE;
    }
    const size_t es = dt == PSPEC_F32 ? 4 : 8;
    const int64_t n = g->n;
    // RG is an output (rhvp) or the given gradient (rhess, read only: may share memory with U or V)
    PSPEC_ARG(!blocks_overlap(RH, ldrh, U, ldu, n, k, es) && !blocks_overlap(RH, ldrh, V, ldv, n, k, es) &&
                  (fixed_u || (!blocks_overlap(RG, ldrg, U, ldu, n, k, es) && !blocks_overlap(RG, ldrg, V, ldv, n, k, es))) &&
                  !blocks_overlap(RG, ldrg, RH, ldrh, n, k, es),
              "%s: RH (and RG) must not overlap the inputs or each other", who);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *w = static_cast<double *>(ws);
#define PSPEC_RHVP_DT(MODE)                                                                                          \
    if (dt == PSPEC_F32) return rhvp_k<float, float, MODE>(g, k, U, ldu, V, ldv, p, eps, RH, ldrh, RG, ldrg, MG, F_col, w, s); \
    if (g->wtype == PSPEC_F32)                                                                                       \
        return rhvp_k<double, float, MODE>(g, k, U, ldu, V, ldv, p, eps, RH, ldrh, RG, ldrg, MG, F_col, w, s);     \
    return rhvp_k<double, double, MODE>(g, k, U, ldu, V, ldv, p, eps, RH, ldrh, RG, ldrg, MG, F_col, w, s);
    if (fixed_u) {
        PSPEC_RHVP_DT(HESS)
    }
    PSPEC_RHVP_DT(HVP)
#undef PSPEC_RHVP_DT
}

extern "C" pspec_status pspec_rhvp(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                                   int64_t ldv, double p, double eps, void *RH, int64_t ldrh, void *RG, int64_t ldrg,
                                   double *MG, double *F_col, void *ws, size_t ws_bytes, pspec_stream stream) {
    return rhvp_entry(g, dt, k, U, ldu, V, ldv, p, eps, RH, ldrh, RG, ldrg, MG, F_col, ws, ws_bytes, stream, false,
                      "rhvp");
}

extern "C" pspec_status pspec_rhess(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                                    int64_t ldv, const void *G, int64_t ldg, double p, double eps, void *RH,
                                    int64_t ldrh, double *MG, double *F_col, void *ws, size_t ws_bytes,
                                    pspec_stream stream) {
    return rhvp_entry(g, dt, k, U, ldu, V, ldv, p, eps, RH, ldrh, const_cast<void *>(G), ldg, MG, F_col, ws, ws_bytes,
                      stream, true, "rhess");
}

extern "C" pspec_status pspec_rhvp_static(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu,
                                          const void *V, int64_t ldv, double p, double eps, void *RH, int64_t ldrh,
                                          void *RG, int64_t ldrg, double *MG, double *F_col, pspec_stream stream) {
    clear_error();
    PSPEC_UNSUP(k >= 1 && k <= PSPEC_STATIC_K_MAX,
                "rhvp_static: k = %d outside 1..%d (the static scratch holds the Gram partials of k <= %d)", k,
                PSPEC_STATIC_K_MAX, PSPEC_STATIC_K_MAX);
    double *ws = nullptr;
    const pspec_status st = static_scratch(&ws, "rhvp_static");
    if (st != PSPEC_OK) return st;
    return pspec_rhvp(g, dt, k, U, ldu, V, ldv, p, eps, RH, ldrh, RG, ldrg, MG, F_col, ws,
                      dense_ws_doubles(PSPEC_STATIC_K_MAX) * sizeof(double), stream);
}
