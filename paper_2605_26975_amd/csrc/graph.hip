// Graph handle: CSR validation and the degree-binned row schedule.
//
// Rows with at most PSPEC_LIGHT_MAX neighbours are processed by the light edge kernel (a group of
// lanes per row, kTileRows rows per workgroup), in node order or, on graphs whose light rows' degrees
// vary widely, in degree order within each tile.  Longer rows are cut into chunks of at most
// PSPEC_CHUNK edges (rows above PSPEC_CHUNK first at the kSegs column-segment boundaries), handed in
// a fixed order to the waves of the persistent heavy-chunk kernel; rows with several chunks are
// summed afterwards in chunk order.  Each row's first entry above the diagonal is recorded for the
// edge-once objective.  The schedule is
// built with three integer kernels (per-block counts, one-block exclusive scan, per-block emission
// with a block-local scan), so chunk order, and with it every floating-point sum, is the same on every
// run.  Everything the handle keeps on the device lives in the caller's workspace, whose size is
// bounded from (n, nnz, k_max) alone; the library allocates no device memory.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>

#include "common.hpp"

namespace pspec {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

bool blocks_overlap(const void *a, int64_t lda, const void *b, int64_t ldb, int64_t n, int k, size_t es) {
    const char *a0 = (const char *)a, *b0 = (const char *)b;
    const char *a1 = a0 + block_extent(n, k, lda, es), *b1 = b0 + block_extent(n, k, ldb, es);
    if (!(a0 < b1 && b0 < a1)) return false;
    if (lda != ldb) return true;
    const int64_t diff = (int64_t)(b0 - a0);
    if (diff % (int64_t)es != 0) return true;
    int64_t d = diff / (int64_t)es;
    if (d < 0) d = -d;
    const int64_t r = d % lda;
    return r < k || lda - r < k;
}

namespace {

constexpr int kPlanBlock = 256;  // rows per block of the schedule kernels
// Per-row counters of the schedule: heavy rows, chunks of the shared list (rows of LIGHT_MAX + 1 ..
// CHUNK edges, one chunk each), split rows (more than CHUNK edges), their chunks, their chunks in
// each of the kSegs column segments, and the count, degree sum and squared-degree sum of the light
// rows (whether to order each tile's rows by degree).
constexpr int kCHeavy = 0, kCGlob = 1, kCSplit = 2, kCSplitChunks = 3, kCSeg = 4;
constexpr int kCLight = kCSeg + kSegs, kCDeg = kCLight + 1, kCDeg2 = kCLight + 2;
constexpr int kCounters = kCDeg2 + 1;

__global__ __launch_bounds__(kBlock) void k_check_rowptr(const int64_t *__restrict__ rowptr, int64_t n, int64_t nnz,
                                                       int *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t r = rowptr[i];
    bool bad = r < 0 || r > nnz;
    if (i == 0 && r != 0) bad = true;
    if (i == n && r != nnz) bad = true;
    if (i < n && rowptr[i + 1] < r) bad = true;
    if (bad) atomicOr(flag, 1);
}

__global__ __launch_bounds__(kBlock) void k_check_col(const int32_t *__restrict__ col, int64_t nnz, int64_t n,
                                                    int *__restrict__ flag) {
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = col[e];
        bad |= (c < 0 || (int64_t)c >= n);
    }
    if (bad) atomicOr(flag, 2);
}

// Upper parts of the rows, for the objective pass: per row, the count of entries with a column at
// most i (ustart[i] = rowptr[i] + that count), and whether the row's columns do not descend; any
// descent sets bit 4 of *flag, and the objective pass then visits every stored entry instead.  Rows
// of at most kUpperShort entries take a group of 16 lanes each (k_upper); longer rows a whole
// workgroup each (k_upper_long), so that a hub row does not hold one group for its whole length.
constexpr int kUpperShort = 256;

__global__ __launch_bounds__(kBlock) void k_upper(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                int64_t n, int64_t *__restrict__ ustart, int *__restrict__ flag) {
    constexpr int G = 16;
    const int gl = threadIdx.x % G;
    const int64_t groups = (int64_t)gridDim.x * (kBlock / G);
    int bad = 0;
    // every group of a wave takes the same number of turns, so the shuffles below see whole waves
    const int64_t turns = (n + groups - 1) / groups;
    for (int64_t tn = 0; tn < turns; ++tn) {
        const int64_t i = (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G + tn * groups;
        int64_t beg = 0, end = 0;
        if (i < n) {
            beg = rowptr[i];
            end = rowptr[i + 1];
        }
        const bool mine = i < n && end - beg <= kUpperShort;
        if (!mine) end = beg;
        int64_t low = 0;
        for (int64_t q = beg + gl; q < end; q += G) {
            const int32_t c = col[q];
            low += c <= (int32_t)i;
            if (q + 1 < end && col[q + 1] < c) bad = 1;
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) low += __shfl_xor(low, o);
        if (mine && gl == 0) ustart[i] = beg + low;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 4);
}

__global__ __launch_bounds__(kBlock) void k_upper_long(const int64_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col, int64_t n,
                                                     int64_t *__restrict__ ustart, int *__restrict__ flag) {
    __shared__ int64_t s_low[kBlock / 64];
    __shared__ int s_bad[kBlock / 64];
    __shared__ int s_long[kBlock];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // workgroup b takes rows b, b + grid, ...: long rows, which cluster at the ids of hubs, spread
    // over the whole grid.  It first marks which of its next kBlock rows are long, one row per
    // thread, and then walks only those.
    const int64_t grid = gridDim.x;
    for (int64_t r0 = blockIdx.x; r0 < n; r0 += grid * kBlock) {
        const int64_t mine = r0 + (int64_t)tid * grid;
        s_long[tid] = mine < n && rowptr[mine + 1] - rowptr[mine] > kUpperShort;
        __syncthreads();
        for (int t = 0; t < kBlock; ++t) {
            if (!s_long[t]) continue;  // the same for the whole workgroup
            const int64_t i = r0 + (int64_t)t * grid;
            const int64_t beg = rowptr[i], end = rowptr[i + 1];
            int64_t low = 0;
            int bad = 0;
            for (int64_t q = beg + tid; q < end; q += kBlock) {
                const int32_t c = col[q];
                low += c <= (int32_t)i;
                if (q + 1 < end && col[q + 1] < c) bad = 1;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) low += __shfl_xor(low, o);
            const bool wbad = __any(bad);
            if (lane == 0) {
                s_low[w] = low;
                s_bad[w] = wbad ? 1 : 0;
            }
            __syncthreads();
            if (tid == 0) {
                int64_t tot = 0;
                int bb = 0;
                for (int v = 0; v < kBlock / 64; ++v) {
                    tot += s_low[v];
                    bb |= s_bad[v];
                }
                ustart[i] = beg + tot;
                if (bb) atomicOr(flag, 4);
            }
            __syncthreads();
        }
        __syncthreads();  // s_long is rewritten by the next round
    }
}

// Rows of each light tile ordered by degree (heavy rows, which the light kernel skips, count as 0),
// and rows of equal degree by their number of entries above the diagonal (ustart, when the columns
// ascend), stably: perm[tile * kTileRows + position] = row.  A wave of the light kernel then takes
// four rows of about the same length, so fewer of its lanes wait for the longest: in the gradient
// passes, which visit whole rows, and in the edge-once objective, which visits the entries above the
// diagonal.  Used by every FP64 call, and by FP32 calls on graphs whose light rows' degrees vary
// widely (see pspec_graph_create).
__global__ __launch_bounds__(kTileRows) void k_tile_sort(const int64_t *__restrict__ rowptr,
                                                       const int64_t *__restrict__ ustart, int64_t n,
                                                       int light_max, int32_t *__restrict__ perm) {
    __shared__ int s_key[kTileRows];
    const int t = threadIdx.x;
    const int64_t row = (int64_t)blockIdx.x * kTileRows + t;
    int key = (light_max + 1) * (light_max + 1);  // past the last row: sorts last, not written
    if (row < n) {
        const int64_t e = rowptr[row + 1], d = e - rowptr[row];
        const int64_t up = ustart != nullptr ? e - ustart[row] : 0;  // 0 <= up <= d
        key = d <= light_max ? (int)(d * (light_max + 1) + up) : 0;
    }
    s_key[t] = key;
    __syncthreads();
    int pos = 0;
    for (int u = 0; u < kTileRows; ++u) {
        const int ku = s_key[u];
        pos += (ku < key) || (ku == key && u < t);
    }
    if (row < n) perm[(int64_t)blockIdx.x * kTileRows + pos] = (int32_t)row;
}

// Column segment boundaries: bound[s] = the first node j with rowptr[j] >= s nnz / kSegs, so each
// segment [bound[s], bound[s + 1]) holds an equal share of the stored entries -- and, the graph being
// symmetric, receives an equal share of the neighbour gathers.  One thread per boundary.
__global__ void k_seg_bounds(const int64_t *__restrict__ rowptr, int64_t n, int64_t nnz, int32_t *__restrict__ bound) {
    const int s = threadIdx.x;
    if (s > kSegs) return;
    if (s == 0 || s == kSegs) {
        bound[s] = s == 0 ? 0 : (int32_t)n;
        return;
    }
    const int64_t target = (nnz * s + kSegs - 1) / kSegs;
    int64_t lo = 0, hi = n;  // smallest j in [0, n] with rowptr[j] >= target
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (rowptr[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    bound[s] = (int32_t)lo;
}

// First position p in [beg, end) with col[p] >= v (binary search).  For any column order the positions
// found for increasing v never decrease, so the kSegs ranges they delimit always partition the row;
// with ascending columns (the usual CSR) each range holds exactly the row's neighbours in one segment.
__device__ __forceinline__ int64_t lower_pos(const int32_t *__restrict__ col, int64_t beg, int64_t end, int32_t v) {
    int64_t lo = beg, hi = end;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (col[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The row's counters and, for split rows, its segment ranges pos[0..kSegs].
__device__ __forceinline__ void row_counts(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                           const int32_t *__restrict__ bound, int64_t n, int64_t i, int light_max,
                                           int chunk, int64_t cnt[kCounters], int64_t pos[kSegs + 1]) {
    for (int q = 0; q < kCounters; ++q) cnt[q] = 0;
    if (i >= n) return;
    const int64_t beg = rowptr[i], end = rowptr[i + 1], d = end - beg;
    if (d <= light_max) {
        cnt[kCLight] = 1;
        cnt[kCDeg] = d;
        cnt[kCDeg2] = d * d;
        return;
    }
    cnt[kCHeavy] = 1;
    if (d <= chunk) {
        cnt[kCGlob] = 1;
        return;
    }
    cnt[kCSplit] = 1;
    pos[0] = beg;
    pos[kSegs] = end;
    for (int s = 1; s < kSegs; ++s) pos[s] = lower_pos(col, pos[s - 1], end, bound[s]);
    for (int s = 0; s < kSegs; ++s) {
        const int64_t c = (pos[s + 1] - pos[s] + chunk - 1) / chunk;
        cnt[kCSeg + s] = c;
        cnt[kCSplitChunks] += c;
    }
}

__global__ __launch_bounds__(kPlanBlock) void k_plan_count(const int64_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ bound, int64_t n, int light_max,
                                                         int chunk, int64_t *__restrict__ bcount) {
    __shared__ int64_t s[kCounters][kPlanBlock];
    const int t = threadIdx.x;
    int64_t cnt[kCounters], pos[kSegs + 1];
    row_counts(rowptr, col, bound, n, (int64_t)blockIdx.x * kPlanBlock + t, light_max, chunk, cnt, pos);
    for (int q = 0; q < kCounters; ++q) s[q][t] = cnt[q];
    __syncthreads();
    for (int o = kPlanBlock / 2; o > 0; o >>= 1) {
        if (t < o)
            for (int q = 0; q < kCounters; ++q) s[q][t] += s[q][t + o];
        __syncthreads();
    }
    if (t == 0)
        for (int q = 0; q < kCounters; ++q) bcount[(int64_t)blockIdx.x * kCounters + q] = s[q][0];
}

// One workgroup: exclusive scan of the per-block counts, in place; totals to tot[kCounters].
__global__ __launch_bounds__(kPlanBlock) void k_plan_scan(int64_t *__restrict__ bcount, int64_t nb,
                                                        int64_t *__restrict__ tot) {
    __shared__ int64_t s[kCounters][kPlanBlock];
    const int t = threadIdx.x;
    const int64_t seg = (nb + kPlanBlock - 1) / kPlanBlock;
    const int64_t b0 = t * seg, b1 = (b0 + seg < nb) ? b0 + seg : nb;
    int64_t loc[kCounters];
    for (int q = 0; q < kCounters; ++q) loc[q] = 0;
    for (int64_t b = b0; b < b1; ++b)
        for (int q = 0; q < kCounters; ++q) loc[q] += bcount[b * kCounters + q];
    for (int q = 0; q < kCounters; ++q) s[q][t] = loc[q];
    __syncthreads();
    if (t == 0) {
        int64_t run[kCounters];
        for (int q = 0; q < kCounters; ++q) run[q] = 0;
        for (int i = 0; i < kPlanBlock; ++i)
            for (int q = 0; q < kCounters; ++q) {
                const int64_t v = s[q][i];
                s[q][i] = run[q];
                run[q] += v;
            }
        for (int q = 0; q < kCounters; ++q) tot[q] = run[q];
    }
    __syncthreads();
    int64_t run[kCounters];
    for (int q = 0; q < kCounters; ++q) run[q] = s[q][t];
    for (int64_t b = b0; b < b1; ++b)
        for (int q = 0; q < kCounters; ++q) {
            const int64_t v = bcount[b * kCounters + q];
            bcount[b * kCounters + q] = run[q];
            run[q] += v;
        }
}

// Chunk list layout: the chunks of column segment 0, ..., segment kSegs - 1 (base.seg[s]), then the
// shared list (base.glob).  Each split row's chunks take consecutive scratch slots in (segment,
// position) order, the order in which they are combined.
struct ChunkBases {
    int64_t seg[kSegs + 1];
    int64_t glob;
};

__global__ __launch_bounds__(kPlanBlock) void k_plan_emit(const int64_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ bound, int64_t n, int light_max,
                                                        int chunk, const int64_t *__restrict__ boff, ChunkBases base,
                                                        Chunk *__restrict__ chunks, Split *__restrict__ splits) {
    __shared__ int64_t s[kCounters][kPlanBlock];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kPlanBlock + t;
    int64_t cnt[kCounters], pos[kSegs + 1];
    row_counts(rowptr, col, bound, n, i, light_max, chunk, cnt, pos);
    for (int q = 0; q < kCounters; ++q) s[q][t] = cnt[q];
    __syncthreads();
    // Hillis-Steele inclusive scan over the block
    for (int o = 1; o < kPlanBlock; o <<= 1) {
        int64_t v[kCounters];
        for (int q = 0; q < kCounters; ++q) v[q] = t >= o ? s[q][t - o] : 0;
        __syncthreads();
        for (int q = 0; q < kCounters; ++q) s[q][t] += v[q];
        __syncthreads();
    }
    if (cnt[kCHeavy] == 0) return;
    auto first = [&](int q) { return boff[(int64_t)blockIdx.x * kCounters + q] + s[q][t] - cnt[q]; };
    if (cnt[kCGlob]) {
        Chunk c;
        c.beg = rowptr[i];
        c.end = rowptr[i + 1];
        c.row = (int32_t)i;
        c.slot = -1;
        chunks[base.glob + first(kCGlob)] = c;
        return;
    }
    const int64_t xbase = first(kCSplitChunks);  // first scratch slot of the row
    int64_t slot = xbase;
    for (int sg = 0; sg < kSegs; ++sg) {
        const int64_t c0 = base.seg[sg] + first(kCSeg + sg);
        for (int64_t q = 0; q < cnt[kCSeg + sg]; ++q) {
            Chunk c;
            c.beg = pos[sg] + q * chunk;
            c.end = (c.beg + chunk < pos[sg + 1]) ? c.beg + chunk : pos[sg + 1];
            c.row = (int32_t)i;
            c.slot = (int32_t)slot++;
            chunks[c0 + q] = c;
        }
    }
    Split sp;
    sp.row = (int32_t)i;
    sp.first = (int32_t)xbase;
    sp.count = (int32_t)cnt[kCSplitChunks];
    sp.pad = 0;
    splits[first(kCSplit)] = sp;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of the caller's workspace.  The first part depends on (n, k_max) only: the schedule kernels'
// counters, the column-segment boundaries, the rows' upper starts, the FP64 partial sums of the
// edge pass and (k_max > 8) the Gram partials of the Riemannian call at 9 <= k <= 16.  The schedule
// itself (chunk list, split-row list, split-row scratch) follows, sized by the counts of the graph:
// exact once they are known, otherwise by bounds from (n, nnz) alone --
//   heavy rows   <= min(n, nnz / (LIGHT_MAX + 1))      (each holds more than LIGHT_MAX edges)
//   split rows   <= min(n, nnz / (CHUNK + 1))
//   split chunks <= nnz / CHUNK + kSegs split rows     (sum over segments of ceil(d_s / C) <= d / C + kSegs)
//   chunks       <= heavy rows + split chunks
//   partial rows  = light tiles + kHeavyGridCap
struct WsLayout {
    size_t bcount = 0, tot = 0, bound = 0, ust = 0, perm = 0, part = 0, red1 = 0, sc = 0, gram = 0, chunks = 0,
           splits = 0, scr = 0;
    size_t fixed = 0, total = 0;
};

WsLayout ws_layout(int64_t n, int k_max, int64_t n_chunks, int64_t n_split, int64_t n_split_chunks) {
    WsLayout L;
    const int64_t tiles = (n + kTileRows - 1) / kTileRows;
    const int64_t nb = (n + kPlanBlock - 1) / kPlanBlock;
    const size_t parts[] = {
        align256(sizeof(int64_t) * (size_t)nb * kCounters),
        align256(sizeof(int64_t) * kCounters + sizeof(int)),
        align256(sizeof(int32_t) * (kSegs + 1)),
        align256(sizeof(int64_t) * (size_t)n),
        align256(sizeof(int32_t) * (size_t)n),
        align256(sizeof(double) * (size_t)(tiles + kHeavyGridCap) * kQ * (size_t)k_max),
        align256(sizeof(double) * (size_t)kReduceSlices * kQ * (size_t)k_max),
        align256(sizeof(double) * (size_t)kScalars * (size_t)k_max),
        pad_k(k_max) >= kGramK ? align256(sizeof(double) * (size_t)gram_area_rows(tiles) * kGramQ * kGramK * kGramK) : 0,
        align256(sizeof(Chunk) * (size_t)n_chunks),
        align256(sizeof(Split) * (size_t)n_split),
        align256(sizeof(double) * (size_t)n_split_chunks * 2 * (size_t)k_max),
    };
    size_t *dst[] = {&L.bcount, &L.tot,  &L.bound, &L.ust,    &L.perm,   &L.part,
                     &L.red1,   &L.sc,   &L.gram,  &L.chunks, &L.splits, &L.scr};
    size_t off = 0;
    for (int i = 0; i < 12; ++i) {
        *dst[i] = off;
        off += parts[i];
        if (i == 8) L.fixed = off;
    }
    L.total = off;
    return L;
}

WsLayout ws_bound(int64_t n, int64_t nnz, int k_max) {
    const int64_t max_heavy = std::min<int64_t>(n, nnz / (PSPEC_LIGHT_MAX + 1));
    const int64_t max_split = std::min<int64_t>(n, nnz / (PSPEC_CHUNK + 1));
    const int64_t max_split_chunks = nnz / PSPEC_CHUNK + (int64_t)kSegs * max_split;
    return ws_layout(n, k_max, max_heavy + max_split_chunks, max_split, max_split_chunks);
}

bool ws_args_ok(int64_t n, int64_t nnz, int k_max) {
    return n >= 1 && nnz >= 0 && k_max >= 1 && k_max <= PSPEC_K_MAX && n < ((int64_t)1 << 31) - 1;
}

// The counts of a graph's schedule (validated CSR): tot[kCounters] from the counting kernels.
struct Plan {
    int64_t tot[kCounters];
    int flag = 0;  // bit 4: some row's columns descend
    int64_t n_chunks() const { return tot[kCGlob] + tot[kCSplitChunks]; }
};

// Shared front half of create and the workspace query: argument checks, CSR validation, segment
// boundaries, upper starts and schedule counts in the workspace's fixed part; synchronises the
// stream twice.
pspec_status plan_counts(const char *who, int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col, int k_max,
                         void *workspace, size_t ws_bytes, hipStream_t s, WsLayout &L, Plan &plan) {
    PSPEC_ARG(n >= 1, "%s: n = %lld < 1", who, (long long)n);
    PSPEC_ARG(nnz >= 0, "%s: nnz = %lld < 0", who, (long long)nnz);
    PSPEC_ARG(rowptr != nullptr, "%s: rowptr is NULL", who);
    PSPEC_ARG(nnz == 0 || col != nullptr, "%s: col is NULL", who);
    PSPEC_UNSUP(k_max >= 1 && k_max <= PSPEC_K_MAX, "%s: k_max = %d outside 1..%d", who, k_max, PSPEC_K_MAX);
    PSPEC_UNSUP(n < ((int64_t)1 << 31) - 1, "%s: n = %lld needs 64-bit node ids", who, (long long)n);
    PSPEC_ARG(workspace != nullptr, "%s: workspace is NULL", who);
    PSPEC_ARG(((uintptr_t)workspace % 256) == 0, "%s: workspace must be 256-byte aligned", who);
    L = ws_layout(n, k_max, 0, 0, 0);
    if (ws_bytes < L.fixed) {
        set_error("%s: workspace of %zu bytes < %zu needed before the schedule", who, ws_bytes, L.fixed);
        return PSPEC_ERR_WORKSPACE;
    }
    char *mem = static_cast<char *>(workspace);
    int64_t *bcount = reinterpret_cast<int64_t *>(mem + L.bcount);
    int64_t *tot = reinterpret_cast<int64_t *>(mem + L.tot);
    int *flag = reinterpret_cast<int *>(tot + kCounters);
    int32_t *bound = reinterpret_cast<int32_t *>(mem + L.bound);
    const int64_t nb = (n + kPlanBlock - 1) / kPlanBlock;
    PSPEC_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_check_rowptr<<<(unsigned)((n + 1 + kBlock - 1) / kBlock), kBlock, 0, s>>>(rowptr, n, nnz, flag);
    if (nnz > 0) {
        const int64_t want = (nnz + kBlock - 1) / kBlock;
        k_check_col<<<(unsigned)(want < 65536 ? want : 65536), kBlock, 0, s>>>(col, nnz, n, flag);
    }
    PSPEC_HIP(hipGetLastError());
    int host_flag = 0;
    PSPEC_HIP(hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PSPEC_HIP(hipStreamSynchronize(s));
    if (host_flag != 0) {
        set_error("%s: malformed CSR (%s%s)", who, (host_flag & 1) ? "row pointers" : "",
                  (host_flag & 2) ? " column indices out of range" : "");
        return PSPEC_ERR_ARG;
    }
    // only a validated CSR is searched: the boundaries, upper starts and counts read rowptr and col
    k_seg_bounds<<<1, 64, 0, s>>>(rowptr, n, nnz, bound);
    {
        const int64_t want = (n + kBlock / 16 - 1) / (kBlock / 16);
        k_upper<<<(unsigned)(want < 65536 ? want : 65536), kBlock, 0, s>>>(
            rowptr, col, n, reinterpret_cast<int64_t *>(mem + L.ust), flag);
        k_upper_long<<<(unsigned)(n < 65536 ? n : 65536), kBlock, 0, s>>>(
            rowptr, col, n, reinterpret_cast<int64_t *>(mem + L.ust), flag);
    }
    k_plan_count<<<(unsigned)nb, kPlanBlock, 0, s>>>(rowptr, col, bound, n, PSPEC_LIGHT_MAX, PSPEC_CHUNK, bcount);
    k_plan_scan<<<1, kPlanBlock, 0, s>>>(bcount, nb, tot);
    PSPEC_HIP(hipGetLastError());
    PSPEC_HIP(hipMemcpyAsync(plan.tot, tot, sizeof(int64_t) * kCounters, hipMemcpyDeviceToHost, s));
    PSPEC_HIP(hipMemcpyAsync(&plan.flag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PSPEC_HIP(hipStreamSynchronize(s));
    // the bounds of ws_bound hold for every valid CSR; a violation means the counts are wrong
    const WsLayout B = ws_bound(n, nnz, k_max);
    if (ws_layout(n, k_max, plan.n_chunks(), plan.tot[kCSplit], plan.tot[kCSplitChunks]).total > B.total) {
        set_error("%s: schedule (%lld chunks, %lld split rows, %lld split chunks) exceeds its bound", who,
                  (long long)plan.n_chunks(), (long long)plan.tot[kCSplit], (long long)plan.tot[kCSplitChunks]);
        return PSPEC_ERR_HIP;
    }
    L = ws_layout(n, k_max, plan.n_chunks(), plan.tot[kCSplit], plan.tot[kCSplitChunks]);
    return PSPEC_OK;
}

}  // namespace
}  // namespace pspec

using namespace pspec;

extern "C" const char *pspec_last_error(void) { return g_err; }

extern "C" size_t pspec_graph_workspace_bytes(int64_t n, int64_t nnz, int k_max) {
    return ws_args_ok(n, nnz, k_max) ? ws_bound(n, nnz, k_max).total : 0;
}

extern "C" size_t pspec_graph_count_workspace_bytes(int64_t n, int k_max) {
    return ws_args_ok(n, 0, k_max) ? ws_layout(n, k_max, 0, 0, 0).fixed : 0;
}

extern "C" pspec_status pspec_graph_exact_workspace(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                                                    int k_max, void *workspace, size_t ws_bytes, pspec_stream stream,
                                                    size_t *needed) {
    clear_error();
    PSPEC_ARG(needed != nullptr, "graph_exact_workspace: needed is NULL");
    *needed = 0;
    WsLayout L;
    Plan plan;
    const pspec_status st = plan_counts("graph_exact_workspace", n, nnz, rowptr, col, k_max, workspace, ws_bytes,
                                        reinterpret_cast<hipStream_t>(stream), L, plan);
    if (st != PSPEC_OK) return st;
    *needed = L.total;
    return PSPEC_OK;
}

extern "C" pspec_status pspec_graph_create(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                                           const void *w, pspec_dtype wtype, int k_max, void *workspace,
                                           size_t ws_bytes, pspec_stream stream, pspec_graph *out) {
    clear_error();
    PSPEC_ARG(out != nullptr, "graph_create: out is NULL");
    *out = nullptr;
    PSPEC_ARG(nnz == 0 || w != nullptr, "graph_create: w is NULL");
    PSPEC_ARG(wtype == PSPEC_F32 || wtype == PSPEC_F64, "graph_create: bad wtype %d", (int)wtype);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    WsLayout L;
    Plan plan;
    pspec_status st = plan_counts("graph_create", n, nnz, rowptr, col, k_max, workspace, ws_bytes, s, L, plan);
    if (st != PSPEC_OK) return st;
    if (ws_bytes < L.total) {
        set_error("graph_create: workspace of %zu bytes < %zu this graph's schedule needs", ws_bytes, L.total);
        return PSPEC_ERR_WORKSPACE;
    }
    char *mem = static_cast<char *>(workspace);
    ChunkBases base;
    base.seg[0] = 0;
    for (int sg = 0; sg < kSegs; ++sg) base.seg[sg + 1] = base.seg[sg] + plan.tot[kCSeg + sg];
    base.glob = base.seg[kSegs];

    int dev = 0;
    PSPEC_HIP(hipGetDevice(&dev));
    pspec_graph g = new pspec_graph_s();
    g->n = n;
    g->nnz = nnz;
    g->rowptr = rowptr;
    g->col = col;
    g->w = w;
    g->wtype = wtype;
    g->k_max = k_max;
    g->device = dev;
    g->tiles = (n + kTileRows - 1) / kTileRows;
    g->heavy_rows = plan.tot[kCHeavy];
    g->n_chunks = plan.n_chunks();
    g->n_split = plan.tot[kCSplit];
    g->n_split_chunks = plan.tot[kCSplitChunks];
    for (int sg = 0; sg <= kSegs; ++sg) g->seg_chunk_base[sg] = base.seg[sg];
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
    g->cus = cus > 0 ? cus : 1;
    // a multiple of kSegs (every segment served by as many workgroups), at least kSegs
    const int64_t hwant = std::max<int64_t>((g->n_chunks + 3) / 4, kSegs);
    const int64_t hmax = std::min<int64_t>(std::min<int64_t>(hwant, (int64_t)kHeavyPerCUMax * g->cus), kHeavyGridCap);
    g->heavy_grid_max = std::max<int64_t>(hmax / kSegs * kSegs, kSegs);
    g->chunks = reinterpret_cast<Chunk *>(mem + L.chunks);
    g->splits = reinterpret_cast<Split *>(mem + L.splits);
    g->partials = reinterpret_cast<double *>(mem + L.part);
    g->red1 = reinterpret_cast<double *>(mem + L.red1);
    g->scalars = reinterpret_cast<double *>(mem + L.sc);
    g->chunk_scratch = reinterpret_cast<double *>(mem + L.scr);
    g->ascending = (plan.flag & 4) == 0;
    g->ustart = reinterpret_cast<const int64_t *>(mem + L.ust);
    g->gram_part = pad_k(k_max) >= kGramK ? reinterpret_cast<double *>(mem + L.gram) : nullptr;
    // Each light tile's rows in degree order (equal degrees by their count of entries above the
    // diagonal), so that rows of equal length share a wave.  FP64 calls, bound by the arithmetic of
    // the power, always take this order.  FP32 calls, bound by the gathers,
    // take it only when the light rows' degrees vary widely (coefficient of variation above 1:
    // power-law graphs such as R-MAT, 1.4-1.9; SBM, kNN, grids and triangulations 0.04-0.3); on graphs
    // of near-uniform degree they keep the node order, which keeps each wave's row writes contiguous.
    {
        const double cntl = (double)plan.tot[kCLight], s1 = (double)plan.tot[kCDeg], s2 = (double)plan.tot[kCDeg2];
        const double mean = cntl > 0 ? s1 / cntl : 0.0, var = cntl > 0 ? s2 / cntl - mean * mean : 0.0;
        g->sorted_tiles = mean > 0.0 && var > mean * mean;
        if (mean > 0.0) {
            int32_t *perm = reinterpret_cast<int32_t *>(mem + L.perm);
            k_tile_sort<<<(unsigned)g->tiles, kTileRows, 0, s>>>(rowptr, g->ascending ? g->ustart : nullptr, n,
                                                                 PSPEC_LIGHT_MAX, perm);
            g->lperm = perm;
        }
    }
    if (g->n_chunks > 0) {
        const int64_t nb = (n + kPlanBlock - 1) / kPlanBlock;
        k_plan_emit<<<(unsigned)nb, kPlanBlock, 0, s>>>(rowptr, col, reinterpret_cast<const int32_t *>(mem + L.bound),
                                                         n, PSPEC_LIGHT_MAX, PSPEC_CHUNK,
                                                         reinterpret_cast<const int64_t *>(mem + L.bcount), base,
                                                         g->chunks, g->splits);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        delete g;
        set_error("graph_create: k_plan_emit: %s", hipGetErrorString(e));
        return PSPEC_ERR_HIP;
    }
    *out = g;
    return PSPEC_OK;
}

extern "C" pspec_status pspec_graph_destroy(pspec_graph g) {
    clear_error();
    delete g;  // host memory only: the device memory is the caller's workspace
    return PSPEC_OK;
}

extern "C" pspec_status pspec_graph_info(pspec_graph g, int64_t *heavy_rows, int64_t *chunks, int64_t *split_rows) {
    clear_error();
    PSPEC_ARG(g != nullptr, "graph_info: NULL handle");
    if (heavy_rows) *heavy_rows = g->heavy_rows;
    if (chunks) *chunks = g->n_chunks;
    if (split_rows) *split_rows = g->n_split;
    return PSPEC_OK;
}

extern "C" pspec_status pspec_graph_ascending(pspec_graph g, int *ascending) {
    clear_error();
    PSPEC_ARG(g != nullptr, "graph_ascending: NULL handle");
    PSPEC_ARG(ascending != nullptr, "graph_ascending: ascending is NULL");
    *ascending = g->ascending ? 1 : 0;
    return PSPEC_OK;
}

extern "C" pspec_status pspec_graph_degree_order(pspec_graph g, int *on) {
    clear_error();
    PSPEC_ARG(g != nullptr, "graph_degree_order: NULL handle");
    PSPEC_ARG(on != nullptr, "graph_degree_order: on is NULL");
    *on = g->sorted_tiles ? 1 : 0;
    return PSPEC_OK;
}

extern "C" pspec_status pspec_graph_set_timing_events(pspec_graph g, pspec_event before, pspec_event after) {
    clear_error();
    PSPEC_ARG(g != nullptr, "graph_set_timing_events: NULL handle");
    PSPEC_ARG((before == nullptr) == (after == nullptr), "graph_set_timing_events: give both events or neither");
    g->ev_before = reinterpret_cast<hipEvent_t>(before);
    g->ev_after = reinterpret_cast<hipEvent_t>(after);
    return PSPEC_OK;
}
