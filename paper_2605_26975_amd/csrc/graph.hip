// Graph handle: CSR validation and the degree-binned row schedule.
//
// Rows with at most PSPEC_LIGHT_MAX neighbours are processed in node order by the light edge
// kernel (a group of lanes per row, kTileRows rows per workgroup).  Longer rows are cut into
// chunks of at most PSPEC_CHUNK edges, handed in a fixed order to the waves of the persistent
// heavy-chunk kernel; rows with several chunks are summed afterwards in chunk order.  The schedule is
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
constexpr int kCounters = 4;     // heavy rows, chunks, split rows, chunks of split rows

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

__device__ __forceinline__ void row_counts(const int64_t *__restrict__ rowptr, int64_t n, int64_t i, int light_max,
                                           int chunk, int64_t cnt[kCounters]) {
    cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0;
    if (i < n) {
        const int64_t d = rowptr[i + 1] - rowptr[i];
        if (d > light_max) {
            const int64_t nch = (d + chunk - 1) / chunk;
            cnt[0] = 1;
            cnt[1] = nch;
            cnt[2] = nch > 1 ? 1 : 0;
            cnt[3] = nch > 1 ? nch : 0;
        }
    }
}

__global__ __launch_bounds__(kPlanBlock) void k_plan_count(const int64_t *__restrict__ rowptr, int64_t n, int light_max,
                                                         int chunk, int64_t *__restrict__ bcount) {
    __shared__ int64_t s[kCounters][kPlanBlock];
    const int t = threadIdx.x;
    int64_t cnt[kCounters];
    row_counts(rowptr, n, (int64_t)blockIdx.x * kPlanBlock + t, light_max, chunk, cnt);
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
    int64_t loc[kCounters] = {0, 0, 0, 0};
    for (int64_t b = b0; b < b1; ++b)
        for (int q = 0; q < kCounters; ++q) loc[q] += bcount[b * kCounters + q];
    for (int q = 0; q < kCounters; ++q) s[q][t] = loc[q];
    __syncthreads();
    if (t == 0) {
        int64_t run[kCounters] = {0, 0, 0, 0};
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

__global__ __launch_bounds__(kPlanBlock) void k_plan_emit(const int64_t *__restrict__ rowptr, int64_t n, int light_max,
                                                        int chunk, const int64_t *__restrict__ boff,
                                                        Chunk *__restrict__ chunks, Split *__restrict__ splits) {
    __shared__ int64_t s[kCounters][kPlanBlock];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kPlanBlock + t;
    int64_t cnt[kCounters];
    row_counts(rowptr, n, i, light_max, chunk, cnt);
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
    if (cnt[1] == 0) return;
    const int64_t cbase = boff[(int64_t)blockIdx.x * kCounters + 1] + s[1][t] - cnt[1];
    const int64_t sbase = boff[(int64_t)blockIdx.x * kCounters + 2] + s[2][t] - cnt[2];
    const int64_t xbase = boff[(int64_t)blockIdx.x * kCounters + 3] + s[3][t] - cnt[3];  // first scratch slot
    const int64_t beg = rowptr[i], end = rowptr[i + 1];
    const bool split = cnt[1] > 1;
    for (int64_t q = 0; q < cnt[1]; ++q) {
        Chunk c;
        c.beg = beg + q * chunk;
        c.end = (c.beg + chunk < end) ? c.beg + chunk : end;
        c.row = (int32_t)i;
        c.slot = split ? (int32_t)(xbase + q) : -1;
        chunks[cbase + q] = c;
    }
    if (split) {
        Split sp;
        sp.row = (int32_t)i;
        sp.first = (int32_t)xbase;
        sp.count = (int32_t)cnt[1];
        sp.pad = 0;
        splits[sbase] = sp;
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of the caller's workspace: every part bounded from (n, nnz, k_max) alone.
//   heavy rows   <= min(n, nnz / (LIGHT_MAX + 1))      (each holds more than LIGHT_MAX edges)
//   chunks       <= nnz / CHUNK + heavy rows           (ceil(d / C) <= floor(d / C) + 1, sum floor <= nnz / C)
//   split rows   <= min(n, nnz / (CHUNK + 1))
//   split chunks <= nnz / CHUNK + split rows
//   partial rows  = light tiles + kHeavyGridCap
struct WsLayout {
    size_t chunks = 0, splits = 0, part = 0, red1 = 0, sc = 0, scr = 0, bcount = 0, tot = 0, total = 0;
    int64_t max_chunks = 0, max_split = 0, max_split_chunks = 0;
};

WsLayout ws_layout(int64_t n, int64_t nnz, int k_max) {
    WsLayout L;
    const int64_t max_heavy = std::min<int64_t>(n, nnz / (PSPEC_LIGHT_MAX + 1));
    L.max_chunks = nnz / PSPEC_CHUNK + max_heavy;
    L.max_split = std::min<int64_t>(n, nnz / (PSPEC_CHUNK + 1));
    L.max_split_chunks = nnz / PSPEC_CHUNK + L.max_split;
    const int64_t tiles = (n + kTileRows - 1) / kTileRows;
    const int64_t nb = (n + kPlanBlock - 1) / kPlanBlock;
    const size_t parts[] = {
        align256(sizeof(Chunk) * (size_t)L.max_chunks),
        align256(sizeof(Split) * (size_t)L.max_split),
        align256(sizeof(double) * (size_t)(tiles + kHeavyGridCap) * kQ * (size_t)k_max),
        align256(sizeof(double) * (size_t)kReduceSlices * kQ * (size_t)k_max),
        align256(sizeof(double) * (size_t)kScalars * (size_t)k_max),
        align256(sizeof(double) * (size_t)L.max_split_chunks * 2 * (size_t)k_max),
        align256(sizeof(int64_t) * (size_t)nb * kCounters),
        align256(sizeof(int64_t) * kCounters + sizeof(int)),
    };
    size_t *dst[] = {&L.chunks, &L.splits, &L.part, &L.red1, &L.sc, &L.scr, &L.bcount, &L.tot};
    size_t off = 0;
    for (int i = 0; i < 8; ++i) {
        *dst[i] = off;
        off += parts[i];
    }
    L.total = off;
    return L;
}

bool ws_args_ok(int64_t n, int64_t nnz, int k_max) {
    return n >= 1 && nnz >= 0 && k_max >= 1 && k_max <= PSPEC_K_MAX && n < ((int64_t)1 << 31) - 1;
}

}  // namespace
}  // namespace pspec

using namespace pspec;

extern "C" const char *pspec_last_error(void) { return g_err; }

extern "C" size_t pspec_graph_workspace_bytes(int64_t n, int64_t nnz, int k_max) {
    return ws_args_ok(n, nnz, k_max) ? ws_layout(n, nnz, k_max).total : 0;
}

extern "C" pspec_status pspec_graph_create(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                                           const void *w, pspec_dtype wtype, int k_max, void *workspace,
                                           size_t ws_bytes, pspec_stream stream, pspec_graph *out) {
    clear_error();
    PSPEC_ARG(out != nullptr, "graph_create: out is NULL");
    *out = nullptr;
    PSPEC_ARG(n >= 1, "graph_create: n = %lld < 1", (long long)n);
    PSPEC_ARG(nnz >= 0, "graph_create: nnz = %lld < 0", (long long)nnz);
    PSPEC_ARG(rowptr != nullptr, "graph_create: rowptr is NULL");
    PSPEC_ARG(nnz == 0 || (col != nullptr && w != nullptr), "graph_create: col or w is NULL");
    PSPEC_ARG(wtype == PSPEC_F32 || wtype == PSPEC_F64, "graph_create: bad wtype %d", (int)wtype);
    PSPEC_UNSUP(k_max >= 1 && k_max <= PSPEC_K_MAX, "graph_create: k_max = %d outside 1..%d", k_max, PSPEC_K_MAX);
    PSPEC_UNSUP(n < ((int64_t)1 << 31) - 1, "graph_create: n = %lld needs 64-bit node ids", (long long)n);
    PSPEC_ARG(workspace != nullptr, "graph_create: workspace is NULL");
    PSPEC_ARG(((uintptr_t)workspace % 256) == 0, "graph_create: workspace must be 256-byte aligned");
    const WsLayout L = ws_layout(n, nnz, k_max);
    if (ws_bytes < L.total) {
        set_error("graph_create: workspace of %zu bytes < %zu needed", ws_bytes, L.total);
        return PSPEC_ERR_WORKSPACE;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *mem = static_cast<char *>(workspace);
    int64_t *bcount = reinterpret_cast<int64_t *>(mem + L.bcount);
    int64_t *tot = reinterpret_cast<int64_t *>(mem + L.tot);
    int *flag = reinterpret_cast<int *>(tot + kCounters);

    int dev = 0;
    PSPEC_HIP(hipGetDevice(&dev));
    const int64_t nb = (n + kPlanBlock - 1) / kPlanBlock;
    PSPEC_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_check_rowptr<<<(unsigned)((n + 1 + kBlock - 1) / kBlock), kBlock, 0, s>>>(rowptr, n, nnz, flag);
    if (nnz > 0) {
        const int64_t want = (nnz + kBlock - 1) / kBlock;
        k_check_col<<<(unsigned)(want < 65536 ? want : 65536), kBlock, 0, s>>>(col, nnz, n, flag);
    }
    k_plan_count<<<(unsigned)nb, kPlanBlock, 0, s>>>(rowptr, n, PSPEC_LIGHT_MAX, PSPEC_CHUNK, bcount);
    k_plan_scan<<<1, kPlanBlock, 0, s>>>(bcount, nb, tot);
    PSPEC_HIP(hipGetLastError());
    int64_t host_tot[kCounters + 1];
    PSPEC_HIP(hipMemcpyAsync(host_tot, tot, sizeof(int64_t) * kCounters + sizeof(int), hipMemcpyDeviceToHost, s));
    PSPEC_HIP(hipStreamSynchronize(s));
    int host_flag = 0;
    std::memcpy(&host_flag, &host_tot[kCounters], sizeof(int));
    if (host_flag != 0) {
        set_error("graph_create: malformed CSR (%s%s)", (host_flag & 1) ? "row pointers" : "",
                  (host_flag & 2) ? " column indices out of range" : "");
        return PSPEC_ERR_ARG;
    }
    // the bounds of ws_layout hold for every valid CSR; a violation means the counts are wrong
    if (host_tot[1] > L.max_chunks || host_tot[2] > L.max_split || host_tot[3] > L.max_split_chunks) {
        set_error("graph_create: schedule (%lld chunks, %lld split rows, %lld split chunks) exceeds its bound",
                  (long long)host_tot[1], (long long)host_tot[2], (long long)host_tot[3]);
        return PSPEC_ERR_HIP;
    }

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
    g->heavy_rows = host_tot[0];
    g->n_chunks = host_tot[1];
    g->n_split = host_tot[2];
    g->n_split_chunks = host_tot[3];
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
    g->cus = cus > 0 ? cus : 1;
    const int64_t hwant = (g->n_chunks + 3) / 4;
    g->heavy_grid_max = std::min<int64_t>(std::min<int64_t>(hwant, (int64_t)kHeavyPerCUMax * g->cus), kHeavyGridCap);
    g->chunks = reinterpret_cast<Chunk *>(mem + L.chunks);
    g->splits = reinterpret_cast<Split *>(mem + L.splits);
    g->partials = reinterpret_cast<double *>(mem + L.part);
    g->red1 = reinterpret_cast<double *>(mem + L.red1);
    g->scalars = reinterpret_cast<double *>(mem + L.sc);
    g->chunk_scratch = reinterpret_cast<double *>(mem + L.scr);
    if (g->n_chunks > 0)
        k_plan_emit<<<(unsigned)nb, kPlanBlock, 0, s>>>(rowptr, n, PSPEC_LIGHT_MAX, PSPEC_CHUNK, bcount, g->chunks,
                                                         g->splits);
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

extern "C" pspec_status pspec_graph_set_timing_events(pspec_graph g, pspec_event before, pspec_event after) {
    clear_error();
    PSPEC_ARG(g != nullptr, "graph_set_timing_events: NULL handle");
    PSPEC_ARG((before == nullptr) == (after == nullptr), "graph_set_timing_events: give both events or neither");
    g->ev_before = reinterpret_cast<hipEvent_t>(before);
    g->ev_after = reinterpret_cast<hipEvent_t>(after);
    return PSPEC_OK;
}
