// Internal declarations shared by the translation units of libpspec.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pspec.h"

namespace pspec {

// ---- error reporting (host) ----------------------------------------------------------------
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define PSPEC_HIP(call)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            ::pspec::set_error("%s failed: %s", #call, hipGetErrorString(e_));                \
            return PSPEC_ERR_HIP;                                                             \
        }                                                                                     \
    } while (0)

#define PSPEC_ARG(cond, ...)                                                                  \
    do {                                                                                      \
        if (!(cond)) {                                                                        \
            ::pspec::set_error(__VA_ARGS__);                                                  \
            return PSPEC_ERR_ARG;                                                             \
        }                                                                                     \
    } while (0)

#define PSPEC_UNSUP(cond, ...)                                                                \
    do {                                                                                      \
        if (!(cond)) {                                                                        \
            ::pspec::set_error(__VA_ARGS__);                                                  \
            return PSPEC_ERR_UNSUPPORTED;                                                     \
        }                                                                                     \
    } while (0)

// ---- row schedule ----------------------------------------------------------------------------
// A heavy row (degree > PSPEC_LIGHT_MAX) of at most PSPEC_CHUNK edges is one chunk of the shared list
// and writes its results directly (slot = -1).  A longer (split) row is cut by column segment (kSegs
// ranges of node ids holding equal shares of the stored entries) and each piece into chunks of at
// most PSPEC_CHUNK edges; the chunks of segment s are processed by the workgroups with
// blockIdx.x % kSegs == s, which the dispatcher places on one XCD, so each XCD's L2 caches the rows of
// one segment only.  Such chunks write partial rows into scratch slot `slot` and the row is combined
// afterwards from slots first .. first + count - 1 (Split).
struct Chunk {
    int64_t beg, end;
    int32_t row, slot;
};
struct Split {
    int32_t row, first, count, pad;
};

constexpr int kSegs = 8;           // column segments of split rows: the XCDs of an MI355X
constexpr int kBlock = 256;        // threads per workgroup of every kernel here
constexpr int kHeavyPerCUMax = 8;  // most resident workgroups per CU of the persistent heavy-chunk kernel
constexpr int kHeavyGridCap = 2048;  // most workgroups of the heavy-chunk kernel (8 per CU on 256 CUs)
constexpr int kTileRows = 256;     // rows per light-kernel workgroup (one FP64 partial row each)
constexpr int kQ = 4;              // FP64 partial sums per column: N, D, a = phi^T v, S_L = L^T v
constexpr int kReduceSlices = 256; // first-stage workgroups of the deterministic reduction
constexpr int kScalars = 6;        // per-column scalars kept on the device (see Sc below)
// Gram products of the Riemannian call at 9 <= k <= 16, formed in the edge pass: kGramQ k x k FP64 partials
// per light tile and per workgroup (at most kGramHeavyBlocks) over the heavy rows, summed in fixed
// order through kGramMid and kGramMid / 32 intermediate rows to one.
constexpr int kGramQ = 4;
constexpr int kGramK = 16;
constexpr int kGramHeavyBlocks = 256;
constexpr int kGramMid = 1024;
// Rows of kGramQ * kGramK^2 doubles in the Gram area of a graph with `tiles` light tiles.
inline int64_t gram_area_rows(int64_t tiles) { return tiles + kGramHeavyBlocks + kGramMid + kGramMid / 32 + 1; }

// Index of each per-column scalar in Graph::scalars ([kScalars][k_max]).
enum Sc { SC_N = 0, SC_D = 1, SC_F = 2, SC_PD = 3, SC_A = 4, SC_B = 5 };

struct Graph {
    int64_t n = 0, nnz = 0;
    const int64_t *rowptr = nullptr;
    const int32_t *col = nullptr;
    const void *w = nullptr;
    pspec_dtype wtype = PSPEC_F32;
    int k_max = 0;
    int device = 0;
    int64_t tiles = 0;         // light tiles = ceil(n / kTileRows)
    int64_t heavy_rows = 0, n_chunks = 0, n_split = 0, n_split_chunks = 0;
    int64_t seg_chunk_base[kSegs + 1] = {};  // chunks of segment s: [seg_chunk_base[s], seg_chunk_base[s + 1]);
                                             // the shared list follows, up to n_chunks
    int64_t heavy_grid_max = 0;  // most workgroups of the heavy-chunk kernel (one partial row each)
    int cus = 1;                 // compute units of the device
    Chunk *chunks = nullptr;   // device [n_chunks]
    Split *splits = nullptr;   // device [n_split]
    double *partials = nullptr;   // device [(tiles + heavy_grid_max) * kQ * k_max]
    double *red1 = nullptr;       // device [kReduceSlices * kQ * k_max]
    double *scalars = nullptr;    // device [kScalars * k_max]
    double *chunk_scratch = nullptr;  // device [n_split_chunks * 2 * k_max] (row partials of split rows)
    // Every row's columns ascend: then ustart[i] is the first position of row i holding a column
    // above i, and the objective pass visits each undirected edge once (entries j > i only).
    bool ascending = false;
    const int64_t *ustart = nullptr;  // device [n]
    double *gram_part = nullptr;      // device [gram_area_rows(tiles)][kGramQ * kGramK^2] (k_max > 8), else NULL
    // Light tiles' rows ordered by degree: the light kernel takes row lperm[tile * kTileRows + slot]
    // in slot order (NULL: no light rows).  FP64 calls always use it; FP32 calls only when
    // sorted_tiles (light-row degrees vary widely), else node order.
    bool sorted_tiles = false;
    const int32_t *lperm = nullptr;   // device [n]
    hipEvent_t ev_before = nullptr, ev_after = nullptr;  // optional edge-pass timing events
};

// ---- device helpers ---------------------------------------------------------------------------
// Buffer-resource loads: 32-bit byte offsets from a base with a hardware range check (an offset
// beyond `bytes` reads 0 instead of faulting).  gfx9-family descriptor word 3.
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3);
}

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off);

template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Bytes spanned by an n x k block with leading dimension ld (elements of `esize` bytes).
inline uint64_t block_extent(int64_t n, int k, int64_t ld, size_t esize) {
    return ((uint64_t)(n - 1) * (uint64_t)ld + (uint64_t)k) * esize;
}

// True if two row-major n x k blocks share an element.  Equal leading dimensions are checked exactly
// (the two halves of one n x 2k array do not overlap); otherwise by address range.
bool blocks_overlap(const void *a, int64_t lda, const void *b, int64_t ldb, int64_t n, int k, size_t es);

inline int pad_k(int k) {
    int K = 4;
    while (K < k) K <<= 1;
    return K;
}

}  // namespace pspec

struct pspec_graph_s : pspec::Graph {};
