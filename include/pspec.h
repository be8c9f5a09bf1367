/*
 * pspec -- graph p-Laplacian hot path of p-spectral clustering on the Grassmann manifold,
 * for AMD Instinct MI355X (gfx950).  C ABI of libpspec.so.
 *
 * The method (Pasadakis, Schenk, Vlacic, Yzelman, "Nonlinear spectral clustering with C++
 * GraphBLAS", Section 2) minimises, over U in Gr(k, n),
 *
 *     F_p(U) = sum_l sum_{i,j} w_ij |u_i^l - u_j^l|^p / (2 ||u^l||_p^p),   p in (1, 2]   (Eq. (1))
 *
 * with (Delta_p u)_i = sum_j w_ij phi_p(u_i - u_j), phi_p(x) = |x|^(p-1) sign(x) and
 * ||u||_p^p = sum_i |u_i|^p (Section 2), by Newton's method with truncated CG, which needs the
 * gradient (the EucGrad callback) and Hessian-vector products (the EucHessianEta callback,
 * Algorithm 1).  This library evaluates those callbacks and the Grassmann projection and
 * retraction around them on the GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graph.   Symmetric CSR with both directions of every edge stored: rowptr (int64, n+1,
 *          rowptr[0] = 0, non-decreasing, rowptr[n] = nnz), col (int32, nnz, 0 <= col < n) and w
 *          (nnz weights, w_ij = w_ji, w > 0).  Self-loops contribute nothing (x = 0) and are allowed.
 * Blocks.  U, V, G, HV, Z, ... are n x k, ROW-MAJOR with leading dimension ld >= k (element (i, l)
 *          at ptr[i*ld + l]); column l is the vector u^l of Eq. (1).  The paper's eta is k x n;
 *          the transpose is used here so that one edge touches k contiguous values.  Passing U and V
 *          as the two halves of one n x 2k array (ldu = ldv = 2k, V = U + k) is supported and makes
 *          each neighbour gather a single contiguous 2k-value row.
 * Memory.  Every array argument is a DEVICE pointer owned by the caller, unless stated otherwise.
 *          Scalar results (F, F_col, M) are FP64 device arrays, so the caller decides when to copy.
 *          The library never allocates device memory: every buffer beyond the inputs and outputs
 *          is a workspace the caller passes in (sizes from the *_workspace_bytes functions).
 * Streams. Every call enqueues its kernels on `stream` and returns without synchronising, except
 *          pspec_graph_create and pspec_graph_exact_workspace (which synchronise `stream` twice,
 *          see there).  `stream` may be NULL
 *          (the null stream).  A graph handle holds the scratch of its calls: at most one call per
 *          handle may be in flight at a time.
 * Types.   dt = PSPEC_F32: U/V/G/HV are float; edge arithmetic in FP32 (|x|^(p-2) as
 *          exp2((p-2) log2 max(|x|, 2^-64)) with the hardware exp2/log2), every reduction (numerators,
 *          p-norms, dot products, Gram matrices) in FP64.
 *          dt = PSPEC_F64: everything double; |x|^(p-2) by the library's own exp((p-2) ln x),
 *          table-driven (Tang's logarithm and exponential: 128-entry tables, ln x and (p-2) ln x
 *          in double-double; within 0.52 units in the last place of the C library's pow on a CPU
 *          transcription), with x clamped to [2^-512, inf) (so only 0 < |x| < 2^-512 is affected;
 *          exact zeros stay exact) and exactly 1 at p = 2.
 * Errors.  Argument errors are found on the host before anything is launched and return
 *          PSPEC_ERR_ARG (PSPEC_ERR_UNSUPPORTED for valid but unsupported requests); a failed HIP
 *          call returns PSPEC_ERR_HIP.  pspec_last_error() describes the last failure of the
 *          calling thread.  A column with ||u^l||_p = 0 makes F_l undefined: F_l and that column of
 *          G and HV come out NaN (IEEE propagation); this is not reported as an error.
 * Near 0.  The singularity of |x|^(p-2) at x = 0 in the Hessian is removed with the caller's eps:
 *          psi(x) = max(|x|, eps)^(p-2), applied to the edge terms and to the diagonal p-norm term.
 *          phi_p and |x|^p are evaluated exactly (0 at x = 0).  The FP32 path evaluates
 *          |x|^(p-2) at max(|x|, 2^-64), which changes nothing for exact zeros and only affects
 *          differences 0 < |x| < 2^-64.
 */
#ifndef PSPEC_H
#define PSPEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSPEC_OK = 0,
    PSPEC_ERR_ARG = 1,         /* invalid argument (detected on the host, nothing launched) */
    PSPEC_ERR_UNSUPPORTED = 2, /* valid but outside what this build supports (e.g. k > 64) */
    PSPEC_ERR_HIP = 3,         /* a HIP runtime call failed */
    PSPEC_ERR_WORKSPACE = 4    /* the caller's workspace is too small */
} pspec_status;

typedef enum { PSPEC_F32 = 0, PSPEC_F64 = 1 } pspec_dtype;

/* Opaque handle (a small host object): a CSR graph and the row schedule and scratch built in the
 * caller's workspace, both borrowed. */
typedef struct pspec_graph_s *pspec_graph;

/* HIP's hipStream_t and hipEvent_t, declared opaquely so this header needs no HIP headers. */
typedef struct ihipStream_t *pspec_stream;
typedef struct ihipEvent_t *pspec_event;

/* Largest k supported by the kernels of this build. */
#define PSPEC_K_MAX 64

/*
 * Graph workspace.  A graph handle keeps its state (the state behind the EucGrad / EucHessianEta
 * callbacks of Section 2: row schedule, FP64 partial sums, per-column scalars, partial rows of long
 * rows) in device memory the caller provides.  Two ways to size it:
 *
 * pspec_graph_workspace_bytes -- a bound from the sizes alone, enough for every CSR with n nodes
 *   and nnz stored entries.  With h = min(n, nnz / (PSPEC_LIGHT_MAX + 1)) possible heavy rows,
 *   s = min(n, nnz / (PSPEC_CHUNK + 1)) possible split rows and c = nnz / PSPEC_CHUNK + 8 s possible
 *   chunks of split rows, it is about
 *     24 (h + c) + 16 s + 16 k_max c + 32 k_max (n / 256 + 2048) + 8240 k_max + 8 n + 96 n / 256
 *       + (k_max > 8 ? 8192 (n / 256 + 1313) : 0)
 *   bytes (SBM n = 8M, nnz = 96M, k_max = 16: ~900 MB; R-MAT n = 4.2M, nnz = 128M, k_max = 32:
 *   ~1.5 GB).  The last term holds the FP64 Gram partials of pspec_rhvp / pspec_rhess at
 *   9 <= k <= 16 in FP32, formed inside the edge pass (one 4 x k x k partial per 256 rows).
 *   Returns 0 for arguments pspec_graph_create would reject (n < 1, nnz < 0, k_max outside
 *   1..PSPEC_K_MAX, n >= 2^31 - 1).
 *
 * pspec_graph_exact_workspace -- the exact size for one graph: validates the CSR and counts its
 *   schedule in `workspace` (device, 256-byte aligned, at least
 *   pspec_graph_count_workspace_bytes(n, k_max) bytes: the counters, row starts and partial sums,
 *   which depend on n and k_max only), writes the bytes pspec_graph_create needs for this graph to
 *   *needed (a host size_t) and synchronises `stream` twice (after validation, after counting).
 *   The same workspace, grown to *needed bytes, can then be passed to pspec_graph_create (SBM
 *   n = 8M, k_max = 16: ~355 MB; R-MAT-22, k_max = 32: ~380 MB).  Arguments and errors as for
 *   pspec_graph_create.
 */
size_t pspec_graph_workspace_bytes(int64_t n, int64_t nnz, int k_max);
size_t pspec_graph_count_workspace_bytes(int64_t n, int k_max);
pspec_status pspec_graph_exact_workspace(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col, int k_max,
                                         void *workspace, size_t ws_bytes, pspec_stream stream, size_t *needed);

/*
 * pspec_graph_create -- build the row schedule of a graph (degree binning) in caller memory.
 *   n, nnz          nodes and stored nonzeros (n >= 1, nnz >= 0).
 *   rowptr, col, w  device CSR arrays as described above; BORROWED: they must stay valid and
 *                   unchanged while the handle is used.
 *   wtype           element type of w.  F32 calls need PSPEC_F32 weights; F64 calls accept
 *                   either (FP32 weights are promoted exactly).
 *   k_max           largest k any later call on this handle will use (1..PSPEC_K_MAX).
 *   workspace       device memory of ws_bytes >= pspec_graph_workspace_bytes(n, nnz, k_max) bytes
 *                   (or at least the exact size pspec_graph_exact_workspace reports for this graph),
 *                   256-byte aligned, owned by the caller and BORROWED like the CSR (a smaller one
 *                   returns PSPEC_ERR_WORKSPACE).  Its contents need no initialisation.
 *   stream          the schedule is built on this stream; the call synchronises it twice, after
 *                   validating the CSR and to read back the sizes of the schedule.
 *   out             receives the handle (a small host object).
 * Rows are binned by degree: rows with at most PSPEC_LIGHT_MAX neighbours are processed by a
 * 16-lane group per row (4 lanes for k <= 4, 8 for k <= 8), in node order or in degree order
 * within each 256-row tile (rows of equal degree by their count of entries above the diagonal;
 * FP64 calls always in degree order; see pspec_graph_degree_order); rows of up to PSPEC_CHUNK
 * edges are one chunk each, handed
 * out in a fixed order to one wavefront each; longer rows are cut at 8 column-segment boundaries
 * (node-id ranges holding equal shares of the stored entries) and each piece into chunks of at
 * most PSPEC_CHUNK edges, the chunks of segment s going to the workgroups that run on XCD s (the
 * objective walks all chunks with one stride), and such rows are combined in a fixed order
 * afterwards, so every result is bit-reproducible.  Any
 * column order within a row is valid; ascending columns (the usual CSR) let each XCD's L2 cache
 * the neighbour rows of one segment only, and let pspec_objective visit each undirected edge once
 * (pspec_graph_ascending).  The CSR is validated on the device (rowptr monotone with
 * rowptr[0] = 0 and rowptr[n] = nnz, every column in [0, n)); a malformed graph returns
 * PSPEC_ERR_ARG.  No device memory is allocated.
 */
#define PSPEC_LIGHT_MAX 32
#define PSPEC_CHUNK 512
pspec_status pspec_graph_create(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                                const void *w, pspec_dtype wtype, int k_max, void *workspace, size_t ws_bytes,
                                pspec_stream stream, pspec_graph *out);

/* Releases the handle (host memory only; no device call, no synchronisation).  The workspace and
 * the CSR stay the caller's: they may be released once the work enqueued on the handle has
 * completed.  NULL is a no-op. */
pspec_status pspec_graph_destroy(pspec_graph g);

/* Schedule statistics: rows above PSPEC_LIGHT_MAX, chunks, rows spanning several chunks. */
pspec_status pspec_graph_info(pspec_graph g, int64_t *heavy_rows, int64_t *chunks, int64_t *split_rows);

/* *ascending (host int) = 1 if every row's columns are non-decreasing (checked at create), else 0.
 * With ascending rows pspec_objective visits each undirected edge once (see there). */
pspec_status pspec_graph_ascending(pspec_graph g, int *ascending);

/* *on (host int) = 1 if FP32 calls take each 256-row tile's light rows in order of degree, else 0
 * (node order).  pspec_graph_create chooses degree order for FP32 when the degrees of the rows of at
 * most PSPEC_LIGHT_MAX entries have a coefficient of variation above 1 (power-law graphs), so that
 * the rows sharing a wavefront are about equally long; on graphs of near-uniform degree node order
 * keeps the row writes contiguous, which counts for more in the gather-bound FP32 pass.  FP64 calls,
 * bound by the arithmetic, take degree order on every graph.  Results do not depend on the order
 * beyond summation order. */
pspec_status pspec_graph_degree_order(pspec_graph g, int *on);

/*
 * pspec_rcm_order -- a locality relabelling of the graph for the edge pass (the vxm of Section 2
 * gathers one neighbour row per edge; graphs numbered without locality, such as triangulations of
 * random points, make every gather a cache miss).  Reverse Cuthill-McKee: per connected component
 * a breadth-first sweep from a pseudo-peripheral node (George-Liu), unvisited neighbours taken in
 * increasing (degree, id), components in increasing (degree, id) of their first node, the whole
 * sequence reversed.  Writes perm[old id] = new id (a permutation of 0..n-1).  Host code: rowptr
 * (n + 1), col (rowptr[n]) and perm (n) are HOST arrays; the graph must be symmetric (the order is
 * valid for any graph, its locality only for symmetric ones).  The caller relabels the CSR and the
 * rows of U once and solves in the new order; nothing in the library applies it.  Invalid CSR
 * returns PSPEC_ERR_ARG.  O(nnz log(max degree)) time, O(n) extra memory.
 */
pspec_status pspec_rcm_order(int64_t n, const int64_t *rowptr, const int32_t *col, int64_t *perm);

/*
 * Timing hook (for benchmarks).  While set, every pspec_objective / pspec_grad / pspec_hvp call on
 * this handle records `before` on its stream immediately before the first kernel of the edge pass
 * and `after` immediately after its last one (light rows, heavy chunks, split-row combine), so
 * hipEventElapsedTime(before, after) is the duration of the edge pass alone.  The events are
 * created and owned by the caller; pass NULL for both to stop recording.
 */
pspec_status pspec_graph_set_timing_events(pspec_graph g, pspec_event before, pspec_event after);

/*
 * pspec_objective -- Eq. (1).  F_col[l] = N_l / D_l with N_l = (1/2) sum over stored edges of
 * w_ij |u_i^l - u_j^l|^p and D_l = ||u^l||_p^p; *F = sum_l F_col[l].
 *   U      n x k block (dt), leading dimension ldu.
 *   F_col  device, k doubles, may be NULL;  F  device, 1 double, may be NULL.
 * When every row's columns ascend (pspec_graph_ascending), N_l is summed over the entries with
 * j > i only, which for the symmetric graphs this library takes is the same sum (w and |x|^p are
 * symmetric in i, j): half the gathers.  F_col then agrees with the F_col of the other calls to
 * rounding, not bit for bit.  Otherwise every stored entry is visited and the result is bitwise
 * that of pspec_grad / pspec_hvp.
 */
pspec_status pspec_objective(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, double p,
                             double *F_col, double *F, pspec_stream stream);

/*
 * pspec_grad -- Euclidean gradient of Eq. (1) (the EucGrad callback of Section 2):
 *   G[i, l] = (p / D_l) ((Delta_p u^l)_i - F_l phi_p(u_i^l)).
 *   G      n x k output (dt), leading dimension ldg; must not overlap U.
 *   F_col  device, k doubles (the objective per column, computed on the way), may be NULL.
 */
pspec_status pspec_grad(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, double p,
                        void *G, int64_t ldg, double *F_col, pspec_stream stream);

/*
 * pspec_hvp -- Hessian-vector product of Eq. (1) (the EucHessianEta callback, Algorithm 1), fused
 * with the gradient, in one pass over the edges:
 *   HV[:, l] = H^l(U) V[:, l] where, with D = D_l, F = F_l, g = G[:, l], phi = phi_p(u^l),
 *   (H v)_i = (p/D) [ (p-1) sum_j w_ij psi(u_i - u_j)(v_i - v_j) - F (p-1) psi(u_i) v_i
 *                     - g_i (phi^T v) - phi_i (g^T v) ]
 *   (the exact Hessian of Eq. (1): Algorithm 1's diag(H^l) eta - (diag(H^l) - H^l) eta).
 *   V      n x k direction (dt), leading dimension ldv (may be U + k with ldu = ldv, see above).
 *   eps    > 0, the cap of psi (see "Near 0").
 *   HV, G  n x k outputs (dt); G is REQUIRED (the gradient is a by-product of the pass); neither
 *          may overlap U, V or each other.
 *   F_col  device, k doubles, may be NULL.
 */
pspec_status pspec_hvp(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                       int64_t ldv, double p, double eps, void *HV, int64_t ldh, void *G, int64_t ldg,
                       double *F_col, pspec_stream stream);

/*
 * pspec_hvp_sparse -- pspec_hvp with the Hessian restricted to its sparse part, the reading of
 * Algorithm 1 in which D[l] = diag(H^l) and H[l] = diag(H^l) - H^l are GraphBLAS matrices with the
 * sparsity of the graph: HV = (p/D)((p - 1) J - F (p - 1) psi(u) v), i.e. the exact Hessian-vector
 * product without its dense rank-2 part -(p/D)(g phi^T + phi g^T) v.  G, F_col, arguments, layout
 * and errors are those of pspec_hvp (G is the exact gradient).  For comparison with the paper's
 * formulation; Newton on this operator is an inexact Newton method.
 */
pspec_status pspec_hvp_sparse(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                              int64_t ldv, double p, double eps, void *HV, int64_t ldh, void *G, int64_t ldg,
                              double *F_col, pspec_stream stream);

/*
 * pspec_hvp_gather_floor -- a MEASUREMENT REFERENCE, not part of the method: the FP32 edge pass of
 * pspec_hvp (same kernels, launch geometry, schedule, neighbour gathers, row stores and reductions)
 * with the arithmetic of every edge-column term replaced by a plain sum of the gathered values.
 * Its duration bounds from below what any arithmetic of the same gathers can take, so the ratio of
 * the two edge-pass times says how far the real pass is from its own memory floor.  HV and G
 * receive meaningless values; the handle's per-column scalars are overwritten.  Arguments, layout
 * and errors are those of pspec_hvp with dt = PSPEC_F32 (no p, eps or F_col).  The timing hook
 * (pspec_graph_set_timing_events) brackets its edge pass as for pspec_hvp.
 */
pspec_status pspec_hvp_gather_floor(pspec_graph g, int k, const void *U, int64_t ldu, const void *V, int64_t ldv,
                                    void *HV, int64_t ldh, void *G, int64_t ldg, pspec_stream stream);

/*
 * Dense n x k operations of the Grassmann geometry (the manifold of Section 2; the formulas are
 * the standard ones of the Edelman-Arias-Smith geometry the paper cites).  They need a caller
 * workspace of pspec_dense_workspace_bytes(k) bytes (device, 256-byte aligned); one call per
 * workspace may be in flight at a time.
 */
size_t pspec_dense_workspace_bytes(int k);

/*
 * pspec_project -- tangent projection at U (orthonormal columns):
 *   M   = U^T Z                                  (k x k, FP64, row-major, written if M != NULL)
 *   out = Z - U M - X MX                         (the X MX term only if X != NULL)
 * With X = eta and MX = U^T G this gives the Riemannian Hessian P_U(H eta) - eta (U^T G).
 *   MX   device k x k FP64 row-major (required when X != NULL).
 *   out  may be the same array as Z (same ld); must not overlap U or X otherwise.
 */
pspec_status pspec_project(int64_t n, int k, pspec_dtype dt, const void *U, int64_t ldu, const void *Z,
                           int64_t ldz, const void *X, int64_t ldx, const double *MX, void *out, int64_t ldo,
                           double *M, void *ws, size_t ws_bytes, pspec_stream stream);

/*
 * pspec_retract -- QR retraction: Uout = qf(U + t eta), the Q factor of the thin QR
 * factorisation with a positive diagonal of R, computed as Cholesky-QR in FP64: R = chol(Y^T Y),
 * Q = Y R^-1.  Uout may be the same array as U (same ld).  If Y is numerically rank deficient the
 * Cholesky factorisation breaks down and Uout is NaN.
 *   R  device k x k FP64 row-major upper-triangular factor (written if not NULL).
 */
pspec_status pspec_retract(int64_t n, int k, pspec_dtype dt, const void *U, int64_t ldu, const void *eta,
                           int64_t lde, double t, void *Uout, int64_t ldo, double *R, void *ws, size_t ws_bytes,
                           pspec_stream stream);

/*
 * pspec_rhvp -- Riemannian gradient and Riemannian Hessian-vector product of Eq. (1) on the
 * Grassmann manifold at U (orthonormal columns), the quantities one truncated-CG iteration of the
 * Newton method of Section 2 needs, in one call:
 *   MG = U^T G                                   (k x k, FP64, row-major, written if MG != NULL)
 *   RG = G - U MG                                (Riemannian gradient P_U(G))
 *   RH = HV - U (U^T HV) - V MG                  (Riemannian Hessian P_U(H V) - V (U^T G))
 * where G and HV are the outputs of pspec_hvp.  G and HV are never written: in FP32 at
 * 9 <= k <= 16 the edge pass itself forms the Gram products U^T (Delta_p u), U^T J, U^T phi_p(u)
 * and U^T (psi(u) v) on the matrix cores, row by row as it finishes them, and MG and U^T HV are
 * combined from these in FP64 (no pass over the rows between the edge pass and the projection);
 * the results then agree with pspec_hvp followed by pspec_project(U, G) and
 * pspec_project(U, HV, X = V, MX = MG) to rounding.  Otherwise one pass forms the epilogue and both
 * Gram matrices and the results are bit-identical to that sequence.
 *   V       n x k tangent direction (dt), leading dimension ldv (may be U + k with ldu = ldv).
 *   RH, RG  n x k outputs (dt); both REQUIRED; neither may overlap U, V or each other.
 *   F_col   device, k doubles (the objective per column), may be NULL.
 *   ws      device workspace of pspec_dense_workspace_bytes(k) bytes, 256-byte aligned; shared
 *           with no other call in flight.
 */
pspec_status pspec_rhvp(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                        int64_t ldv, double p, double eps, void *RH, int64_t ldrh, void *RG, int64_t ldrg,
                        double *MG, double *F_col, void *ws, size_t ws_bytes, pspec_stream stream);

/*
 * pspec_rhess -- the Riemannian Hessian-vector product of pspec_rhvp at a point U whose Euclidean
 * gradient G is already known: the form truncated CG needs, since U stays fixed while the Hessian is
 * applied to one direction after another within a Newton step (Section 2):
 *   RH = HV - U (U^T HV) - V MG,   MG = U^T G   (MG written if not NULL)
 * with HV the exact Hessian-vector product of pspec_hvp.  G (n x k, dt, leading dimension ldg) is
 * the Euclidean gradient at U as pspec_grad or pspec_hvp returns it; it is only read.  Compared
 * with pspec_rhvp the edge pass forms no (Delta_p u) rows and writes none, g^T v is summed from G
 * directly, and RG is not formed or written: one n x k row block less written per call on each side
 * (SBM n = 8M, k = 16: 1 GB of the ~20 GB a pspec_rhvp call moves).  RH agrees with pspec_rhvp's
 * to rounding (b = g^T v is summed from the rounded G instead of from (Delta_p u)^T v), F_col bit
 * for bit, MG bit for bit unless the Gram products are formed in the edge pass (FP32,
 * 9 <= k <= 16: then to rounding).  V, RH, ws, F_col, layout and errors as for pspec_rhvp; RH must not overlap U, V or
 * G.
 */
pspec_status pspec_rhess(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                         int64_t ldv, const void *G, int64_t ldg, double p, double eps, void *RH, int64_t ldrh,
                         double *MG, double *F_col, void *ws, size_t ws_bytes, pspec_stream stream);

/*
 * pspec_rhvp_static -- pspec_rhvp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): no workspace argument; the
 * Gram partials and k x k matrices live in a file-scope device array of the library, one per GPU,
 * of pspec_dense_workspace_bytes(PSPEC_STATIC_K_MAX) bytes (17,318,400 bytes, held by every GPU the library
 * runs on until the process ends).  Results are identical to pspec_rhvp's, bit for bit.
 *   k    1..PSPEC_STATIC_K_MAX; a wider block returns PSPEC_ERR_UNSUPPORTED.
 * Every call on one GPU uses that GPU's single array: calls that overlap in time on one GPU (two
 * streams, two threads) race and must be serialised by the caller.  The array keeps the last
 * call's contents; nothing in it needs clearing between calls.  Other arguments, layout and errors
 * are those of pspec_rhvp.  The graph handle's own workspace is the caller's, as always.
 */
#define PSPEC_STATIC_K_MAX 32
pspec_status pspec_rhvp_static(pspec_graph g, pspec_dtype dt, int k, const void *U, int64_t ldu, const void *V,
                               int64_t ldv, double p, double eps, void *RH, int64_t ldrh, void *RG, int64_t ldrg,
                               double *MG, double *F_col, pspec_stream stream);

/* pspec_dot -- *out = sum_{i,l} A[i,l] B[i,l] (Frobenius inner product, FP64, fixed order). */
pspec_status pspec_dot(int64_t n, int k, pspec_dtype dt, const void *A, int64_t lda, const void *B, int64_t ldb,
                       double *out, void *ws, size_t ws_bytes, pspec_stream stream);

/* pspec_axpby -- Y = alpha X + beta Y (elementwise, n x k; beta = 0 ignores Y's old contents). */
pspec_status pspec_axpby(int64_t n, int k, pspec_dtype dt, double alpha, const void *X, int64_t ldx, double beta,
                         void *Y, int64_t ldy, pspec_stream stream);

/*
 * k-means discretisation (Section 1: the rows of the minimiser U are grouped into clusters by
 * k-means; the paper does not fix the variant).  One Lloyd step on the rows of the n x d block X:
 *   labels[i] = the first j minimising dist(i, j) = sum_{t < d} (X[i,t] - C[j,t])^2, the sum taken in
 *               t order in FP64, each square rounded before it is added (ties go to the lower j);
 *   dist[i]   = that minimum;
 *   stats[j * (d + 2) + t] = sum of X[i,t] over the rows i with labels[i] = j      (t < d),
 *   stats[j * (d + 2) + d] = the number of such rows, stats[j * (d + 2) + d + 1] = the sum of their
 *               dist (per-cluster inertia).
 * The next Lloyd centroids are stats[j, t] / stats[j, d].  labels and dist are exact functions of X
 * and C; stats are FP64 sums in a fixed order, identical from run to run.  X must be finite.
 *   n           rows (0 is allowed: stats are then zero and labels, dist untouched).
 *   d, c        columns and clusters, 1..PSPEC_KMEANS_MAX each.
 *   X           device, n x d (dt), row-major with leading dimension ldx >= d.
 *   C           device, c x d FP64 centroids, row-major, leading dimension d.
 *   labels      device, n int32, or NULL;  dist: device, n doubles, or NULL.
 *   stats       device, c * (d + 2) doubles (REQUIRED).
 *   ws          device workspace of pspec_kmeans_workspace_bytes(c, d) bytes, 256-byte aligned,
 *               shared with no other call in flight.
 */
#define PSPEC_KMEANS_MAX 32
size_t pspec_kmeans_workspace_bytes(int c, int d);
pspec_status pspec_kmeans_step(int64_t n, int d, pspec_dtype dt, const void *X, int64_t ldx, int c, const double *C,
                               int32_t *labels, double *dist, double *stats, void *ws, size_t ws_bytes,
                               pspec_stream stream);

/* Message describing the last non-OK status returned on the calling thread ("" if none). */
const char *pspec_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSPEC_H */
