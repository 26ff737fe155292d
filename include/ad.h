/*
 * ad.h -- C ABI of the MI355X (gfx950) algebraic-distance sparsification
 * library (libad.so).
 *
 * The method (John & Safro, "Single- and Multi-level Network Sparsification
 * by Algebraic Distance", arXiv 1601.05527):
 *   Algorithm 1 (ComputeAlgDist): R random test vectors, k Jacobi
 *     over-relaxation (JOR) sweeps each, a rescale of every vector back to
 *     (-1/2, 1/2), and the per-edge L2 algebraic distance
 *     rho_ij = sqrt(sum_r (xhat_i - xhat_j)^2); the paper's strength is
 *     delta_ij = 1/sqrt(rho_ij^2 + eps), large for close (delta-strong) pairs.
 *   Algorithm 3 (Sparsify): every vertex keeps its top d_i^e neighbours,
 *     ranked by delta ascending or descending; the sparse graph is the union.
 *   Section 6.2: e is fitted by binary search to a target retention ratio.
 *   Algorithm 4 (SparsifyB): the selection with per-vertex bins.
 *   Algorithm 6 (MLSparsify): the multilevel cycle (coarsening by seeds and
 *     the restriction P, Galerkin coarse graphs, inheritance on the way back).
 *   Around the path: an edge-list ingest into the graph model of Section 2,
 *     and the graph properties of the Preliminaries for comparing G_s with G.
 *
 * Conventions for every call below.
 *   - Pointers are DEVICE pointers unless the name ends in _host.
 *   - The caller owns every buffer.  The library reads/writes them only from
 *     work enqueued on the caller's stream and never keeps them after that
 *     work completes.  No call allocates or frees device memory except
 *     ad_ml_sparsify and the ad_batch_* object; scratch space comes from the
 *     caller's workspace `ws` of `ws_bytes` bytes (at least what the matching
 *     *_workspace_size call returns, 256-byte aligned).
 *   - Calls only enqueue work on `stream` and return, except where a call
 *     says it synchronises.
 *   - Errors: host-side argument checks return AD_ERR_INVALID_ARG,
 *     AD_ERR_UNSUPPORTED or AD_ERR_WORKSPACE before any work is enqueued; a
 *     failed HIP launch or copy returns AD_ERR_HIP.  ad_last_error() gives a
 *     thread-local message for the last failure.  No C++ exception crosses
 *     this boundary.  The library does not check the graph's structure on
 *     the device except in ad_validate_graph.
 *   - Calls that share a workspace must not overlap (same stream, or
 *     ordered by the caller).
 *   - Library-owned state: the selection calls on FP32 distances
 *     (ad_sparsify, ad_sparsify_fit, ad_sparsify_fit_both,
 *     ad_edge_dist_sparsify, ad_edge_dist_fit_both, ad_sparsify_binned)
 *     rank rows longer than 64 on three helper streams per device, of
 *     default priority, created on first use and kept until
 *     the process ends; they are forked from the caller's stream with an
 *     event after the call's first kernels and joined back into it with
 *     events before the call returns, so the caller's stream orders all of
 *     the call's work, and a per-device mutex serialises the forks of calls
 *     made from several host threads.  Under stream capture the call stays
 *     on the caller's stream.  The retention fits (ad_sparsify_fit,
 *     ad_sparsify_fit_both, ad_edge_dist_fit_both, ad_sparsify_binned with
 *     a target) share one pinned, device-mapped host buffer for their
 *     budget tables and read-backs, grown on demand and kept until the
 *     process ends; a mutex lets one fit at a time use it, so fits from
 *     several host threads run one after another.  The kernel trace
 *     (ad_trace_*) keeps a pool of events per device.
 */
#ifndef AD_H
#define AD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The enum types below have int32_t as their underlying type in C++ too, so
 * that any 32-bit value a caller passes is a value of the type: an unknown
 * one reaches the argument checks and is rejected with AD_ERR_INVALID_ARG. */
#ifdef __cplusplus
#define AD_ENUM_I32 : int32_t
#else
#define AD_ENUM_I32
#endif

typedef enum AD_ENUM_I32 {
    AD_OK = 0,
    AD_ERR_INVALID_ARG = 1,   /* a null pointer, a size or a parameter out of range  */
    AD_ERR_UNSUPPORTED = 2,   /* a valid but unimplemented combination               */
    AD_ERR_WORKSPACE = 3,     /* ws too small or misaligned                          */
    AD_ERR_GRAPH = 4,         /* a structural defect (ad_validate_graph, ad_ingest)  */
    AD_ERR_HIP = 5,           /* a HIP runtime call failed                           */
    AD_ERR_INTERNAL = 6       /* an internal consistency check failed                */
} ad_status;

typedef enum AD_ENUM_I32 { AD_F64 = 0, AD_F32 = 1, AD_BF16 = 2 } ad_dtype;

/* Orientation of the per-vertex ranking (Algorithm 3 sorts N_i by delta in
 * ascending or descending order; Section 4 names the two uses):
 *   AD_LOCAL  keeps the delta-strong edges = smallest rho first
 *             ("preserve local structure");
 *   AD_GLOBAL keeps the delta-weak edges   = largest rho first
 *             ("preserve global structure").
 * Ties in rho go to the neighbour with the smaller orig_id in both. */
typedef enum AD_ENUM_I32 { AD_LOCAL = 0, AD_GLOBAL = 1 } ad_orient;

/* Symmetric CSR of an undirected simple weighted graph G = (V, E, w)
 * (Preliminaries: undirected, no self-loops, no multi-edges, w >= 0; this
 * library requires finite w > 0 so that every non-isolated vertex has a
 * positive weighted degree). */
typedef struct {
    int64_t n;                /* |V|                                                   */
    int64_t m;                /* |E|, undirected edges; row_ptr[n] == 2m              */
    const int64_t *row_ptr;   /* [n+1]                                                 */
    const int32_t *col;       /* [2m] neighbour of each stored entry, ascending within
                                 each row (ad_validate_graph checks it)                 */
    const float *w;           /* [2m] w_ij == w_ji; NULL means unit weights            */
    const int32_t *eid;       /* [2m] undirected edge id in [0, m); (i,j) and (j,i)
                                 share it                                              */
    const int32_t *orig_id;   /* [n] vertex id before any relabelling (keys the random
                                 start vectors, breaks ranking ties); NULL = identity  */
    int32_t d_max;            /* host value: maximum degree (selection calls need it) */
    const int32_t *col_orig;  /* [2m] optional: orig_id[col[p]] per entry (ad_graph_col_orig
                                 builds it); lets ranking read neighbour ids in storage
                                 order instead of gathering them; NULL = gather          */
} ad_graph;

/* Connected components of a graph, grouped so that the relaxation can centre
 * each component by its own weighted mean (see ad_relax).  Built once per
 * graph by ad_components_build; every array is DEVICE memory owned by the
 * caller.  Isolated vertices (no edges) belong to no component.           */
typedef struct {
    int64_t n_comp;           /* host: components with at least one edge               */
    int64_t n_chunks;         /* host: sum over components of ceil(size / 256)         */
    const int32_t *comp_of;   /* [n] component of each vertex, -1 when isolated        */
    const int32_t *members;   /* [n_live] the non-isolated vertices, component by
                                 component (components in increasing order of their
                                 smallest vertex, vertices ascending within each)      */
    const int64_t *comp_start;/* [n_comp+1] offsets of the components in members       */
    const int64_t *chunk_start;/* [n_comp+1] cumulative 256-member chunks              */
} ad_components;

/* Parameters of Algorithm 1's relaxation. */
typedef struct {
    int32_t R;                /* test vectors, 1..64                                   */
    int32_t k;                /* JOR sweeps, >= 0                                      */
    double omega;             /* weight on the neighbour average, (0, 1]; the paper's
                                 alpha (weight on the old value) is 1 - omega          */
    uint64_t seed;            /* Philox key word 0                                     */
    uint64_t graph_id;        /* Philox key word 1                                     */
    ad_dtype store;           /* AD_F64: FP64 storage and arithmetic.
                                 AD_F32: FP32 storage and arithmetic.
                                 AD_BF16: FP32 arithmetic; sweeps 1..k-fp32_tail are
                                 stored in BF16 (round to nearest even), x^(0) and the
                                 last fp32_tail sweeps in FP32                         */
    int32_t fp32_tail;        /* AD_BF16 only: number of final sweeps stored in FP32
                                 (>= 1)                                                */
    int32_t ckpt_every;       /* 0: no checkpoints.  c > 0: write x^(0), x^(c),
                                 x^(2c), ... (every t = q*c < k) to `ckpt` for
                                 ad_relax_backward                                     */
    int32_t rows_per_wave;    /* launch shape, 0 = automatic: rows sharing one 64-lane
                                 wave (power of two); results do not depend on it
                                 except through FP summation order                     */
    int32_t hub_degree;       /* launch shape, 0 = automatic: rows with more neighbours
                                 get a 256-thread workgroup each                       */
    int32_t fp64_tail;        /* AD_F32 / AD_BF16: the last fp64_tail sweeps are stored
                                 in FP64 with FP64 arithmetic (0 = none); x_out is then
                                 FP64.  With AD_BF16 it must be below fp32_tail, which
                                 counts every final sweep stored wider than BF16       */
    const ad_components *comp;/* NULL: one shift per vector (the weighted mean over the
                                 whole graph).  Else: one shift per vector and connected
                                 component (its own weighted mean), see ad_relax       */
} ad_relax_opts;

/* ----------------------------------------------------------- components -- */

/* Workspace bytes for ad_components_build (0 when n >= 2^31). */
size_t ad_components_workspace_size(const ad_graph *g);

/* The connected components of g (Preliminaries: G undirected) in the
 * grouped form of ad_components, for ad_relax's per-component centring.
 * Outputs, DEVICE and caller-owned: comp_of [n]; members [n] (the first
 * n_live written); comp_start and chunk_start [n+1] (the first n_comp + 1
 * written).  n_comp_host, n_chunks_host: HOST.  Components are labelled by
 * hooking and pointer jumping and grouped by rocPRIM's stable radix sort, so
 * the result depends only on the graph.  SYNCHRONISES `stream`.  Errors:
 * AD_ERR_INVALID_ARG, AD_ERR_WORKSPACE, AD_ERR_UNSUPPORTED (n >= 2^31). */
ad_status ad_components_build(const ad_graph *g, int32_t *comp_of, int32_t *members,
                              int64_t *comp_start, int64_t *chunk_start, int64_t *n_comp_host,
                              int64_t *n_chunks_host, void *ws, size_t ws_bytes,
                              hipStream_t stream);

/* ---------------------------------------------------------------- relax -- */

/* Workspace bytes for ad_relax on this graph and these options. */
size_t ad_relax_workspace_size(const ad_graph *g, const ad_relax_opts *o);

/* Number of checkpoint slots ad_relax writes: ceil(k / ckpt_every), or 0. */
int32_t ad_relax_num_checkpoints(const ad_relax_opts *o);

/* Algorithm 1, relaxation part: the start vectors and k JOR sweeps
 *     x_i^(t) = (1 - omega) x_i^(t-1) + omega * sum_j w_ij x_j^(t-1) / sum_j w_ij
 * (isolated vertices keep their value), followed by the min and max of each
 * vector over the non-isolated vertices, which define the rescale
 *     xhat = (x - min) / (max - min) - 1/2   (0 when max == min).
 *
 * Start vectors: x0 == NULL draws x_i^(0) for vector r as word (r % 4) of
 * Philox4x64-10(key = (seed, graph_id), counter = (orig_id[i], r / 4, 0, 0)),
 * shifted right by 40 bits, times 2^-24, minus 1/2 -- uniform on the 2^24
 * grid in [-1/2, 1/2).  Otherwise x0 holds [n][R] start values (FP64 when
 * store == AD_F64, else FP32).
 *
 * Centring (a change of frame that leaves x^(k) and xhat unchanged): the
 * sweeps keep every vector that is constant on each connected component
 * fixed, and conserve each component's weighted mean sum s_i x_i / sum s_i
 * (s_i = sum_j w_ij).  The library subtracts from x^(0), per vector, that
 * mean rounded to a multiple of 2^-24 -- one shift per component when
 * o->comp is given, else one for the whole graph -- and sweeps the
 * differences, whose rounding errors then scale with how far each
 * component still is from its own limit instead of with its mean.
 *
 * Arithmetic: AD_F64 sweeps in FP64; AD_F32 in FP32; AD_BF16 stores sweeps
 * 1..k-fp32_tail in BF16 (round to nearest even) and computes in FP32.  The
 * last fp64_tail sweeps are stored in FP64 and computed in FP64, the
 * neighbour average as a correctly rounded quotient sum_j w_ij x_j / s_i (as
 * in every FP64 sweep).
 *
 * Outputs:
 *   x_out      [n][R] row-major, FP64 when store == AD_F64 or fp64_tail > 0,
 *              else FP32: x^(k) minus the shift of the vertex's component
 *              (isolated vertices: minus 0).
 *   minmax_out [2R] doubles: min_r then max_r of x^(k) itself (shift added
 *              back) over the non-isolated vertices.
 *   shift_out  NULL, or [n_comp][R] doubles (o->comp given) or [R] doubles:
 *              the shifts above.
 *   ckpt       NULL, or [ad_relax_num_checkpoints][n][R] in x_out's type:
 *              the (shifted) x^(0), x^(c), x^(2c), ...; needs fp64_tail == 0.
 * x_out must not alias x0 or ckpt. */
ad_status ad_relax(const ad_graph *g, const ad_relax_opts *o, const void *x0,
                   void *x_out, double *minmax_out, double *shift_out, void *ckpt,
                   void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------- distance -- */

/* Workspace bytes for ad_edge_dist. */
size_t ad_edge_dist_workspace_size(const ad_graph *g);

/* Algorithm 1, distance part: for every undirected edge e = (i, j)
 *     rho_e = sqrt( sum_r ((x_i,r - x_j,r) / (max_r - min_r))^2 ),
 * i.e. the L2 distance of the rescaled vectors (a vector with max_r == min_r
 * contributes 0).  x: [n][R] in x_dtype (AD_F64 or AD_F32), as written by
 * ad_relax (both ends of an edge lie in one component, so its shift
 * cancels); minmax: [2R] doubles as written by ad_relax.  rho: [m] in
 * rho_dtype: AD_F64 needs FP64 x; AD_F32 takes either (with FP64 x the
 * arithmetic is FP64 and only rho is rounded to FP32). */
ad_status ad_edge_dist(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                       const double *minmax, ad_dtype rho_dtype, void *rho, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and kernels as ad_edge_dist, with no workspace argument.  The
 * distance pass's launch plan lives in a fixed device array of
 * ad_edge_dist_noalloc_max_bytes() bytes (32 MiB), one per GPU, which
 * exists while the library's code is loaded on that GPU (until the process
 * ends); a graph
 * whose plan needs more (ad_edge_dist_workspace_size, about 12 bytes per
 * vertex: up to roughly 2.5M vertices) is refused with AD_ERR_UNSUPPORTED
 * before any work is enqueued.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  Every call on one GPU uses that
 * GPU's array: calls that overlap on one GPU (several streams or host
 * threads at once) race on it and must be ordered by the caller.  Results
 * equal ad_edge_dist's bit for bit. */
size_t ad_edge_dist_noalloc_max_bytes(void);
ad_status ad_edge_dist_noalloc(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                               const double *minmax, ad_dtype rho_dtype, void *rho, hipStream_t stream);

/* ------------------------------------------------------------ selection -- */

/* Host helper: the per-vertex budget of Algorithm 3 for every degree,
 *     budget_host[d] = min(d, max(1, floor(pow(d, e)))),  budget_host[0] = 0,
 * for d = 0..d_max, with the C library's double pow.  e in [0, 1]. */
ad_status ad_budget_table(int32_t d_max, double e, int32_t *budget_host);

/* Workspace bytes for ad_sparsify / ad_sparsify_fit. */
size_t ad_sparsify_workspace_size(const ad_graph *g);

/* Algorithm 3 at a fixed exponent: every vertex i ranks its neighbours by
 * (rho ascending for AD_LOCAL, descending for AD_GLOBAL; then neighbour
 * orig_id ascending) and selects the first budget[d_i]; keep[e] = 1 when
 * either endpoint selects edge e, else 0.  rho: [m] in rho_dtype (AD_F64 or
 * AD_F32).  budget: DEVICE copy of ad_budget_table's [d_max+1] (or any
 * budget with budget[d] in [0, d]).  n_kept: device int64, receives sum(keep).
 */
ad_status ad_sparsify(const ad_graph *g, ad_dtype rho_dtype, const void *rho,
                      ad_orient orient, const int32_t *budget, uint8_t *keep,
                      int64_t *n_kept, void *ws, size_t ws_bytes, hipStream_t stream);

/* Algorithm 3 with e fitted to a retention target (Section 6.2's binary
 * search): returns, through e_used_host, the value the bisection
 *     lo = 0, hi = 1; if ratio(0) >= target return 0;
 *     40 times: mid = (lo + hi) / 2; ratio(mid) >= target ? hi = mid : lo = mid;
 *     return hi
 * returns, with ratio(e) = (edges kept at e) / m, and writes keep and n_kept
 * at that e.  target in (0, 1].  With m == 0 it returns e = 0.
 * SYNCHRONISES `stream` (the fit reads counts back to the host). */
ad_status ad_sparsify_fit(const ad_graph *g, ad_dtype rho_dtype, const void *rho,
                          ad_orient orient, double target, uint8_t *keep,
                          int64_t *n_kept, double *e_used_host, void *ws,
                          size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for ad_sparsify_fit_both (the ranks of both orders). */
size_t ad_sparsify_fit_both_workspace_size(const ad_graph *g);

/* ad_sparsify_fit for AD_LOCAL and AD_GLOBAL at one target from a single
 * ranking pass (Algorithm 3's two orders share each row's comparisons: the
 * LOCAL rank of an entry is #{rho' < rho} + #{rho' == rho, id' < id}, the
 * GLOBAL rank #{rho' > rho} + #{rho' == rho, id' < id}).  Outputs equal those
 * of the two single calls: keep_local, keep_global [m]; n_kept: device
 * int64[2] (local, global); e_used_host: double[2].  SYNCHRONISES `stream`. */
ad_status ad_sparsify_fit_both(const ad_graph *g, ad_dtype rho_dtype, const void *rho,
                               double target, uint8_t *keep_local, uint8_t *keep_global,
                               int64_t *n_kept, double *e_used_host, void *ws,
                               size_t ws_bytes, hipStream_t stream);

/* Distances and selection in one call: Algorithm 1's distances (as
 * ad_edge_dist writes them, FP32 rho) and Algorithm 3 on them, with results
 * equal to ad_edge_dist followed by ad_sparsify or ad_sparsify_fit_both.
 * The distance pass visits whole rows and also writes every CSR entry's
 * distance in entry order into the workspace (an edge's two entries get
 * equal values: the squared differences and their summation order are the
 * same from either end); the ranking reads its keys from there, contiguously,
 * instead of gathering rho by edge id.  R in [1, 64]; x: [n][R] in x_dtype
 * (AD_F64 or AD_F32) and minmax [2R] as ad_relax writes them; rho: [m] FP32
 * output.  Workspace: ad_edge_dist_select_workspace_size bytes (the
 * distance plan, 4 bytes per CSR entry, and the selection workspace of both
 * orders).  The other arguments are those of ad_sparsify and
 * ad_sparsify_fit_both (all buffers DEVICE and caller-owned except
 * e_used_host); ad_edge_dist_sparsify is asynchronous, ad_edge_dist_fit_both
 * SYNCHRONISES `stream`.  Errors: AD_ERR_INVALID_ARG for R outside [1, 64],
 * an x_dtype other than AD_F64 / AD_F32, a bad orientation or target, or a
 * NULL buffer that is needed; AD_ERR_WORKSPACE for a short or misaligned
 * workspace; all before any work is enqueued. */
size_t ad_edge_dist_select_workspace_size(const ad_graph *g);
ad_status ad_edge_dist_sparsify(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                                const double *minmax, float *rho, ad_orient orient,
                                const int32_t *budget, uint8_t *keep, int64_t *n_kept, void *ws,
                                size_t ws_bytes, hipStream_t stream);
ad_status ad_edge_dist_fit_both(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                                const double *minmax, float *rho, double target,
                                uint8_t *keep_local, uint8_t *keep_global, int64_t *n_kept,
                                double *e_used_host, void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for ad_normalize_dist. */
size_t ad_normalize_dist_workspace_size(const ad_graph *g);

/* Algorithm 1's optional normalization (its last step; Appendix A): delta_e
 * divided by sqrt(f_i f_j), with f the degree d_i as Algorithm 1 writes it
 * (by_strength = 0) or the weighted degree s_i = sum_j w_ij as the text
 * beside it says (by_strength = 1; with unit weights the two agree).
 * Written as a distance, so that the selection calls apply unchanged:
 *     rho_out[e] = sqrt(rho[e]^2 + eps) * sqrt(f_i * f_j),
 * and the normalized delta is 1 / rho_out[e] (eps >= 0, the epsilon of
 * Algorithm 1's return step).  rho, rho_out: [m] in rho_dtype (AD_F32 or
 * AD_F64; arithmetic in FP64); rho_out may equal rho.  Asynchronous. */
ad_status ad_normalize_dist(const ad_graph *g, ad_dtype rho_dtype, const void *rho,
                            int32_t by_strength, double eps, void *rho_out, void *ws,
                            size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for ad_sparsify_binned. */
size_t ad_sparsify_binned_workspace_size(const ad_graph *g);

/* Algorithm 4 (SparsifyB): selection with binning (bin rule of Section 4).
 * Every vertex i spreads the distances of its d_i edges over bins of width
 *     h = 3.5 sigma / cbrt(d_i)   (Scott's rule),
 * sigma the population standard deviation of those distances (computed in
 * double, rounded to single precision), B_i = max(1, ceil((max - min) / h))
 * bins (one when h == 0), entry q in bin min(B_i - 1, floor((rho_q - min) /
 * h)); cbrt is the C library's.  It then takes budget(d_i, e) of its edges
 * (budget as ad_budget_table) in rounds: in round r every non-empty bin, in
 * increasing order of its smallest priority, gives up its edge of (r+1)-th
 * smallest priority, so all bins give one edge before any gives two.  The
 * priority of neighbour j is fmix32(orig_id[j] ^ K_i) (fmix32: the 32-bit
 * finalizer of MurmurHash3), K_i the low 32 bits of word 0 of
 * Philox4x64-10 with key (seed, graph_id) and counter (orig_id[i], 0, 1, 0).
 * keep[e] = 1 when either endpoint takes edge e.
 *   rho: [m] distances (AD_F32 or AD_F64), e.g. from ad_edge_dist or
 *        ad_normalize_dist.
 *   target == 0: fixed exponent e in [0, 1]; target in (0, 1]: e is fitted
 *        as in ad_sparsify_fit (the taken sets grow with e) and returned
 *        through e_used_host, which is then required.
 *   n_kept: device int64, receives sum(keep).  e_used_host may be NULL for a
 *        fixed e (else it receives e).
 * The graph needs d_max set.  SYNCHRONISES `stream` (host tables by degree
 * are uploaded, and a fit reads counts back); not for stream capture.
 * Errors: AD_ERR_INVALID_ARG for bad arguments, AD_ERR_WORKSPACE when ws is
 * smaller than ad_sparsify_binned_workspace_size or not 256-byte aligned. */
ad_status ad_sparsify_binned(const ad_graph *g, ad_dtype rho_dtype, const void *rho,
                             uint64_t seed, uint64_t graph_id, double e, double target,
                             uint8_t *keep, int64_t *n_kept, double *e_used_host, void *ws,
                             size_t ws_bytes, hipStream_t stream);

/* --------------------------------------------------------------- ingest --- */

/* Workspace bytes for ad_ingest (0 when n or m_in is negative or >= 2^31). */
size_t ad_ingest_workspace_size(int64_t n, int64_t m_in);

/* An undirected edge list into the symmetric CSR of the graph model every
 * other call reads (Section 2: undirected, no self-loops, no repeated
 * pairs).  (u[q], v[q]) and (v[q], u[q]) name the same edge; self-loops are
 * dropped; repeated pairs become one edge whose weight is the exact sum of
 * the listed weights, rounded once to single precision (to nearest, ties to
 * even), so it does not depend on the list order.  Listed weights must be
 * finite and positive.  Edge ids enumerate the edges in (smaller, larger endpoint)
 * order (the CSR order of their upper entries); every row lists its
 * neighbours in ascending order.
 *   n, m_in: vertices and listed pairs, both < 2^31; u, v: DEVICE [m_in].
 *   w: DEVICE [m_in] or NULL (unweighted: w_out unused, may be NULL).
 *   orig_id: DEVICE [n] names of the listed vertices or NULL (identity).
 *   order: 0 keeps the listed ids; 1 stores vertices by decreasing degree,
 *          ties by listed id (the layout the sweeps prefer); 2 stores them
 *          in reverse Cuthill-McKee order (the bandwidth-reducing layout):
 *          components by increasing smallest listed id, each searched
 *          breadth first from its vertex of least (degree, listed id), the
 *          unqueued neighbours of each dequeued vertex queued by increasing
 *          (degree, listed id), the whole order reversed (one host
 *          read-back per level of the search).
 *   Outputs (DEVICE, caller-owned): row_ptr [n+1]; col, eid and w_out
 *   [2*m_in] (the first 2*m entries written); orig_id_out [n], the name of
 *   every stored vertex (orig_id of its listed vertex, or the listed id).
 *   m_host, d_max_host, n_dropped_host: HOST; the edge count m, the largest
 *   degree and m_in - m (self-loops plus merged repeats); d_max_host and
 *   n_dropped_host may be NULL.
 * The sorts are rocPRIM's radix sort (stable).  SYNCHRONISES `stream` (the
 * edge count sizes the later passes).  Errors: AD_ERR_GRAPH when a weight is
 * not finite and positive or when an endpoint
 * lies outside [0, n) (nothing is written past the check);
 * AD_ERR_INVALID_ARG / AD_ERR_UNSUPPORTED for bad arguments or sizes;
 * AD_ERR_WORKSPACE for a short or misaligned workspace. */
ad_status ad_ingest(int64_t n, int64_t m_in, const int32_t *u, const int32_t *v, const float *w,
                    const int32_t *orig_id, int32_t order, int64_t *row_ptr, int32_t *col,
                    float *w_out, int32_t *eid, int32_t *orig_id_out, int64_t *m_host,
                    int32_t *d_max_host, int64_t *n_dropped_host, void *ws, size_t ws_bytes,
                    hipStream_t stream);

/* ----------------------------------------------------------- properties -- */

/* Workspace bytes for ad_subgraph. */
size_t ad_subgraph_workspace_size(const ad_graph *g);

/* The sparsified graph G_s = (V, {e : keep[e]}) as a CSR of the same vertex
 * set: every row's kept entries in their order; sub_eid renumbers the kept
 * edges in increasing original id (so it is a valid ad_graph eid);
 * orig_edge[p] (DEVICE, optional) is the original id of entry p.  keep:
 * DEVICE [m] (0 / non-zero).  Outputs DEVICE, caller-owned: sub_row_ptr
 * [n+1]; sub_col, sub_eid, sub_w (only when g->w), orig_edge: [2m] (the
 * first 2 * m_sub written).  m_sub_host: HOST, the kept edge count.
 * SYNCHRONISES `stream`. */
ad_status ad_subgraph(const ad_graph *g, const uint8_t *keep, int64_t *sub_row_ptr, int32_t *sub_col,
                      float *sub_w, int32_t *sub_eid, int32_t *orig_edge, int64_t *m_sub_host, void *ws,
                      size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for ad_graph_properties. */
size_t ad_graph_properties_workspace_size(const ad_graph *g);

/* The single-graph properties of the Preliminaries, for comparing G_s with G:
 *   lambda[i] (DEVICE int64 [n], optional): triangles vertex i belongs to;
 *   c[i] (DEVICE double [n], optional): lambda_i / (d_i (d_i - 1) / 2),
 *        0 where d_i <= 1;
 *   comp[i] (DEVICE int32 [n], optional): the smallest vertex id of i's
 *        connected component;
 *   summary_host[0] = C_G, the mean of c_i over {i : d_i > 1} (Eq. cc; 0 if
 *        that set is empty), summary_host[1] = the number of components.
 * Counts are exact; C_G is summed in a fixed order.  Needs g->col ascending
 * within rows.  SYNCHRONISES `stream` (the component rounds read a flag). */
ad_status ad_graph_properties(const ad_graph *g, int64_t *lambda, double *c, int32_t *comp,
                              double *summary_host, void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for ad_spearman (0 when n < 0 or n >= 2^31). */
size_t ad_spearman_workspace_size(int64_t n);

/* Spearman rank correlation of two per-vertex scores by the Preliminaries'
 * formula rho = 1 - 6 sum_i p_i^2 / (n (n^2 - 1)), p_i the difference of the
 * ranks of x[i] and y[i]; tied scores share the mean of their ranks.  x, y:
 * DEVICE double [n], no NaN.  rho_host: HOST (0 when n < 2).  SYNCHRONISES
 * `stream`. */
ad_status ad_spearman(int64_t n, const double *x, const double *y, double *rho_host, void *ws,
                      size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for ad_compare_properties (0 when n or m >= 2^31). */
size_t ad_compare_properties_workspace_size(const ad_graph *g);

/* The comparisons of G_s = (V, {e : keep[e]}) with G that Section 6 makes
 * and that need no external package, all on the device: out_host
 * [AD_CMP_FIELDS] doubles, HOST:
 *   [0] edges kept (m of G_s);
 *   [1] C_G of G, [2] C_G of G_s (Eq. cc, as ad_graph_properties);
 *   [3] components of G, [4] components of G_s, [5] their ratio [4] / [3];
 *   [6] Spearman's rho of the degree sequences of G and G_s,
 *   [7] Spearman's rho of the clustering coefficients c_i of G and G_s
 *       (the Preliminaries' formula, tied scores at their mean rank).
 * The properties read the structure only (weights play no part).  keep:
 * DEVICE [m].  SYNCHRONISES `stream`.  Errors as ad_subgraph,
 * ad_graph_properties and ad_spearman. */
#define AD_CMP_FIELDS 8
ad_status ad_compare_properties(const ad_graph *g, const uint8_t *keep, double *out_host, void *ws,
                                size_t ws_bytes, hipStream_t stream);

/* ----------------------------------------------------------- multilevel -- */

/* Workspace bytes for ad_ml_aggregate (0 when n or m is negative or at least
 * 2^31). */
size_t ad_ml_aggregate_workspace_size(const ad_graph *g);

/* One coarsening step of Algorithm 6 (Section 5): the seeds and the
 * restriction P of Eq. P from the distances rho.  With the strength
 *     delta_e = 1 / sqrt(rho_e^2 + eps)
 * and smax_i the largest strength at i, i and j are strongly coupled when
 * delta_ij >= theta smax_i or delta_ij >= theta smax_j.  Seeds are chosen
 * as by visiting the vertices in decreasing degree (ties: smaller
 * fmix32(orig_id), then smaller orig_id) and taking each one that has no
 * strongly coupled seed yet.  Every seed is its own aggregate, numbered in
 * increasing vertex id; every other vertex joins its seed neighbour of
 * largest strength (ties: smaller orig_id), -1 if it has none.
 *   rho: DEVICE [m] (AD_F32 or AD_F64, strengths in double).
 *   agg: DEVICE int32 [n], the aggregate (coarse vertex) of every vertex.
 *   is_seed: DEVICE uint8 [n] or NULL.  n_coarse_host: HOST, the number of
 *   seeds (coarse vertices).
 * SYNCHRONISES `stream` (the seed rounds read a count back).  Errors:
 * AD_ERR_INVALID_ARG, AD_ERR_WORKSPACE, AD_ERR_UNSUPPORTED (n >= 2^31). */
ad_status ad_ml_aggregate(const ad_graph *g, ad_dtype rho_dtype, const void *rho, double eps,
                          double theta, int32_t *agg, uint8_t *is_seed, int64_t *n_coarse_host,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* Parameters of ad_ml_sparsify. */
typedef struct {
    int32_t R, k;             /* relaxation at every level (as ad_relax_opts)        */
    double omega;
    uint64_t seed;            /* Philox key word 0 of the test vectors and bin keys   */
    uint64_t graph_id;        /* level l uses graph_id + l                            */
    ad_dtype store;           /* AD_F64 or AD_F32: relaxation and distances           */
    int32_t levels;           /* at most this many levels, 1..64 (1 = SparsifyB only) */
    int64_t n_min;            /* a graph with n <= n_min is not coarsened            */
    const double *e_host;     /* HOST [levels]: the per-level ratio vector, COARSEST
                                 level first (entry t for the level t steps finer than
                                 the coarsest one reached); every entry <= 1; a
                                 negative entry: no SparsifyB at that level          */
    double eps, theta;        /* strength and coupling of ad_ml_aggregate            */
    uint64_t bin_seed;        /* Philox key word 0 of SparsifyB's vertex keys         */
    int32_t fit;              /* 0: entries are SparsifyB exponents e in [0, 1];
                                 1: entries are the fractions of each level's edges
                                 SparsifyB keeps (e fitted as in ad_sparsify_binned) */
    int32_t span;             /* > 0: e_host is ignored and the vector is
                                 ad_ml_level_span(levels reached, span, segment,
                                 span_value)                                       */
    int32_t segment;          /* 0 coarsest, 1 middle, 2 finest third of the levels  */
    double span_value;        /* the entry the level-span rule gives, <= 1           */
    int32_t fp64_tail;        /* AD_F32: final sweeps stored in FP64 (ad_relax_opts)  */
} ad_ml_opts;

/* Host helper: the level-span ratio vector of Section 6 (implementation
 * paragraph) over n_levels levels (1..64), coarsest first: the levels split
 * into thirds, third s holding entries floor(s n / 3) .. floor((s+1) n / 3) - 1;
 * the first `span` entries of third `segment` (0 coarsest, 1 middle, 2
 * finest) are `value`, all others -1.  out_host: HOST [n_levels]. */
ad_status ad_ml_level_span(int32_t n_levels, int32_t span, int32_t segment, double value,
                           double *out_host);

/* Algorithm 6 (MLSparsify).  Level 0 is g.  At level l: distances by
 * ad_relax + ad_edge_dist (graph id graph_id + l, the level's connected
 * components from ad_components_build, fp64_tail for FP32); if n <= n_min, or
 * l == levels - 1, or the graph has no edges, or ad_ml_aggregate would keep
 * more than 90% of the vertices, level l is the coarsest (D = l): SparsifyB
 * (ad_sparsify_binned, graph id graph_id + D) selects with the vector's
 * entry 0 and the recursion ends.
 * Otherwise the coarse graph P^T L P (aggregate pairs of the fine edges,
 * merged by ad_ingest with summed weights; a unit weight per edge when g is
 * unweighted; coarse vertices named by their seeds' orig_id) is sparsified
 * at level l + 1; every fine edge joining two aggregates inherits its coarse
 * edge's state, every edge inside an aggregate is kept; distances are then
 * recomputed on the fine graph less the dropped edges (ad_subgraph) and
 * SparsifyB, with the vector's entry D - l, selects among its edges:
 * keep[e] = 1 for those.  A negative entry leaves the inherited state (at the
 * coarsest level: every edge) as the level's result.
 *   keep: DEVICE uint8 [m].  n_kept_host: HOST, sum(keep).  depth_host:
 *   HOST or NULL, the index of the coarsest level reached.
 * The call allocates the per-level graphs and buffers itself (their sizes
 * follow from the coarsening) with hipMalloc and frees them before it
 * returns; it SYNCHRONISES `stream` and is not for stream capture.  Errors:
 * AD_ERR_INVALID_ARG for bad options, AD_ERR_UNSUPPORTED for m >= 2^30,
 * AD_ERR_HIP when an allocation fails. */
ad_status ad_ml_sparsify(const ad_graph *g, const ad_ml_opts *o, uint8_t *keep,
                         int64_t *n_kept_host, int32_t *depth_host, hipStream_t stream);

/* ------------------------------------------------------------- adjoint --- */

/* Workspace bytes for ad_relax_backward. */
size_t ad_relax_backward_workspace_size(const ad_graph *g, const ad_relax_opts *o);

/* Reverse-mode derivative of a loss L(rho) with respect to the edge weights,
 * through ad_edge_dist, the rescale and the k sweeps of ad_relax (start
 * vectors do not depend on w).  Requires store == AD_F32, fp64_tail == 0
 * and ckpt_every > 0.
 *   ckpt     : checkpoints written by ad_relax with the same graph and opts.
 *   x_k      : x_out of that ad_relax call; minmax, shift: its minmax_out
 *              and shift_out (per component when o->comp is given).
 *   grad_rho : [m] FP32, dL/drho_e.
 *   grad_w   : [m] FP32 output, dL/dw_e with w_ij = w_ji = w_e.
 * The min and max of the rescale are differentiated at the first vertex
 * attaining them; edges with rho_e == 0 pass no gradient. */
ad_status ad_relax_backward(const ad_graph *g, const ad_relax_opts *o, const void *ckpt,
                            const void *x_k, const double *minmax, const double *shift,
                            const float *grad_rho, float *grad_w, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* Edge weights to CSR order: w_entries[p] = w_edge[eid[p]] for p < 2m (the
 * layout ad_relax reads; used when the weights are the variables of the
 * adjoint).  w_edge: [m] FP32, w_entries: [2m] FP32. */
ad_status ad_edge_to_entries(const ad_graph *g, const float *w_edge, float *w_entries,
                             hipStream_t stream);

/* Per-entry neighbour ids for ad_graph.col_orig: col_orig[p] = orig_id[col[p]]
 * (= col[p] when orig_id is NULL), p < 2m.  Build once per graph. */
ad_status ad_graph_col_orig(const ad_graph *g, int32_t *col_orig, hipStream_t stream);

/* --------------------------------------------------------------- batch --- */

/* Batched form: G independent graphs, each run through ad_relax (FP32
 * storage, optionally with an FP64 tail), ad_edge_dist (FP32 rho) and
 * ad_sparsify at one fixed e, as one captured sequence of kernel launches
 * covering all graphs (a HIP graph replayed by ad_batch_run).  Graph q is
 * relaxed with key word o->graph_id + q and centred per connected component
 * (the batch builds the components of its packed graph at creation;
 * o->comp is ignored); its distances, kept edges and count equal, bit for
 * bit, those of the three calls on graph q alone with the same options
 * (including rows_per_wave) and its own ad_components_build.
 * The batch owns a packed copy of the graphs, its workspaces and its
 * outputs (device memory allocated by ad_batch_create, freed by
 * ad_batch_destroy -- the one exception to "no call allocates").
 * ad_batch_create synchronises `stream`; it may first time the candidate
 * rows_per_wave values on the batch (autotune) and keep the fastest. */
typedef struct ad_batch ad_batch;
typedef struct {
    ad_orient orient;         /* Algorithm 3 orientation for every graph          */
    double e;                 /* fixed exponent in [0, 1]                          */
    int32_t autotune;         /* 1: choose rows_per_wave by timing on the batch    */
} ad_batch_opts;

/* graphs: host array of G graph descriptions (device pointers, host n, m,
 * d_max); o: relaxation options (store must be AD_F32, no checkpoints;
 * fp64_tail allowed). */
ad_status ad_batch_create(int32_t G, const ad_graph *graphs, const ad_relax_opts *o,
                          const ad_batch_opts *bo, ad_batch **out, hipStream_t stream);
/* Replays the captured sequence on `stream`. */
ad_status ad_batch_run(ad_batch *b, hipStream_t stream);
/* The same sequence enqueued kernel by kernel (no graph replay). */
ad_status ad_batch_run_uncaptured(ad_batch *b, hipStream_t stream);
/* Host copies of the packing: row_off_host [G+1], edge_off_host [G+1] (edge
 * ids of graph q are [edge_off[q], edge_off[q+1]) in the packed outputs),
 * and the rows_per_wave in use.  Any pointer may be NULL. */
ad_status ad_batch_info(const ad_batch *b, int64_t *row_off_host, int64_t *edge_off_host,
                        int32_t *rows_per_wave_host);
/* Device pointers to the outputs of the last run: rho [sum m] FP32, keep
 * [sum m], n_kept [G] int64, minmax [G][2R] doubles.  Valid until the next
 * run or destroy. */
ad_status ad_batch_results(const ad_batch *b, const float **rho, const uint8_t **keep,
                           const int64_t **n_kept, const double **minmax);
/* The same outputs copied (device to device, on `stream`) into caller
 * buffers of the sizes above; any pointer may be NULL. */
ad_status ad_batch_copy_results(const ad_batch *b, float *rho, uint8_t *keep, int64_t *n_kept,
                                double *minmax, hipStream_t stream);
void ad_batch_destroy(ad_batch *b);

/* ---------------------------------------------------------- diagnostics -- */

/* Checks on the device that the CSR is a valid symmetric simple graph:
 * sorted columns in range, no self-loops or repeats, every (i,j) has its
 * mirror (j,i) with the same eid and weight, eids in [0, m) used exactly
 * twice, weights finite and > 0.  SYNCHRONISES `stream`.  Returns AD_OK or
 * AD_ERR_GRAPH (message in ad_last_error()).  ws: ad_validate_workspace_size. */
size_t ad_validate_workspace_size(const ad_graph *g);
ad_status ad_validate_graph(const ad_graph *g, void *ws, size_t ws_bytes, hipStream_t stream);

/* Kernel timing (for measurement, off by default).  While enabled, the
 * library brackets its main kernel launches (JOR sweeps, distance, ranking,
 * fit passes, ...) with HIP events on the caller's stream; the k sweeps of
 * one ad_relax call share one pair of events around the whole sequence (so
 * the per-launch figure is the span over k, gaps between sweeps included).
 * Events come from a pool that grows on first use.  ad_trace_summary waits for
 * the recorded events and writes one line per kernel name,
 * "<name> <launches> <total_ms>\n", into buf (len bytes, NUL-terminated);
 * ad_trace_reset waits for them and keeps their events for reuse by later
 * scopes (so a traced region after a first traced pass creates none). */
void ad_trace_enable(int32_t on);
void ad_trace_reset(void);
ad_status ad_trace_summary(char *buf, size_t len);

const char *ad_status_string(ad_status s);
const char *ad_last_error(void);
int32_t ad_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AD_H */
