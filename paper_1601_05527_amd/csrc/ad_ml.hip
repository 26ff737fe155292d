// Multilevel sparsification (Algorithm 6, MLSparsify; coarsening of
// Section 5), driving the library's own calls level by level.
//
// Readings (shared with the oracle, which is written separately):
//   - strength delta_ij = 1 / sqrt(rho_ij^2 + eps) from the level's
//     distances (Algorithm 1's return value);
//   - i and j are strongly coupled when delta_ij >= theta * smax_i or
//     delta_ij >= theta * smax_j, smax_i the largest strength at i;
//   - seeds: the vertices in decreasing degree, ties by fmix32(name) and
//     then the name (orig_id), each becoming a seed unless a strong
//     neighbour already is one.  On the device this sequential traversal is
//     run as rounds: an undecided vertex with a seed among its strong
//     neighbours is not a seed; one whose strong neighbours of higher
//     priority are all decided non-seeds becomes a seed; the others wait.
//     A strong seed neighbour of an undecided vertex always has the higher
//     priority, so the rounds choose exactly the sequential seeds;
//   - restriction P (Eq. P): a seed is its own aggregate (numbered in id
//     order); any other vertex joins the seed neighbour of largest delta_ij,
//     ties by smaller name;
//   - Galerkin coarse graph P^T L P: the fine edges' aggregate pairs with
//     repeats merged, their weights summed exactly (ad_ingest; unit weights
//     count edges), coarse vertices named by their seeds;
//   - a level is the coarsest at n <= n_min, at level levels - 1, with no
//     edges, or when coarsening would keep more than 90% of the vertices;
//   - level l uses graph id graph_id + l (test vectors and bin order);
//   - the per-level ratio vector (Section 6, implementation paragraph) lists
//     the levels from the coarsest one reached: with D the index of the
//     coarsest level, level l takes entry D - l.  A negative entry means no
//     SparsifyB at that level (it keeps what it inherits; the coarsest level
//     keeps all its edges); otherwise the entry is SparsifyB's exponent, or
//     with `fit` the fraction of the level's edges to keep (e fitted as in
//     ad_sparsify_binned);
//   - level-span: the D + 1 levels split into thirds (coarsest, middle,
//     finest), third s holding entries floor(s (D+1) / 3) .. floor((s+1)
//     (D+1) / 3) - 1; the first `span` entries of the chosen third take the
//     value, all others -1;
//   - uncoarsening: an edge between two aggregates keeps its coarse edge's
//     state, an edge inside an aggregate is kept; distances are recomputed
//     on the fine graph less the dropped edges (ad_subgraph) and SparsifyB
//     chooses among its edges.
// The call allocates its per-level graphs and buffers (their sizes are
// known only as coarsening proceeds) and frees them before it returns.
#include "ad_internal.h"

#include <algorithm>
#include <cstdint>
#include <vector>

namespace ad {

constexpr int MBLOCK = 256;

static unsigned mgrid(int64_t count) { return grid_for(std::max<int64_t>(1, count), MBLOCK); }
static unsigned mwgrid(int64_t rows) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(rows, MBLOCK / WAVE)));
}

// ------------------------------------------------------------- kernels --

template <typename Tr>
__device__ __forceinline__ double ml_strength(Tr rho, double eps) {
#pragma clang fp contract(off)
    const double r = (double)rho;
    const double t = r * r + eps;
    return 1.0 / sqrt(t);
}

__device__ __forceinline__ uint32_t ml_hash(uint32_t h) {    // MurmurHash3's 32-bit finalizer
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Is vertex b ahead of vertex a in the seed traversal?
__device__ __forceinline__ bool ml_ahead(int64_t da, int32_t ka, int64_t db, int32_t kb) {
    if (db != da) return db > da;
    const uint32_t ha = ml_hash((uint32_t)ka), hb = ml_hash((uint32_t)kb);
    if (hb != ha) return hb < ha;
    return kb < ka;
}

// What a coupling test reads of a vertex, in one 16-byte record: theta
// times its largest strength, its degree and its name.
struct __align__(16) MlVert {
    double tsmax;
    uint32_t deg;
    int32_t key;
};

template <typename Tr>
__global__ __launch_bounds__(MBLOCK) void k_ml_smax(int64_t n, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ eid,
                                                     const int32_t *__restrict__ orig_id, const Tr *__restrict__ rho,
                                                     double eps, double theta, MlVert *__restrict__ vert) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (MBLOCK / WAVE);
    for (int64_t i = (int64_t)blockIdx.x * (MBLOCK / WAVE) + (threadIdx.x >> 6); i < n; i += nw) {
        const int64_t b0 = row_ptr[i], b1 = row_ptr[i + 1];
        double mx = 0.0;
        for (int64_t p = b0 + lane; p < b1; p += WAVE) mx = fmax(mx, ml_strength(rho[eid[p]], eps));
        for (int o = WAVE / 2; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, WAVE));
        if (lane == 0) vert[i] = MlVert{theta * mx, (uint32_t)(b1 - b0), orig_id ? orig_id[i] : (int32_t)i};
    }
}

// Coupling of every stored entry (i, j): 0 not strong, 1 strong with j
// after i in the traversal, 2 strong with j ahead of i; acnt[i] = the number
// of entries of row i coupled strongly to a vertex ahead.
template <typename Tr>
__global__ __launch_bounds__(MBLOCK) void k_ml_strong(int64_t n, const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, const int32_t *__restrict__ eid,
                                                      const Tr *__restrict__ rho, double eps,
                                                      const MlVert *__restrict__ vert,
                                                      uint8_t *__restrict__ sflag, uint32_t *__restrict__ acnt) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (MBLOCK / WAVE);
    for (int64_t i = (int64_t)blockIdx.x * (MBLOCK / WAVE) + (threadIdx.x >> 6); i < n; i += nw) {
        const int64_t b0 = row_ptr[i], b1 = row_ptr[i + 1];
        const MlVert vi = vert[i];
        int ahead = 0;
        for (int64_t p = b0 + lane; p < b1; p += WAVE) {
            const int32_t j = col[p];
            const double d = ml_strength(rho[eid[p]], eps);
            const MlVert vj = vert[j];
            uint8_t f = 0;
            if (d >= vi.tsmax || d >= vj.tsmax) f = ml_ahead(vi.deg, vi.key, vj.deg, vj.key) ? 2 : 1;
            sflag[p] = f;
            ahead += f == 2;
        }
        for (int o = WAVE / 2; o >= 1; o >>= 1) ahead += __shfl_xor(ahead, o, WAVE);
        if (lane == 0) acnt[i] = (uint32_t)ahead;
    }
}

// The strongly coupled neighbours ahead of each vertex, in row order:
// alist[aoff[i], aoff[i + 1]).
__global__ __launch_bounds__(MBLOCK) void k_ml_ahead_list(int64_t n, const int64_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col,
                                                          const uint8_t *__restrict__ sflag,
                                                          const uint32_t *__restrict__ aoff,
                                                          int32_t *__restrict__ alist) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (MBLOCK / WAVE);
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int64_t i = (int64_t)blockIdx.x * (MBLOCK / WAVE) + (threadIdx.x >> 6); i < n; i += nw) {
        const int64_t b0 = row_ptr[i], b1 = row_ptr[i + 1];
        uint32_t o = aoff[i];
        for (int64_t p0 = b0; p0 < b1; p0 += WAVE) {            // the bound is the same for the whole wave
            const int64_t p = p0 + lane;
            const bool f2 = p < b1 && sflag[p] == 2;
            const unsigned long long bal = __ballot(f2);
            if (f2) alist[o + (uint32_t)__popcll(bal & below)] = col[p];
            o += (uint32_t)__popcll(bal);
        }
    }
}

// One round of the seed traversal over the undecided vertices (state 0;
// 1 = seed, 2 = not a seed): a vertex with a strongly coupled seed is not a
// seed; one whose strongly coupled vertices ahead of it are all decided
// becomes a seed; the others wait, and *left is set to 1 if any does.  Only the
// strongly coupled vertices ahead of i matter while i is undecided (one
// behind i cannot be decided a seed before i is decided), so a round reads
// i's list of those; and since a decided state never changes, a waiting
// vertex keeps in resume[i] the place in its list of its first undecided
// neighbour (every one before it is final and not a seed) and the next round
// reads the list from there.  States are read and written with device
// scope, so a decision made during a round can already settle other
// vertices in the same round (with workgroup scope the rounds were more and
// no shorter).
constexpr uint32_t SEED_LANE_MAX = 32;   // lists up to this length: one lane per vertex, longer: one wave
constexpr int SEED_LOADS = 8;            // list entries a lane reads per step

__global__ __launch_bounds__(MBLOCK) void k_ml_seed_round(int64_t n, const uint32_t *__restrict__ aoff,
                                                          const int32_t *__restrict__ alist,
                                                          uint8_t *__restrict__ state,
                                                          uint32_t *__restrict__ resume,
                                                          unsigned long long *__restrict__ left) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (MBLOCK / WAVE);
    unsigned long long waiting = 0;
    // wave gw owns rows gw + k nw (the high-degree rows, stored first, spread
    // over the waves), 64 at a time: short lists by their own lane, then
    // long ones by the whole wave, one at a time
    const int64_t gw = (int64_t)blockIdx.x * (MBLOCK / WAVE) + (threadIdx.x >> 6);
    for (int64_t base = gw; base < n; base += nw * WAVE) {
        const int64_t mine = base + (int64_t)lane * nw;
        // the row's state (only this wave writes its rows' states), list
        // bounds and resume point, loaded together
        const bool in = mine < n;
        const uint8_t own = in ? state[mine] : (uint8_t)1;
        const uint32_t a = in ? aoff[mine] : 0u, len = in ? aoff[mine + 1] - a : 0u;
        const uint32_t from = in ? resume[mine] : 0u;
        const bool undecided = own == 0;
        if (undecided && len <= SEED_LANE_MAX) {
            bool seed_nb = false;
            uint32_t wait_at = len;
            for (uint32_t q0 = from; q0 < len && !seed_nb; q0 += SEED_LOADS) {
                int32_t v[SEED_LOADS];
                uint8_t sj[SEED_LOADS];
#pragma unroll
                for (int t = 0; t < SEED_LOADS; ++t) v[t] = q0 + t < len ? alist[a + q0 + t] : -1;
#pragma unroll
                for (int t = 0; t < SEED_LOADS; ++t)
                    sj[t] = v[t] >= 0
                                ? __hip_atomic_load(&state[v[t]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : (uint8_t)2;
#pragma unroll
                for (int t = 0; t < SEED_LOADS; ++t) {
                    if (sj[t] == 1) seed_nb = true;
                    else if (sj[t] == 0 && wait_at == len) wait_at = q0 + t;
                }
            }
            if (seed_nb) __hip_atomic_store(&state[mine], (uint8_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else if (wait_at == len)
                __hip_atomic_store(&state[mine], (uint8_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else {
                resume[mine] = wait_at;
                ++waiting;
            }
        }
        unsigned long long todo = __ballot(undecided && len > SEED_LANE_MAX);
        while (todo) {
            const int t = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int64_t i = base + (int64_t)t * nw;
            const uint32_t ai = aoff[i], li = aoff[i + 1] - ai;
            bool seed_nb = false;
            uint32_t wait_at = li;
            for (uint32_t q = resume[i] + (uint32_t)lane; q < li; q += WAVE) {
                const uint8_t sj =
                    __hip_atomic_load(&state[alist[ai + q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (sj == 1) seed_nb = true;
                else if (sj == 0) wait_at = min(wait_at, q);
            }
            const bool any_seed = __ballot(seed_nb) != 0ull;
            for (int o = WAVE / 2; o >= 1; o >>= 1)
                wait_at = min(wait_at, (uint32_t)__shfl_xor((int)wait_at, o, WAVE));
            if (lane == 0) {
                if (any_seed) __hip_atomic_store(&state[i], (uint8_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else if (wait_at == li)
                    __hip_atomic_store(&state[i], (uint8_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else {
                    resume[i] = wait_at;
                    ++waiting;
                }
            }
        }
    }
    // a flag, not a count: the host only asks whether any vertex waits, and
    // an atomic add from every wave on one address serialises at the memory
    // side (each writer stores the same value; the host reads it after the
    // round's kernel has completed)
    if (__ballot(waiting != 0) != 0ull && lane == 0) *left = 1ull;
}

__global__ void k_ml_seed_flags(int64_t n, const uint8_t *__restrict__ state, unsigned int *__restrict__ flag,
                                uint8_t *__restrict__ is_seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const bool s = state[i] == 1;
        flag[i] = s ? 1u : 0u;
        if (is_seed) is_seed[i] = s ? 1 : 0;
    }
}

__global__ void k_ml_degree_max(int64_t n, const int64_t *__restrict__ row_ptr, unsigned int *__restrict__ out) {
    unsigned int mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mx = max(mx, (unsigned int)(row_ptr[i + 1] - row_ptr[i]));
    for (int o = WAVE / 2; o >= 1; o >>= 1) mx = max(mx, (unsigned int)__shfl_xor((int)mx, o, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0 && mx) atomicMax(out, mx);
}

// Aggregates (Eq. P): a seed's own rank; otherwise the rank of the seed
// neighbour of largest strength, ties by smaller name (-1 if none).
template <typename Tr>
__global__ __launch_bounds__(MBLOCK) void k_ml_aggregate(int64_t n, const int64_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ eid,
                                                         const int32_t *__restrict__ orig_id,
                                                         const Tr *__restrict__ rho, double eps,
                                                         const uint8_t *__restrict__ state,
                                                         const uint32_t *__restrict__ rank, int32_t *__restrict__ agg) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (MBLOCK / WAVE);
    for (int64_t i = (int64_t)blockIdx.x * (MBLOCK / WAVE) + (threadIdx.x >> 6); i < n; i += nw) {
        if (state[i] == 1) {
            if (lane == 0) agg[i] = (int32_t)rank[i];
            continue;
        }
        double bd = -1.0;
        int32_t bk = 0x7fffffff, bj = -1;
        for (int64_t p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += WAVE) {
            const int32_t j = col[p];
            if (state[j] != 1) continue;
            const double d = ml_strength(rho[eid[p]], eps);
            const int32_t k = orig_id ? orig_id[j] : j;
            if (d > bd || (d == bd && k < bk)) {
                bd = d;
                bk = k;
                bj = j;
            }
        }
        for (int o = WAVE / 2; o >= 1; o >>= 1) {
            const double od = __shfl_xor(bd, o, WAVE);
            const int32_t ok = __shfl_xor(bk, o, WAVE), oj = __shfl_xor(bj, o, WAVE);
            if (od > bd || (od == bd && ok < bk)) {
                bd = od;
                bk = ok;
                bj = oj;
            }
        }
        if (lane == 0) agg[i] = bj >= 0 ? (int32_t)rank[bj] : -1;
    }
}

// The fine edges' aggregate pairs (edge id order) and weights (1 when unweighted).
__global__ __launch_bounds__(MBLOCK) void k_ml_pairs(int64_t n, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const float *__restrict__ w,
                                                     const int32_t *__restrict__ eid, const int32_t *__restrict__ agg,
                                                     int32_t *__restrict__ cu, int32_t *__restrict__ cv,
                                                     float *__restrict__ cw) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (MBLOCK / WAVE);
    for (int64_t i = (int64_t)blockIdx.x * (MBLOCK / WAVE) + (threadIdx.x >> 6); i < n; i += nw) {
        const int32_t ai = agg[i];
        for (int64_t p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += WAVE) {
            const int32_t j = col[p];
            if (j <= i) continue;
            const int32_t e = eid[p];
            cu[e] = ai;
            cv[e] = agg[j];
            cw[e] = w ? w[p] : 1.0f;
        }
    }
}

__global__ void k_ml_names(int64_t n, const uint8_t *__restrict__ state, const int32_t *__restrict__ agg,
                           const int32_t *__restrict__ orig_id, int32_t *__restrict__ names) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (state[i] == 1) names[agg[i]] = orig_id ? orig_id[i] : (int32_t)i;
}

// Inherited state of every fine edge from the coarse keep.
__global__ void k_ml_inherit(int64_t m, const int32_t *__restrict__ cu, const int32_t *__restrict__ cv,
                             const int64_t *__restrict__ crp, const int32_t *__restrict__ ccol,
                             const int32_t *__restrict__ ceid, const uint8_t *__restrict__ ckeep,
                             uint8_t *__restrict__ inh) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = cu[e], b = cv[e];
        if (a == b) {
            inh[e] = 1;
            continue;
        }
        const int32_t x = a < b ? a : b, y = a < b ? b : a;
        int64_t lo = crp[x], hi = crp[x + 1];
        const int64_t end = hi;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ccol[mid] < y) lo = mid + 1;
            else hi = mid;
        }
        inh[e] = (lo < end && ccol[lo] == y) ? (ckeep[ceid[lo]] ? 1 : 0) : 0;
    }
}

// keep[original edge] from the subgraph's keep (both entries write the same value).
__global__ void k_ml_map_back(int64_t nnz_sub, const int32_t *__restrict__ sub_eid,
                              const int32_t *__restrict__ orig_edge, const uint8_t *__restrict__ sub_keep,
                              uint8_t *__restrict__ keep) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz_sub; p += (int64_t)gridDim.x * blockDim.x)
        if (sub_keep[sub_eid[p]]) keep[orig_edge[p]] = 1;
}

__global__ void k_ml_count(int64_t m, const uint8_t *__restrict__ keep, unsigned long long *__restrict__ cnt) {
    unsigned long long k = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        k += keep[e] ? 1 : 0;
    for (int o = WAVE / 2; o >= 1; o >>= 1) k += __shfl_xor(k, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0 && k) atomicAdd(cnt, k);
}

// ---------------------------------------------------------- coarsening --

constexpr int SEED_BATCH = 4;            // seed rounds per read-back

struct AggLayout {
    MlVert *vert;                 // [n] theta * largest strength, degree and name of every vertex
    uint8_t *state;               // [n]
    uint32_t *resume;             // [n] where a waiting vertex's next seed round reads its row from
    uint8_t *sflag;               // [nnz] coupling of every entry
    uint32_t *aoff;               // [n + 1] offsets of the lists of strongly coupled neighbours ahead
    int32_t *alist;               // [nnz / 2] those lists (a strong edge is ahead from one end only)
    unsigned int *rank;           // [n] seed flags, scanned in place into aggregate ids
    unsigned int *total;          // [1] number of seeds
    unsigned long long *left;     // [SEED_BATCH] 1 when a vertex is still undecided after a round of a batch
    ScanScratch scan;
};

static size_t agg_layout(int64_t n, int64_t nnz, void *ws, size_t ws_bytes, AggLayout *L) {
    Carver c(ws, ws_bytes);
    const size_t nn = (size_t)std::max<int64_t>(1, n);
    AggLayout l;
    l.vert = c.take<MlVert>(nn);
    l.state = c.take<uint8_t>(nn);
    l.resume = c.take<uint32_t>(nn);
    l.sflag = c.take<uint8_t>((size_t)std::max<int64_t>(1, nnz));
    l.aoff = c.take<uint32_t>(nn + 1);
    l.alist = c.take<int32_t>((size_t)std::max<int64_t>(1, nnz / 2));
    l.rank = c.take<unsigned int>(nn);
    l.total = c.take<unsigned int>(1);
    l.left = c.take<unsigned long long>(SEED_BATCH);
    const size_t nblk = scan_scratch_blocks((int64_t)nn);
    l.scan.blk_v = c.take<unsigned int>(nblk);
    l.scan.blk_w = c.take<unsigned long long>(nblk);
    l.scan.total_w = c.take<unsigned long long>(1);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

static ad_status ml_check_ws(void *ws, size_t need, size_t ws_bytes) {
    if (!ws) return fail(AD_ERR_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (need == 0 || ws_bytes < need) return fail(AD_ERR_WORKSPACE, "workspace too small");
    return AD_OK;
}

// Seeds and aggregates of one coarsening step; *nc_host = number of seeds.
// Synchronises the stream (the rounds read a count back).
template <typename Tr>
static ad_status aggregate_impl(const ad_graph *g, const Tr *rho, double eps, double theta, int32_t *agg,
                                uint8_t *is_seed, int64_t *nc_host, const AggLayout &L, hipStream_t st) {
    const int64_t n = g->n;
    *nc_host = 0;
    if (n == 0) return AD_OK;
    hipLaunchKernelGGL(k_ml_smax<Tr>, dim3(mwgrid(n)), dim3(MBLOCK), 0, st, n, g->row_ptr, g->eid, g->orig_id, rho,
                       eps, theta, L.vert);
    AD_LAUNCH_CHECK("k_ml_smax");
    hipLaunchKernelGGL(k_ml_strong<Tr>, dim3(mwgrid(n)), dim3(MBLOCK), 0, st, n, g->row_ptr, g->col, g->eid,
                       rho, eps, L.vert, L.sflag, L.aoff);
    AD_LAUNCH_CHECK("k_ml_strong");
    ad_status s = scan_exclusive(n, L.aoff, nullptr, L.aoff + n, nullptr, L.scan, st);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_ml_ahead_list, dim3(mwgrid(n)), dim3(MBLOCK), 0, st, n, g->row_ptr, g->col, L.sflag,
                       L.aoff, L.alist);
    AD_LAUNCH_CHECK("k_ml_ahead_list");
    s = fill_u8(L.state, 0, n, st);
    if (s != AD_OK) return s;
    s = fill_i32((int32_t *)L.resume, 0, n, st);
    if (s != AD_OK) return s;
    // each round decides at least the undecided vertex of highest priority
    // rounds are enqueued SEED_BATCH at a time and only the last one's count
    // is read back (a round after the last undecided vertex changes nothing)
    for (int64_t round = 0;; round += SEED_BATCH) {
        if (round > n) return fail(AD_ERR_INTERNAL, "seed rounds did not settle");
        s = fill_u64(L.left, 0, SEED_BATCH, st);
        if (s != AD_OK) return s;
        for (int b = 0; b < SEED_BATCH; ++b) {
            hipLaunchKernelGGL(k_ml_seed_round, dim3(mwgrid(n)), dim3(MBLOCK), 0, st, n, L.aoff, L.alist, L.state,
                               L.resume, L.left + b);
            AD_LAUNCH_CHECK("k_ml_seed_round");
        }
        unsigned long long waiting = 0;
        AD_HIP(hipMemcpyAsync(&waiting, L.left + (SEED_BATCH - 1), sizeof(waiting), hipMemcpyDeviceToHost, st));
        AD_HIP(hipStreamSynchronize(st));
        if (waiting == 0) break;
    }
    hipLaunchKernelGGL(k_ml_seed_flags, dim3(mgrid(n)), dim3(MBLOCK), 0, st, n, L.state, L.rank, is_seed);
    AD_LAUNCH_CHECK("k_ml_seed_flags");
    s = scan_exclusive(n, L.rank, nullptr, L.total, nullptr, L.scan, st);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_ml_aggregate<Tr>, dim3(mwgrid(n)), dim3(MBLOCK), 0, st, n, g->row_ptr, g->col, g->eid,
                       g->orig_id, rho, eps, L.state, L.rank, agg);
    AD_LAUNCH_CHECK("k_ml_aggregate");
    unsigned int nc = 0;
    AD_HIP(hipMemcpyAsync(&nc, L.total, sizeof(nc), hipMemcpyDeviceToHost, st));
    AD_HIP(hipStreamSynchronize(st));
    *nc_host = nc;
    return AD_OK;
}

// --------------------------------------------------------------- driver --

// Device memory of the call: a stack arena.  Buffers are carved from large
// chunks (hipMalloc'd as needed, the first sized for level 0); freeing a
// buffer releases it at once when it is the newest live one, otherwise when
// the buffers above it are gone (the levels' buffers are nested scopes, so
// almost every release is immediate).  Carving is host arithmetic, so the
// levels allocate without device calls; every chunk is freed when the call
// ends.  Without an arena (outside a call) plain hipMalloc / hipFree.
struct MlArena {
    struct Chunk {
        char *base;
        size_t cap, top;
    };
    struct Block {
        size_t chunk, off;
        bool live;
    };
    std::vector<Chunk> chunks;
    std::vector<Block> blocks;     // in allocation order

    ad_status take(size_t bytes, void **out) {
        bytes = (bytes + 255) & ~size_t(255);
        // the first chunk with room above its top (each chunk's blocks are
        // still released in reverse order, so its top stays a stack)
        size_t c = 0;
        while (c < chunks.size() && chunks[c].top + bytes > chunks[c].cap) ++c;
        if (c == chunks.size()) {
            const size_t want = std::max(bytes, chunks.empty() ? (size_t)(64u << 20) : 2 * chunks.back().cap);
            void *p = nullptr;
            const hipError_t e = hipMalloc(&p, want);
            if (e != hipSuccess) return fail(AD_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
            chunks.push_back(Chunk{(char *)p, want, 0});
            c = chunks.size() - 1;
        }
        blocks.push_back(Block{c, chunks[c].top, true});
        *out = chunks[c].base + chunks[c].top;
        chunks[c].top += bytes;
        return AD_OK;
    }
    void give(void *p) {
        for (size_t k = blocks.size(); k-- > 0;) {
            const Block &b = blocks[k];
            if (b.live && chunks[b.chunk].base + b.off == (char *)p) {
                blocks[k].live = false;
                break;
            }
        }
        while (!blocks.empty() && !blocks.back().live) {
            chunks[blocks.back().chunk].top = blocks.back().off;
            blocks.pop_back();
        }
    }
    void release() {
        for (const Chunk &c : chunks) (void)hipFree(c.base);
        chunks.clear();
        blocks.clear();
    }
};
static thread_local MlArena *ml_arena = nullptr;

struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { reset(); }
    void reset() {
        if (p) {
            if (ml_arena) ml_arena->give(p);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *get() const { return (T *)p; }
};

static ad_status dev_alloc(DevMem &d, size_t bytes) {
    d.reset();
    const size_t b = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
    if (ml_arena) {
        ad_status s = ml_arena->take(b, &d.p);
        if (s != AD_OK) {
            d.p = nullptr;
            return s;
        }
    } else {
        const hipError_t e = hipMalloc(&d.p, b);
        if (e != hipSuccess) {
            d.p = nullptr;
            return fail(AD_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    d.bytes = b;
    return AD_OK;
}

// The call's arena, its first chunk sized for level 0 of a graph with n
// vertices and m edges; the destructor waits for the stream (work in flight
// may still use the chunks) and frees them.
struct MlArenaScope {
    hipStream_t stream;
    MlArena arena;
    MlArenaScope(hipStream_t st, int64_t n, int64_t m) : stream(st) {
        void *p = nullptr;
        const size_t first = (size_t)(104 * std::max<int64_t>(1, m) + 104 * std::max<int64_t>(1, n)) + (64u << 20);
        if (hipMalloc(&p, first) == hipSuccess) arena.chunks.push_back(MlArena::Chunk{(char *)p, first, 0});
        else (void)hipGetLastError();
        ml_arena = &arena;
    }
    ~MlArenaScope() {
        (void)hipStreamSynchronize(stream);
        ml_arena = nullptr;
        arena.release();
    }
};

#define ML_TRY(x)                          \
    do {                                   \
        ad_status s_ = (x);                \
        if (s_ != AD_OK) return s_;        \
    } while (0)

// Distances of g at level l (relax with graph id graph_id + l, each
// connected component centred by its own mean, then ad_edge_dist).
static ad_status ml_distances(const ad_graph *g, const ad_ml_opts *o, int l, DevMem &rho, hipStream_t st) {
    const int64_t n1 = std::max<int64_t>(1, g->n);
    DevMem comp_of, members, comp_start, chunk_start, cws;
    ML_TRY(dev_alloc(comp_of, (size_t)n1 * sizeof(int32_t)));
    ML_TRY(dev_alloc(members, (size_t)n1 * sizeof(int32_t)));
    ML_TRY(dev_alloc(comp_start, (size_t)(n1 + 1) * sizeof(int64_t)));
    ML_TRY(dev_alloc(chunk_start, (size_t)(n1 + 1) * sizeof(int64_t)));
    const size_t cb = ad_components_workspace_size(g);
    if (cb == 0) return fail(AD_ERR_INTERNAL, "component workspace size");
    ML_TRY(dev_alloc(cws, cb));
    ad_components comps{};
    ML_TRY(ad_components_build(g, comp_of.get<int32_t>(), members.get<int32_t>(), comp_start.get<int64_t>(),
                               chunk_start.get<int64_t>(), &comps.n_comp, &comps.n_chunks, cws.p, cb, st));
    comps.comp_of = comp_of.get<const int32_t>();
    comps.members = members.get<const int32_t>();
    comps.comp_start = comp_start.get<const int64_t>();
    comps.chunk_start = chunk_start.get<const int64_t>();
    ad_relax_opts ro{};
    ro.R = o->R;
    ro.k = o->k;
    ro.omega = o->omega;
    ro.seed = o->seed;
    ro.graph_id = o->graph_id + (uint64_t)l;
    ro.store = o->store;
    ro.fp32_tail = 1;
    ro.fp64_tail = o->store == AD_F32 ? o->fp64_tail : 0;
    ro.comp = &comps;
    const ad_dtype xt = (o->store == AD_F64 || ro.fp64_tail > 0) ? AD_F64 : AD_F32;
    const size_t xb = xt == AD_F64 ? 8 : 4;
    const size_t rb = o->store == AD_F64 ? 8 : 4;
    DevMem x, mm, ws, wsd;
    ML_TRY(dev_alloc(x, (size_t)n1 * o->R * xb));
    ML_TRY(dev_alloc(mm, 2 * (size_t)o->R * sizeof(double)));
    const size_t wb = ad_relax_workspace_size(g, &ro);
    if (wb == 0) return fail(AD_ERR_INTERNAL, "relax workspace size");
    ML_TRY(dev_alloc(ws, wb));
    ML_TRY(ad_relax(g, &ro, nullptr, x.p, mm.get<double>(), nullptr, nullptr, ws.p, wb, st));
    ML_TRY(dev_alloc(rho, (size_t)std::max<int64_t>(1, g->m) * rb));
    const size_t db = ad_edge_dist_workspace_size(g);
    if (db == 0) return fail(AD_ERR_INTERNAL, "distance workspace size");
    ML_TRY(dev_alloc(wsd, db));
    ML_TRY(ad_edge_dist(g, o->R, xt, x.p, mm.get<double>(), o->store, rho.p, wsd.p, db, st));
    return AD_OK;
}

static void level_span(int32_t n_levels, int32_t span, int32_t segment, double value, double *out) {
    const int32_t lo = segment * n_levels / 3, hi = (segment + 1) * n_levels / 3;
    for (int32_t t = 0; t < n_levels; ++t) out[t] = (t >= lo && t < hi && t - lo < span) ? value : -1.0;
}

// The ratio-vector entry of level l when the coarsest level is D.
static double ml_entry(const ad_ml_opts *o, int32_t D, int32_t l) {
    if (o->span > 0) {
        std::vector<double> v((size_t)D + 1);
        level_span(D + 1, o->span, o->segment, o->span_value, v.data());
        return v[(size_t)(D - l)];
    }
    return o->e_host[D - l];
}

// SparsifyB of one level with its entry x (x < 0: keep every edge).
static ad_status ml_binned(const ad_graph *g, const ad_ml_opts *o, int l, double x, const void *rho, uint8_t *keep,
                           hipStream_t st) {
    if (x < 0.0) return fill_u8(keep, 1, g->m, st);
    DevMem ws, nk;
    const size_t wb = ad_sparsify_binned_workspace_size(g);
    if (wb == 0) return fail(AD_ERR_INTERNAL, "binned workspace size");
    ML_TRY(dev_alloc(ws, wb));
    ML_TRY(dev_alloc(nk, sizeof(int64_t)));
    double e_used = 0.0;
    return ad_sparsify_binned(g, o->store, rho, o->bin_seed, o->graph_id + (uint64_t)l, o->fit ? 0.0 : x,
                              o->fit ? x : 0.0, keep, nk.get<int64_t>(), &e_used, ws.p, wb, st);
}

// keep [g->m] for the graph at level l.
template <typename Tr>
static ad_status ml_level(const ad_graph *g, const ad_ml_opts *o, int l, uint8_t *keep, int32_t *depth,
                          hipStream_t st) {
    const int64_t n = g->n, m = g->m;
    *depth = std::max(*depth, l);
    DevMem rho;
    ML_TRY(ml_distances(g, o, l, rho, st));
    bool coarsest = n <= o->n_min || l + 1 >= o->levels || m == 0;
    DevMem agg, aws;
    int64_t nc = 0;
    if (!coarsest) {
        ML_TRY(dev_alloc(agg, (size_t)n * sizeof(int32_t)));
        const size_t ab = agg_layout(n, 2 * m, nullptr, 0, nullptr);
        ML_TRY(dev_alloc(aws, ab));
        AggLayout L;
        agg_layout(n, 2 * m, aws.p, aws.bytes, &L);
        ML_TRY(aggregate_impl<Tr>(g, rho.get<const Tr>(), o->eps, o->theta, agg.get<int32_t>(), nullptr, &nc, L, st));
        if ((double)nc > 0.9 * (double)n) coarsest = true;
    }
    if (coarsest) return ml_binned(g, o, l, ml_entry(o, l, l), rho.p, keep, st);
    // coarse graph: the fine edges' aggregate pairs merged by ad_ingest (P^T L P)
    DevMem cu, cv, cw, names;
    ML_TRY(dev_alloc(cu, (size_t)m * sizeof(int32_t)));
    ML_TRY(dev_alloc(cv, (size_t)m * sizeof(int32_t)));
    ML_TRY(dev_alloc(cw, (size_t)m * sizeof(float)));
    ML_TRY(dev_alloc(names, (size_t)nc * sizeof(int32_t)));
    hipLaunchKernelGGL(k_ml_pairs, dim3(mwgrid(n)), dim3(MBLOCK), 0, st, n, g->row_ptr, g->col, g->w, g->eid,
                       agg.get<const int32_t>(), cu.get<int32_t>(), cv.get<int32_t>(), cw.get<float>());
    AD_LAUNCH_CHECK("k_ml_pairs");
    AggLayout L;
    agg_layout(n, 2 * m, aws.p, aws.bytes, &L);
    hipLaunchKernelGGL(k_ml_names, dim3(mgrid(n)), dim3(MBLOCK), 0, st, n, L.state, agg.get<const int32_t>(),
                       g->orig_id, names.get<int32_t>());
    AD_LAUNCH_CHECK("k_ml_names");
    DevMem crp, ccol, cwo, ceid, corig, wsi;
    ML_TRY(dev_alloc(crp, (size_t)(nc + 1) * sizeof(int64_t)));
    ML_TRY(dev_alloc(ccol, (size_t)2 * m * sizeof(int32_t)));
    ML_TRY(dev_alloc(cwo, (size_t)2 * m * sizeof(float)));
    ML_TRY(dev_alloc(ceid, (size_t)2 * m * sizeof(int32_t)));
    ML_TRY(dev_alloc(corig, (size_t)nc * sizeof(int32_t)));
    const size_t ib = ad_ingest_workspace_size(nc, m);
    if (ib == 0) return fail(AD_ERR_INTERNAL, "ingest workspace size");
    ML_TRY(dev_alloc(wsi, ib));
    int64_t mc = 0;
    int32_t cdmax = 0;
    ML_TRY(ad_ingest(nc, m, cu.get<int32_t>(), cv.get<int32_t>(), cw.get<float>(), names.get<int32_t>(), 0,
                     crp.get<int64_t>(), ccol.get<int32_t>(), cwo.get<float>(), ceid.get<int32_t>(),
                     corig.get<int32_t>(), &mc, &cdmax, nullptr, wsi.p, ib, st));
    rho.reset();          // the level's distances are no longer needed
    aws.reset();
    wsi.reset();
    ad_graph cg{};
    cg.n = nc;
    cg.m = mc;
    cg.row_ptr = crp.get<int64_t>();
    cg.col = ccol.get<int32_t>();
    cg.w = cwo.get<float>();
    cg.eid = ceid.get<int32_t>();
    cg.orig_id = corig.get<int32_t>();
    cg.d_max = cdmax;
    cg.col_orig = nullptr;
    DevMem ckeep;
    ML_TRY(dev_alloc(ckeep, (size_t)std::max<int64_t>(1, mc)));
    ML_TRY(ml_level<Tr>(&cg, o, l + 1, ckeep.get<uint8_t>(), depth, st));
    // inherit, then SparsifyB on the fine graph less the dropped edges
    DevMem inh;
    ML_TRY(dev_alloc(inh, (size_t)m));
    hipLaunchKernelGGL(k_ml_inherit, dim3(mgrid(m)), dim3(MBLOCK), 0, st, m, cu.get<const int32_t>(),
                       cv.get<const int32_t>(), crp.get<const int64_t>(), ccol.get<const int32_t>(),
                       ceid.get<const int32_t>(), ckeep.get<const uint8_t>(), inh.get<uint8_t>());
    AD_LAUNCH_CHECK("k_ml_inherit");
    const double x = ml_entry(o, *depth, l);
    if (x < 0.0) {          // no SparsifyB here: the inherited state is the result
        AD_HIP(hipMemcpyAsync(keep, inh.p, (size_t)m, hipMemcpyDeviceToDevice, st));
        return AD_OK;
    }
    DevMem srp, scol, sw, seid, soe, wss, dmx;
    ML_TRY(dev_alloc(srp, (size_t)(n + 1) * sizeof(int64_t)));
    ML_TRY(dev_alloc(scol, (size_t)2 * m * sizeof(int32_t)));
    ML_TRY(dev_alloc(seid, (size_t)2 * m * sizeof(int32_t)));
    ML_TRY(dev_alloc(soe, (size_t)2 * m * sizeof(int32_t)));
    if (g->w) ML_TRY(dev_alloc(sw, (size_t)2 * m * sizeof(float)));
    const size_t sb = ad_subgraph_workspace_size(g);
    if (sb == 0) return fail(AD_ERR_INTERNAL, "subgraph workspace size");
    ML_TRY(dev_alloc(wss, sb));
    int64_t ms = 0;
    ML_TRY(ad_subgraph(g, inh.get<uint8_t>(), srp.get<int64_t>(), scol.get<int32_t>(), g->w ? sw.get<float>() : nullptr,
                       seid.get<int32_t>(), soe.get<int32_t>(), &ms, wss.p, sb, st));
    ML_TRY(fill_u8(keep, 0, m, st));
    if (ms > 0) {
        ML_TRY(dev_alloc(dmx, sizeof(unsigned int)));
        ML_TRY(fill_i32(dmx.get<int32_t>(), 0, 1, st));
        hipLaunchKernelGGL(k_ml_degree_max, dim3(std::min<unsigned>(256, mgrid(n))), dim3(MBLOCK), 0, st, n,
                           srp.get<const int64_t>(), dmx.get<unsigned int>());
        AD_LAUNCH_CHECK("k_ml_degree_max");
        unsigned int sdmax = 0;
        AD_HIP(hipMemcpyAsync(&sdmax, dmx.p, sizeof(sdmax), hipMemcpyDeviceToHost, st));
        AD_HIP(hipStreamSynchronize(st));
        ad_graph sg{};
        sg.n = n;
        sg.m = ms;
        sg.row_ptr = srp.get<int64_t>();
        sg.col = scol.get<int32_t>();
        sg.w = g->w ? sw.get<float>() : nullptr;
        sg.eid = seid.get<int32_t>();
        sg.orig_id = g->orig_id;
        sg.d_max = (int32_t)sdmax;
        sg.col_orig = nullptr;
        DevMem srho, skeep;
        ML_TRY(ml_distances(&sg, o, l, srho, st));
        ML_TRY(dev_alloc(skeep, (size_t)ms));
        ML_TRY(ml_binned(&sg, o, l, x, srho.p, skeep.get<uint8_t>(), st));
        hipLaunchKernelGGL(k_ml_map_back, dim3(mgrid(2 * ms)), dim3(MBLOCK), 0, st, 2 * ms, seid.get<const int32_t>(),
                           soe.get<const int32_t>(), skeep.get<const uint8_t>(), keep);
        AD_LAUNCH_CHECK("k_ml_map_back");
    }
    return AD_OK;
}

}  // namespace ad

using namespace ad;

extern "C" ad_status ad_ml_level_span(int32_t n_levels, int32_t span, int32_t segment, double value,
                                      double *out_host) {
    if (n_levels < 1 || n_levels > 64) return fail(AD_ERR_INVALID_ARG, "n_levels must be in [1, 64]");
    if (span < 0 || segment < 0 || segment > 2) return fail(AD_ERR_INVALID_ARG, "span >= 0, segment in 0..2");
    if (!out_host) return fail(AD_ERR_INVALID_ARG, "out_host is NULL");
    level_span(n_levels, span, segment, value, out_host);
    return AD_OK;
}

extern "C" size_t ad_ml_aggregate_workspace_size(const ad_graph *g) {
    if (!g || g->n < 0 || g->n >= ((int64_t)1 << 31)) return 0;
    if (g->m < 0 || g->m >= ((int64_t)1 << 31)) return 0;
    return agg_layout(g->n, 2 * g->m, nullptr, 0, nullptr);
}

extern "C" ad_status ad_ml_aggregate(const ad_graph *g, ad_dtype rho_dtype, const void *rho, double eps, double theta,
                                     int32_t *agg, uint8_t *is_seed, int64_t *n_coarse_host, void *ws,
                                     size_t ws_bytes, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (rho_dtype != AD_F32 && rho_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "rho_dtype must be F32 or F64");
    if (g->m > 0 && !rho) return fail(AD_ERR_INVALID_ARG, "rho is NULL");
    if (g->n > 0 && !agg) return fail(AD_ERR_INVALID_ARG, "agg is NULL");
    if (!n_coarse_host) return fail(AD_ERR_INVALID_ARG, "n_coarse_host is NULL");
    if (!(eps >= 0.0) || !(theta >= 0.0 && theta <= 1.0))
        return fail(AD_ERR_INVALID_ARG, "eps must be >= 0 and theta in [0, 1]");
    if (g->n >= ((int64_t)1 << 31)) return fail(AD_ERR_UNSUPPORTED, "graph too large");
    const size_t need = agg_layout(g->n, 2 * g->m, nullptr, 0, nullptr);
    s = ml_check_ws(ws, need, ws_bytes);
    if (s != AD_OK) return s;
    AggLayout L;
    agg_layout(g->n, 2 * g->m, ws, ws_bytes, &L);
    TraceScope trace("k_ml_aggregate", stream);
    return rho_dtype == AD_F64
               ? aggregate_impl<double>(g, (const double *)rho, eps, theta, agg, is_seed, n_coarse_host, L, stream)
               : aggregate_impl<float>(g, (const float *)rho, eps, theta, agg, is_seed, n_coarse_host, L, stream);
}

extern "C" ad_status ad_ml_sparsify(const ad_graph *g, const ad_ml_opts *o, uint8_t *keep, int64_t *n_kept_host,
                                    int32_t *depth_host, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (!o) return fail(AD_ERR_INVALID_ARG, "opts is NULL");
    if (o->R < 1 || o->R > 64) return fail(AD_ERR_INVALID_ARG, "R must be in [1, 64]");
    if (o->k < 0) return fail(AD_ERR_INVALID_ARG, "k must be >= 0");
    if (!(o->omega > 0.0 && o->omega <= 1.0)) return fail(AD_ERR_INVALID_ARG, "omega must be in (0, 1]");
    if (o->store != AD_F32 && o->store != AD_F64) return fail(AD_ERR_INVALID_ARG, "store must be F32 or F64");
    if (o->levels < 1 || o->levels > 64) return fail(AD_ERR_INVALID_ARG, "levels must be in [1, 64]");
    if (o->n_min < 0) return fail(AD_ERR_INVALID_ARG, "n_min must be >= 0");
    if (o->fit != 0 && o->fit != 1) return fail(AD_ERR_INVALID_ARG, "fit must be 0 or 1");
    if (o->fp64_tail < 0) return fail(AD_ERR_INVALID_ARG, "fp64_tail must be >= 0");
    if (o->span > 0) {
        if (o->segment < 0 || o->segment > 2) return fail(AD_ERR_INVALID_ARG, "segment must be 0, 1 or 2");
        if (!(o->span_value <= 1.0)) return fail(AD_ERR_INVALID_ARG, "span_value must be <= 1");
    } else {
        if (o->span < 0) return fail(AD_ERR_INVALID_ARG, "span must be >= 0");
        if (!o->e_host) return fail(AD_ERR_INVALID_ARG, "e_host is NULL");
        for (int l = 0; l < o->levels; ++l)
            if (!(o->e_host[l] <= 1.0)) return fail(AD_ERR_INVALID_ARG, "ratio entries must be <= 1 (not NaN)");
    }
    if (!(o->eps >= 0.0) || !(o->theta >= 0.0 && o->theta <= 1.0))
        return fail(AD_ERR_INVALID_ARG, "eps must be >= 0 and theta in [0, 1]");
    if (g->m > 0 && !keep) return fail(AD_ERR_INVALID_ARG, "keep is NULL");
    if (!n_kept_host) return fail(AD_ERR_INVALID_ARG, "n_kept_host is NULL");
    if (g->m > 0 && g->d_max <= 0) return fail(AD_ERR_INVALID_ARG, "d_max must be set");
    if (g->m >= ((int64_t)1 << 30) || g->n >= ((int64_t)1 << 31)) return fail(AD_ERR_UNSUPPORTED, "graph too large");
    int32_t depth = 0;
    *n_kept_host = 0;
    if (g->m > 0) {
        TraceScope trace("k_ml_sparsify", stream);
        MlArenaScope arena(stream, g->n, g->m);
        s = o->store == AD_F64 ? ml_level<double>(g, o, 0, keep, &depth, stream)
                               : ml_level<float>(g, o, 0, keep, &depth, stream);
        if (s != AD_OK) return s;
        DevMem cnt;
        ML_TRY(dev_alloc(cnt, sizeof(unsigned long long)));
        ML_TRY(fill_u64(cnt.get<unsigned long long>(), 0, 1, stream));
        hipLaunchKernelGGL(k_ml_count, dim3(std::min<unsigned>(256, mgrid(g->m))), dim3(MBLOCK), 0, stream, g->m,
                           keep, cnt.get<unsigned long long>());
        AD_LAUNCH_CHECK("k_ml_count");
        unsigned long long kept = 0;
        AD_HIP(hipMemcpyAsync(&kept, cnt.p, sizeof(kept), hipMemcpyDeviceToHost, stream));
        AD_HIP(hipStreamSynchronize(stream));
        *n_kept_host = (int64_t)kept;
    }
    if (depth_host) *depth_host = depth;
    return AD_OK;
}
