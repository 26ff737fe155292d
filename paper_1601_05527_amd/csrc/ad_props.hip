// Properties by which the paper compares a sparsified graph with the
// original (Preliminaries): the sparsified subgraph itself, per-vertex
// triangle counts lambda_i, clustering c_i = lambda_i / (d_i (d_i - 1) / 2),
// C_G = the mean of c_i over d_i > 1 (Eq. cc), connected components, and the
// Spearman rank correlation of two per-vertex scores by the stated formula
// rho = 1 - 6 sum p_i^2 / (n (n^2 - 1)) (tied scores share the mean of
// their ranks).
#include "ad_internal.h"

#include <cstring>    // before rocPRIM: its host code calls memset

#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <cstdint>

namespace ad {

constexpr int PBLOCK = 256;
constexpr int PREDUCE_BLOCKS = 1024;     // fixed grid: reductions in a fixed order
constexpr int64_t TRI_LANE = 64;         // pairs whose shorter row fits this are counted by one lane

static unsigned pgrid(int64_t count) { return grid_for(std::max<int64_t>(1, count), PBLOCK); }

// ------------------------------------------------------------- subgraph --

__global__ void k_keep_u32(int64_t m, const uint8_t *__restrict__ keep, uint32_t *__restrict__ k32) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        k32[e] = keep[e] ? 1u : 0u;
}

// Kept flag of every stored entry, as the input of the entry scan.
struct EntryKept {
    const uint8_t *keep;
    const int32_t *eid;
    __device__ uint32_t operator()(int64_t p) const { return keep[eid[p]] ? 1u : 0u; }
};
using EntryKeptIt = rocprim::transform_iterator<rocprim::counting_iterator<int64_t>, EntryKept, uint32_t>;
static EntryKeptIt entry_kept(const uint8_t *keep, const int32_t *eid) {
    return EntryKeptIt(rocprim::counting_iterator<int64_t>(0), EntryKept{keep, eid});
}

// The subgraph keeps the stored order, so pos[p] (kept entries before p)
// places entry p, and a row starts at pos of its first entry.
__global__ void k_sub_rows(int64_t n, int64_t nnz, const int64_t *__restrict__ row_ptr,
                           const int32_t *__restrict__ eid, const uint8_t *__restrict__ keep,
                           const uint32_t *__restrict__ pos, int64_t *__restrict__ sub_row_ptr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = row_ptr[i];
        int64_t v = 0;
        if (p < nnz) v = pos[p];
        else if (nnz > 0) v = (int64_t)pos[nnz - 1] + (keep[eid[nnz - 1]] ? 1 : 0);
        sub_row_ptr[i] = v;
    }
}

__global__ void k_compact_entries(int64_t nnz, const int32_t *__restrict__ col, const float *__restrict__ w,
                                  const int32_t *__restrict__ eid, const uint8_t *__restrict__ keep,
                                  const uint32_t *__restrict__ new_id, const uint32_t *__restrict__ pos,
                                  int32_t *__restrict__ sub_col, float *__restrict__ sub_w,
                                  int32_t *__restrict__ sub_eid, int32_t *__restrict__ orig_edge) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = eid[p];
        if (!keep[e]) continue;
        const uint32_t q = pos[p];
        sub_col[q] = col[p];
        if (sub_w) sub_w[q] = w[p];
        sub_eid[q] = (int32_t)new_id[e];
        if (orig_edge) orig_edge[q] = e;
    }
}

// ------------------------------------------------------------ triangles --

// |N_a ∩ N_b| for sorted rows, by binary searches of the shorter row's
// entries [s0 + first, s1) (stepping by `step`) in the longer one.
__device__ __forceinline__ int64_t common_count(const int32_t *__restrict__ col, int64_t s0, int64_t s1,
                                                int64_t l0, int64_t l1, int64_t first, int64_t step) {
    int64_t t = 0;
    for (int64_t q = s0 + first; q < s1; q += step) {
        const int32_t x = col[q];
        int64_t lo = l0, hi = l1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (col[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        t += (lo < l1 && col[lo] == x) ? 1 : 0;
    }
    return t;
}

// Every edge (i, j), i < j, adds |N_i ∩ N_j| to both ends (each triangle at i
// is then counted once through each of its two edges at i).  Pairs whose
// shorter row exceeds TRI_LANE are left to k_triangles_hub(_bits), and with
// both_short also those whose longer row does (k_triangles_hub_bits takes
// them from the long row's bitmap).
__global__ void k_triangles_lane(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                 int both_short, unsigned long long *__restrict__ lam2) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (PBLOCK / WAVE);
    for (int64_t i = (int64_t)blockIdx.x * (PBLOCK / WAVE) + (threadIdx.x >> 6); i < n; i += nw) {
        const int64_t b0 = row_ptr[i], b1 = row_ptr[i + 1];
        unsigned long long own = 0;
        for (int64_t base = b0; base < b1; base += WAVE) {
            const int64_t p = base + lane;
            const int32_t j = p < b1 ? col[p] : -1;
            const bool up = j > i;
            int64_t c0 = 0, c1 = 0;
            if (up) {
                c0 = row_ptr[j];
                c1 = row_ptr[j + 1];
            }
            const bool i_short = (b1 - b0) <= (c1 - c0);
            const int64_t shorter = i_short ? b1 - b0 : c1 - c0;
            const int64_t longer = i_short ? c1 - c0 : b1 - b0;
            const bool is_big = up && (shorter > TRI_LANE || (both_short && longer > TRI_LANE));
            if (up && !is_big) {
                const int64_t t =
                    i_short ? common_count(col, b0, b1, c0, c1, 0, 1) : common_count(col, c0, c1, b0, b1, 0, 1);
                own += (unsigned long long)t;
                if (t) atomicAdd(&lam2[j], (unsigned long long)t);
            }
        }
        for (int o = WAVE / 2; o >= 1; o >>= 1) own += __shfl_xor(own, o, WAVE);
        if (lane == 0 && own) atomicAdd(&lam2[i], own);
    }
}

// Pairs of rows both longer than TRI_LANE, each counted by the endpoint of
// larger (degree, id): one workgroup per such row L holds N_L in LDS (when
// it has at most TRI_LDS entries, else it is searched in memory) for all of
// its pairs; each wave takes a neighbour j and its lanes, striding over
// N_j, binary-search N_L.
constexpr int TRI_LDS = 8192;

__global__ __launch_bounds__(PBLOCK) void k_triangles_hub(int64_t n, const int64_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col,
                                                          unsigned long long *__restrict__ lam2) {
    __shared__ int32_t lrow[TRI_LDS];
    __shared__ unsigned long long wsum[PBLOCK / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
    for (int64_t L = blockIdx.x; L < n; L += gridDim.x) {
        const int64_t l0 = row_ptr[L], l1 = row_ptr[L + 1], dl = l1 - l0;
        if (dl <= TRI_LANE) continue;                       // uniform over the workgroup
        const bool in_lds = dl <= TRI_LDS;
        if (in_lds)
            for (int64_t q = threadIdx.x; q < dl; q += PBLOCK) lrow[q] = col[l0 + q];
        __syncthreads();
        unsigned long long own = 0;
        for (int64_t p = l0 + wv; p < l1; p += PBLOCK / WAVE) {
            const int32_t j = col[p];
            const int64_t c0 = row_ptr[j], c1 = row_ptr[j + 1], dj = c1 - c0;
            if (dj <= TRI_LANE || dj > dl || (dj == dl && j > L)) continue;     // uniform over the wave
            int64_t t = 0;
            for (int64_t q = c0 + lane; q < c1; q += WAVE) {
                const int32_t x = col[q];
                if (in_lds) {
                    int lo = 0, hi = (int)dl;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (lrow[mid] < x) lo = mid + 1;
                        else hi = mid;
                    }
                    t += (lo < dl && lrow[lo] == x) ? 1 : 0;
                } else {
                    int64_t lo = l0, hi = l1;
                    while (lo < hi) {
                        const int64_t mid = (lo + hi) >> 1;
                        if (col[mid] < x) lo = mid + 1;
                        else hi = mid;
                    }
                    t += (lo < l1 && col[lo] == x) ? 1 : 0;
                }
            }
            for (int o = WAVE / 2; o >= 1; o >>= 1) t += __shfl_xor(t, o, WAVE);
            if (lane == 0 && t) {
                atomicAdd(&lam2[j], (unsigned long long)t);
                own += (unsigned long long)t;
            }
        }
        if (lane == 0) wsum[wv] = own;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int q = 0; q < PBLOCK / WAVE; ++q) tot += wsum[q];
            if (tot) atomicAdd(&lam2[L], tot);
        }
        __syncthreads();     // lrow and wsum are reused by the next row
    }
}

// The pairs of a long row L with every neighbour of no larger (degree, id),
// short neighbours included, with N_L held as a bitmap over its id range [lo, hi]
// (rows are sorted, so lo and hi are its first and last entries) when that
// range has at most TRI_BITS ids: a lookup is one LDS read instead of a
// binary search (used for graphs of at most TRI_BITS vertices; a row with
// a wider range would search N_L in memory).  The bitmap
// is cleared once per workgroup and, after each row, only in the words that
// row set.  Needs TRI_BITS / 8 bytes of LDS per workgroup.
constexpr int TRI_BT = 1024;
constexpr int64_t TRI_BITS = (int64_t)1 << 20;

__global__ __launch_bounds__(TRI_BT) void k_triangles_hub_bits(int64_t n, const int64_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col,
                                                               unsigned long long *__restrict__ lam2) {
    extern __shared__ uint32_t bm[];                       // TRI_BITS / 32 words
    __shared__ unsigned long long wsum[TRI_BT / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
    for (int64_t q = threadIdx.x; q < TRI_BITS / 32; q += TRI_BT) bm[q] = 0u;
    __syncthreads();
    for (int64_t L = blockIdx.x; L < n; L += gridDim.x) {
        const int64_t l0 = row_ptr[L], l1 = row_ptr[L + 1], dl = l1 - l0;
        if (dl <= TRI_LANE) continue;                       // uniform over the workgroup
        const int64_t lo = col[l0], span = (int64_t)col[l1 - 1] - lo + 1;
        const bool bits = span <= TRI_BITS;
        if (bits) {
            for (int64_t q = threadIdx.x; q < dl; q += TRI_BT) {
                const int64_t r = (int64_t)col[l0 + q] - lo;
                atomicOr(&bm[r >> 5], 1u << (r & 31));
            }
        }
        __syncthreads();
        // whether id x is in N_L
        auto in_l = [&](int32_t x) -> int64_t {
            if (bits) {
                const int64_t r = (int64_t)x - lo;
                return (r >= 0 && r < span) ? (int64_t)((bm[r >> 5] >> (r & 31)) & 1u) : 0;
            }
            int64_t a = l0, b = l1;
            while (a < b) {
                const int64_t mid = (a + b) >> 1;
                if (col[mid] < x) a = mid + 1;
                else b = mid;
            }
            return (a < l1 && col[a] == x) ? 1 : 0;
        };
        unsigned long long own = 0;
        // short neighbours: one lane each, over the whole of N_j
        for (int64_t p0 = l0 + (int64_t)wv * WAVE; p0 < l1; p0 += TRI_BT) {
            const int64_t p = p0 + lane;
            if (p >= l1) continue;
            const int32_t j = col[p];
            const int64_t c0 = row_ptr[j], c1 = row_ptr[j + 1];
            if (c1 - c0 > TRI_LANE) continue;
            int64_t t = 0;
            for (int64_t q0 = c0; q0 < c1; q0 += 8) {                  // eight loads in flight
                int32_t x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = q0 + u < c1 ? col[q0 + u] : -1;
#pragma unroll
                for (int u = 0; u < 8; ++u) t += x[u] >= 0 ? in_l(x[u]) : 0;
            }
            if (t) {
                atomicAdd(&lam2[j], (unsigned long long)t);
                own += (unsigned long long)t;
            }
        }
        // long neighbours: one wave each, lanes striding over N_j
        for (int64_t p = l0 + wv; p < l1; p += TRI_BT / WAVE) {
            const int32_t j = col[p];
            const int64_t c0 = row_ptr[j], c1 = row_ptr[j + 1], dj = c1 - c0;
            if (dj <= TRI_LANE || dj > dl || (dj == dl && j > L)) continue;     // uniform over the wave
            int64_t t = 0;
            for (int64_t q = c0 + lane; q < c1; q += WAVE) t += in_l(col[q]);
            for (int o = WAVE / 2; o >= 1; o >>= 1) t += __shfl_xor(t, o, WAVE);
            if (lane == 0 && t) {
                atomicAdd(&lam2[j], (unsigned long long)t);
                own += (unsigned long long)t;
            }
        }
        for (int o = WAVE / 2; o >= 1; o >>= 1) own += __shfl_xor(own, o, WAVE);
        if (lane == 0) wsum[wv] = own;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int q = 0; q < TRI_BT / WAVE; ++q) tot += wsum[q];
            if (tot) atomicAdd(&lam2[L], tot);
        }
        if (bits)
            for (int64_t q = threadIdx.x; q < dl; q += TRI_BT) bm[((int64_t)col[l0 + q] - lo) >> 5] = 0u;
        __syncthreads();     // bm and wsum are reused by the next row
    }
}

// Whether the current device gives a workgroup the bitmap's LDS.
static bool tri_bits_fit() {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return false;
    return (int64_t)lds >= TRI_BITS / 8 + (int64_t)sizeof(unsigned long long) * (TRI_BT / WAVE);
}

// lambda_i and c_i; per-block partial sums of c_i over d_i > 1 (and their
// count), in a fixed order for the host to finish.
__global__ void k_clustering(int64_t n, const int64_t *__restrict__ row_ptr, const unsigned long long *__restrict__ lam2,
                             int64_t *__restrict__ lambda, double *__restrict__ c, double *__restrict__ part_sum,
                             unsigned long long *__restrict__ part_cnt) {
    __shared__ double ssum[PBLOCK];
    __shared__ unsigned long long scnt[PBLOCK];
    double s = 0.0;
    unsigned long long k = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = (int64_t)(lam2[i] / 2);
        const int64_t d = row_ptr[i + 1] - row_ptr[i];
        double ci = 0.0;
        if (d > 1) {
            ci = (double)l / ((double)d * (double)(d - 1) / 2.0);
            s += ci;
            ++k;
        }
        if (lambda) lambda[i] = l;
        if (c) c[i] = ci;
    }
    ssum[threadIdx.x] = s;
    scnt[threadIdx.x] = k;
    __syncthreads();
    for (int o = PBLOCK / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            ssum[threadIdx.x] += ssum[threadIdx.x + o];
            scnt[threadIdx.x] += scnt[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_sum[blockIdx.x] = ssum[0];
        part_cnt[blockIdx.x] = scnt[0];
    }
}

// ----------------------------------------------------------- components --

__global__ void k_parent_init(int64_t n, int32_t *__restrict__ parent) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        parent[i] = (int32_t)i;
}

// Root of x, halving the path on the way: x is pointed at its grandparent
// with atomicMin.  Ids decrease along every path, so the smaller of two
// ancestors is the one nearer the root: a halving never moves a vertex away
// from its root, whatever other halvings or final writes it races with.
__device__ __forceinline__ int32_t uf_root(int32_t *parent, int32_t x) {
    int32_t px = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (px != x) {
        const int32_t ppx = __hip_atomic_load(&parent[px], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ppx != px) atomicMin(&parent[x], ppx);
        x = px;
        px = ppx;
    }
    return x;
}

// Join the trees of a and b: the larger root goes under the smaller; a
// failed compare-and-swap means that root was just joined elsewhere, and
// the roots are looked up again.
__device__ __forceinline__ void uf_union(int32_t *parent, int32_t a, int32_t b) {
    for (;;) {
        a = uf_root(parent, a);
        b = uf_root(parent, b);
        if (a == b) return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&parent[b], b, a) == b) return;
    }
}

// Joins in two passes (the sampling idea of Afforest, Sutton et al., 2018):
// first the first UF_FIRST entries of every row, which in a connected
// power-law graph already gather most vertices under the root of vertex 0
// (its component's smallest id); then the remaining entries of every row
// whose root is not 0 at that moment.  A skipped row's vertex is joined to
// 0, and any edge from it to a vertex outside 0's tree is taken from that
// vertex's own row, which is not skipped, so every component is found.
constexpr int UF_FIRST = 2;

__global__ void k_union_first(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                              int32_t *__restrict__ parent) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = row_ptr[i], e = min(row_ptr[i + 1], b + UF_FIRST);
        for (int64_t p = b; p < e; ++p) uf_union(parent, (int32_t)i, col[p]);
    }
}

// One wave per row: the entries after the first UF_FIRST, unless the row's
// vertex already hangs under 0.
__global__ void k_union_rest(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                             int32_t *__restrict__ parent) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (PBLOCK / WAVE);
    for (int64_t i = (int64_t)blockIdx.x * (PBLOCK / WAVE) + (threadIdx.x >> 6); i < n; i += nw) {
        const int64_t b = row_ptr[i] + UF_FIRST, b1 = row_ptr[i + 1];
        if (b >= b1) continue;                                    // uniform across the wave
        int32_t r = 0;
        if (lane == 0) r = uf_root(parent, (int32_t)i);
        if (shfl(r, 0) == 0) continue;
        for (int64_t p = b + lane; p < b1; p += WAVE) uf_union(parent, (int32_t)i, col[p]);
    }
}

// Every vertex points at the root of its tree (atomicMin: the root is the
// smallest ancestor, so a late halving by another thread cannot replace it).
__global__ void k_flatten(int64_t n, int32_t *__restrict__ parent) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        atomicMin(&parent[i], uf_root(parent, (int32_t)i));
}

__global__ void k_count_roots(int64_t n, const int32_t *__restrict__ parent, unsigned long long *__restrict__ cnt) {
    unsigned long long k = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        k += parent[i] == (int32_t)i ? 1 : 0;
    for (int o = WAVE / 2; o >= 1; o >>= 1) k += __shfl_xor(k, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0 && k) atomicAdd(cnt, k);
}

// Grouping of the components for the relaxation's per-component centring:
// sort keys (the component's smallest vertex; isolated vertices last).
__global__ void k_comp_keys(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ parent,
                            uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        key[i] = row_ptr[i + 1] > row_ptr[i] ? (uint32_t)parent[i] : (uint32_t)n;   // isolated: n, sorted last
        val[i] = (uint32_t)i;
    }
}

// head[p] = 1 where sorted position p starts a component.
__global__ void k_comp_heads(int64_t n, const uint32_t *__restrict__ key, uint32_t *__restrict__ head) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        head[p] = (key[p] != (uint32_t)n && (p == 0 || key[p] != key[p - 1])) ? 1u : 0u;
}

// comp_of, members and the component starts from the sorted order and the
// exclusive scan of the heads; the last live position closes the last
// component.
__global__ void k_comp_fill(int64_t n, const uint32_t *__restrict__ key, const uint32_t *__restrict__ val,
                            const uint32_t *__restrict__ head, const uint32_t *__restrict__ before,
                            int32_t *__restrict__ comp_of, int32_t *__restrict__ members,
                            int64_t *__restrict__ comp_start) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)val[p];
        if (key[p] == (uint32_t)n) {
            comp_of[v] = -1;
            continue;
        }
        const int64_t c = (int64_t)before[p] + head[p] - 1;
        comp_of[v] = (int32_t)c;
        members[p] = v;
        if (head[p]) comp_start[c] = p;
        if (p + 1 == n || key[p + 1] == (uint32_t)n) comp_start[c + 1] = p + 1;
    }
}

// Chunks of COMP_CHUNK members per component (the entry after the last is 0,
// so an exclusive scan ends with the total).
__global__ void k_comp_chunks(int64_t nc, const int64_t *__restrict__ comp_start, int64_t *__restrict__ cnt) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= nc; c += (int64_t)gridDim.x * blockDim.x)
        cnt[c] = c < nc ? (comp_start[c + 1] - comp_start[c] + COMP_CHUNK - 1) / COMP_CHUNK : 0;
}

// ------------------------------------------------------------- spearman --

__global__ void k_iota(int64_t n, uint32_t *__restrict__ idx) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        idx[i] = (uint32_t)i;
}

// Twice the mean rank of every score, from the sorted scores: a run of equal
// scores at sorted positions [a, b) holds ranks a+1 .. b, mean (a + 1 + b) / 2.
__global__ void k_mean_ranks(int64_t n, const double *__restrict__ sorted, const uint32_t *__restrict__ idx,
                             int64_t *__restrict__ rank2) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double v = sorted[t];
        int64_t a = t, b = t + 1;
        // run bounds by binary search over the sorted scores
        int64_t lo = 0, hi = t;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sorted[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        a = lo;
        lo = t + 1;
        hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sorted[mid] <= v) lo = mid + 1;
            else hi = mid;
        }
        b = lo;
        rank2[idx[t]] = a + 1 + b;
    }
}

// Per-block sums of (2 p_i)^2 in a fixed order (exact while below 2^53 per term).
__global__ void k_rank_diff2(int64_t n, const int64_t *__restrict__ rx2, const int64_t *__restrict__ ry2,
                             double *__restrict__ part) {
    __shared__ double s[PBLOCK];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)(rx2[i] - ry2[i]);
        acc += d * d;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = PBLOCK / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// ------------------------------------------------------------- layouts --

struct SubLayout {
    uint32_t *k32, *new_id;   // [m]
    uint32_t *pos;            // [2m] kept entries before each stored entry
    void *temp;
    size_t temp_bytes;
};

static size_t sub_layout(const ad_graph *g, void *ws, size_t ws_bytes, SubLayout *L) {
    Carver c(ws, ws_bytes);
    const size_t m = (size_t)std::max<int64_t>(1, g->m);
    SubLayout l;
    l.k32 = c.take<uint32_t>(m);
    l.new_id = c.take<uint32_t>(m);
    l.pos = c.take<uint32_t>(2 * m);
    size_t t1 = 0, t2 = 0;
    if (rocprim::exclusive_scan(nullptr, t1, (uint32_t *)nullptr, (uint32_t *)nullptr, 0u, m,
                                rocprim::plus<uint32_t>()) != hipSuccess)
        t1 = 0;
    if (rocprim::exclusive_scan(nullptr, t2, entry_kept(nullptr, nullptr), (uint32_t *)nullptr, 0u, 2 * m,
                                rocprim::plus<uint32_t>()) != hipSuccess)
        t2 = 0;
    l.temp_bytes = std::max(t1, t2);
    l.temp = c.take<char>(l.temp_bytes);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

struct PropLayout {
    unsigned long long *lam2;     // [n]
    unsigned int *flags;          // [4]: listed pairs, changed
    unsigned long long *roots;    // [1]
    double *part_sum;             // [PREDUCE_BLOCKS]
    unsigned long long *part_cnt; // [PREDUCE_BLOCKS]
    int32_t *parent;              // [n] when the caller passes no comp array
};

static size_t prop_layout(const ad_graph *g, void *ws, size_t ws_bytes, PropLayout *L) {
    Carver c(ws, ws_bytes);
    const size_t m = (size_t)std::max<int64_t>(1, g->m), n = (size_t)std::max<int64_t>(1, g->n);
    PropLayout l;
    l.lam2 = c.take<unsigned long long>(n);
    l.flags = c.take<unsigned int>(4);
    l.roots = c.take<unsigned long long>(1);
    l.part_sum = c.take<double>(PREDUCE_BLOCKS);
    l.part_cnt = c.take<unsigned long long>(PREDUCE_BLOCKS);
    l.parent = c.take<int32_t>(n);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

// Connected components by union-find: the entries (i, j) join the trees of
// i and j (k_union_first, then k_union_rest for the rows not yet under 0),
// hanging the larger root under the smaller with a compare-and-swap, then
// every vertex is pointed at its root.  Parent ids only ever decrease (a
// parent is always smaller than its child), so the trees have no cycles,
// every root search ends, and each component's root is its smallest vertex
// whatever the order of the joins.  flags is unused.  No host round trips.
ad_status label_components(const ad_graph *g, int32_t *parent, unsigned int *flags, hipStream_t stream) {
    (void)flags;
    const int64_t n = g->n;
    const unsigned wgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(n, PBLOCK / WAVE)));
    hipLaunchKernelGGL(k_parent_init, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, parent);
    AD_LAUNCH_CHECK("k_parent_init");
    if (g->m > 0) {
        hipLaunchKernelGGL(k_union_first, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, g->row_ptr, g->col, parent);
        AD_LAUNCH_CHECK("k_union_first");
        hipLaunchKernelGGL(k_union_rest, dim3(wgrid), dim3(PBLOCK), 0, stream, n, g->row_ptr, g->col, parent);
        AD_LAUNCH_CHECK("k_union_rest");
    }
    hipLaunchKernelGGL(k_flatten, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, parent);
    AD_LAUNCH_CHECK("k_flatten");
    return AD_OK;
}

struct CompLayout {
    int32_t *parent;              // [n]
    unsigned int *flags;          // [4]
    uint32_t *key0, *key1, *val0, *val1, *head, *before;   // [n]
    int64_t *cnt;                 // [n + 1]
    void *temp;
    size_t temp_bytes;
};

static size_t comp_layout(int64_t n, void *ws, size_t ws_bytes, CompLayout *L) {
    Carver c(ws, ws_bytes);
    const size_t nn = (size_t)std::max<int64_t>(1, n);
    CompLayout l;
    l.parent = c.take<int32_t>(nn);
    l.flags = c.take<unsigned int>(4);
    l.key0 = c.take<uint32_t>(nn);
    l.key1 = c.take<uint32_t>(nn);
    l.val0 = c.take<uint32_t>(nn);
    l.val1 = c.take<uint32_t>(nn);
    l.head = c.take<uint32_t>(nn);
    l.before = c.take<uint32_t>(nn);
    l.cnt = c.take<int64_t>(nn + 1);
    size_t t0 = 0, t1 = 0, t2 = 0;
    if (rocprim::radix_sort_pairs(nullptr, t0, (uint32_t *)nullptr, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                  (uint32_t *)nullptr, nn) != hipSuccess)
        t0 = 0;
    if (rocprim::exclusive_scan(nullptr, t1, (uint32_t *)nullptr, (uint32_t *)nullptr, 0u, nn,
                                rocprim::plus<uint32_t>()) != hipSuccess)
        t1 = 0;
    if (rocprim::exclusive_scan(nullptr, t2, (int64_t *)nullptr, (int64_t *)nullptr, (int64_t)0, nn + 1,
                                rocprim::plus<int64_t>()) != hipSuccess)
        t2 = 0;
    l.temp_bytes = std::max(t0, std::max(t1, t2));
    l.temp = c.take<char>(l.temp_bytes);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

struct RankLayout {
    double *keys0, *keys1;        // [n]
    uint32_t *idx0, *idx1;        // [n]
    int64_t *rx2, *ry2;           // [n]
    double *part;                 // [PREDUCE_BLOCKS]
    void *temp;
    size_t temp_bytes;
};

static size_t rank_layout(int64_t n, void *ws, size_t ws_bytes, RankLayout *L) {
    Carver c(ws, ws_bytes);
    const size_t nn = (size_t)std::max<int64_t>(1, n);
    RankLayout l;
    l.keys0 = c.take<double>(nn);
    l.keys1 = c.take<double>(nn);
    l.idx0 = c.take<uint32_t>(nn);
    l.idx1 = c.take<uint32_t>(nn);
    l.rx2 = c.take<int64_t>(nn);
    l.ry2 = c.take<int64_t>(nn);
    l.part = c.take<double>(PREDUCE_BLOCKS);
    size_t t = 0;
    if (rocprim::radix_sort_pairs(nullptr, t, (double *)nullptr, (double *)nullptr, (uint32_t *)nullptr,
                                  (uint32_t *)nullptr, nn) != hipSuccess)
        t = 0;
    l.temp_bytes = t;
    l.temp = c.take<char>(t);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

#define AD_RP(call)                                                         \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) return fail(AD_ERR_HIP, std::string("rocPRIM: ") + hipGetErrorString(e_)); \
    } while (0)

static ad_status check_ws(void *ws, size_t need, size_t ws_bytes) {
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (need == 0 || ws_bytes < need) return fail(AD_ERR_WORKSPACE, "workspace too small");
    return AD_OK;
}

}  // namespace ad

using namespace ad;

extern "C" size_t ad_subgraph_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK) return 0;
    return sub_layout(g, nullptr, 0, nullptr);
}

extern "C" ad_status ad_subgraph(const ad_graph *g, const uint8_t *keep, int64_t *sub_row_ptr, int32_t *sub_col,
                                 float *sub_w, int32_t *sub_eid, int32_t *orig_edge, int64_t *m_sub_host, void *ws,
                                 size_t ws_bytes, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (g->m > 0 && !keep) return fail(AD_ERR_INVALID_ARG, "keep is NULL");
    if (!sub_row_ptr || !m_sub_host) return fail(AD_ERR_INVALID_ARG, "sub_row_ptr or m_sub_host is NULL");
    if (g->m > 0 && (!sub_col || !sub_eid)) return fail(AD_ERR_INVALID_ARG, "sub_col or sub_eid is NULL");
    if (g->m >= ((int64_t)1 << 31)) return fail(AD_ERR_UNSUPPORTED, "more than 2^31 - 1 edges");
    s = check_ws(ws, sub_layout(g, nullptr, 0, nullptr), ws_bytes);
    if (s != AD_OK) return s;
    SubLayout L;
    if (sub_layout(g, ws, ws_bytes, &L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    TraceScope trace("k_subgraph", stream);
    const int64_t n = g->n, m = g->m;
    uint32_t last[2] = {0, 0};
    if (m > 0) {
        hipLaunchKernelGGL(k_keep_u32, dim3(pgrid(m)), dim3(PBLOCK), 0, stream, m, keep, L.k32);
        AD_LAUNCH_CHECK("k_keep_u32");
        size_t tb = L.temp_bytes;
        AD_RP(rocprim::exclusive_scan(L.temp, tb, L.k32, L.new_id, 0u, (size_t)m, rocprim::plus<uint32_t>(), stream));
        AD_HIP(hipMemcpyAsync(&last[0], L.new_id + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        AD_HIP(hipMemcpyAsync(&last[1], L.k32 + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    }
    if (m > 0) {
        size_t tb = L.temp_bytes;
        AD_RP(rocprim::exclusive_scan(L.temp, tb, entry_kept(keep, g->eid), L.pos, 0u, (size_t)(2 * m),
                                      rocprim::plus<uint32_t>(), stream));
    }
    hipLaunchKernelGGL(k_sub_rows, dim3(pgrid(n + 1)), dim3(PBLOCK), 0, stream, n, 2 * m, g->row_ptr, g->eid, keep,
                       L.pos, sub_row_ptr);
    AD_LAUNCH_CHECK("k_sub_rows");
    if (m > 0) {
        hipLaunchKernelGGL(k_compact_entries, dim3(pgrid(2 * m)), dim3(PBLOCK), 0, stream, 2 * m, g->col, g->w,
                           g->eid, keep, L.new_id, L.pos, sub_col, g->w ? sub_w : nullptr, sub_eid, orig_edge);
        AD_LAUNCH_CHECK("k_compact_entries");
    }
    AD_HIP(hipStreamSynchronize(stream));
    *m_sub_host = (int64_t)last[0] + (int64_t)last[1];
    return AD_OK;
}

extern "C" size_t ad_graph_properties_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK) return 0;
    return prop_layout(g, nullptr, 0, nullptr);
}

extern "C" ad_status ad_graph_properties(const ad_graph *g, int64_t *lambda, double *c, int32_t *comp,
                                         double *summary_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (!summary_host) return fail(AD_ERR_INVALID_ARG, "summary_host is NULL");
    if (g->m >= ((int64_t)1 << 31)) return fail(AD_ERR_UNSUPPORTED, "more than 2^31 - 1 edges");
    s = check_ws(ws, prop_layout(g, nullptr, 0, nullptr), ws_bytes);
    if (s != AD_OK) return s;
    PropLayout L;
    if (prop_layout(g, ws, ws_bytes, &L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    TraceScope trace("k_properties", stream);
    const int64_t n = g->n;
    summary_host[0] = 0.0;
    summary_host[1] = 0.0;
    if (n == 0) return AD_OK;
    const unsigned wgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(n, PBLOCK / WAVE)));
    // triangles and clustering
    s = fill_u64(L.lam2, 0, n, stream);
    if (s != AD_OK) return s;
    s = fill_i32((int32_t *)L.flags, 0, 4, stream);
    if (s != AD_OK) return s;
    if (g->m > 0) {
        // with at most TRI_BITS vertices every row's id range fits the bitmap
        const bool use_bits = n <= TRI_BITS && tri_bits_fit();
        hipLaunchKernelGGL(k_triangles_lane, dim3(wgrid), dim3(PBLOCK), 0, stream, n, g->row_ptr, g->col,
                           use_bits ? 1 : 0, L.lam2);
        AD_LAUNCH_CHECK("k_triangles_lane");
        if (use_bits) {
            hipLaunchKernelGGL(k_triangles_hub_bits, dim3((unsigned)std::min<int64_t>(4096, n)), dim3(TRI_BT),
                               (size_t)(TRI_BITS / 8), stream, n, g->row_ptr, g->col, L.lam2);
            AD_LAUNCH_CHECK("k_triangles_hub_bits");
        } else {
            hipLaunchKernelGGL(k_triangles_hub, dim3((unsigned)std::min<int64_t>(4096, n)), dim3(PBLOCK), 0, stream,
                               n, g->row_ptr, g->col, L.lam2);
            AD_LAUNCH_CHECK("k_triangles_hub");
        }
    }
    hipLaunchKernelGGL(k_clustering, dim3(PREDUCE_BLOCKS), dim3(PBLOCK), 0, stream, n, g->row_ptr, L.lam2, lambda, c,
                       L.part_sum, L.part_cnt);
    AD_LAUNCH_CHECK("k_clustering");
    // components: hook and jump until no hook changes a parent
    int32_t *parent = comp ? comp : L.parent;
    s = label_components(g, parent, L.flags, stream);
    if (s != AD_OK) return s;
    s = fill_u64(L.roots, 0, 1, stream);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_count_roots, dim3(std::min<unsigned>(256, pgrid(n))), dim3(PBLOCK), 0, stream, n, parent,
                       L.roots);
    AD_LAUNCH_CHECK("k_count_roots");
    double psum[PREDUCE_BLOCKS];
    unsigned long long pcnt[PREDUCE_BLOCKS], roots = 0;
    AD_HIP(hipMemcpyAsync(psum, L.part_sum, sizeof(psum), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipMemcpyAsync(pcnt, L.part_cnt, sizeof(pcnt), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipMemcpyAsync(&roots, L.roots, sizeof(roots), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipStreamSynchronize(stream));
    double sum = 0.0;
    unsigned long long cnt = 0;
    for (int b = 0; b < PREDUCE_BLOCKS; ++b) {
        sum += psum[b];
        cnt += pcnt[b];
    }
    summary_host[0] = cnt ? sum / (double)cnt : 0.0;
    summary_host[1] = (double)roots;
    return AD_OK;
}

extern "C" size_t ad_components_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK || g->n >= ((int64_t)1 << 31)) return 0;
    return comp_layout(g->n, nullptr, 0, nullptr);
}

extern "C" ad_status ad_components_build(const ad_graph *g, int32_t *comp_of, int32_t *members, int64_t *comp_start,
                                         int64_t *chunk_start, int64_t *n_comp_host, int64_t *n_chunks_host,
                                         void *ws, size_t ws_bytes, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (!n_comp_host || !n_chunks_host) return fail(AD_ERR_INVALID_ARG, "n_comp_host or n_chunks_host is NULL");
    if (!comp_start || !chunk_start) return fail(AD_ERR_INVALID_ARG, "comp_start or chunk_start is NULL");
    if (g->n > 0 && (!comp_of || !members)) return fail(AD_ERR_INVALID_ARG, "comp_of or members is NULL");
    if (g->n >= ((int64_t)1 << 31)) return fail(AD_ERR_UNSUPPORTED, "n must be below 2^31");
    s = check_ws(ws, comp_layout(g->n, nullptr, 0, nullptr), ws_bytes);
    if (s != AD_OK) return s;
    CompLayout L;
    if (comp_layout(g->n, ws, ws_bytes, &L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    TraceScope trace("k_components", stream);
    const int64_t n = g->n;
    *n_comp_host = 0;
    *n_chunks_host = 0;
    int64_t zero[2] = {0, 0};
    if (n == 0) {
        AD_HIP(hipMemcpyAsync(comp_start, zero, sizeof(int64_t), hipMemcpyHostToDevice, stream));
        AD_HIP(hipMemcpyAsync(chunk_start, zero, sizeof(int64_t), hipMemcpyHostToDevice, stream));
        AD_HIP(hipStreamSynchronize(stream));
        return AD_OK;
    }
    s = fill_i32((int32_t *)L.flags, 0, 4, stream);
    if (s != AD_OK) return s;
    s = label_components(g, L.parent, L.flags, stream);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_comp_keys, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, g->row_ptr, L.parent, L.key0, L.val0);
    AD_LAUNCH_CHECK("k_comp_keys");
    size_t tb = L.temp_bytes;
    // keys are at most n (< 2^31): only their low bit_width(n) bits are sorted
    int key_bits = 1;
    while (key_bits < 32 && ((uint64_t)n >> key_bits) != 0) ++key_bits;
    AD_RP(rocprim::radix_sort_pairs(L.temp, tb, L.key0, L.key1, L.val0, L.val1, (size_t)n, 0, key_bits, stream));
    hipLaunchKernelGGL(k_comp_heads, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, L.key1, L.head);
    AD_LAUNCH_CHECK("k_comp_heads");
    tb = L.temp_bytes;
    AD_RP(rocprim::exclusive_scan(L.temp, tb, L.head, L.before, 0u, (size_t)n, rocprim::plus<uint32_t>(), stream));
    uint32_t last[2] = {0, 0};
    AD_HIP(hipMemcpyAsync(&last[0], L.before + (n - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipMemcpyAsync(&last[1], L.head + (n - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipStreamSynchronize(stream));
    const int64_t nc = (int64_t)last[0] + (int64_t)last[1];
    if (nc == 0) {
        hipLaunchKernelGGL(k_comp_fill, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, L.key1, L.val1, L.head, L.before,
                           comp_of, members, comp_start);
        AD_LAUNCH_CHECK("k_comp_fill");
        AD_HIP(hipMemcpyAsync(comp_start, zero, sizeof(int64_t), hipMemcpyHostToDevice, stream));
        AD_HIP(hipMemcpyAsync(chunk_start, zero, sizeof(int64_t), hipMemcpyHostToDevice, stream));
        AD_HIP(hipStreamSynchronize(stream));
        return AD_OK;
    }
    hipLaunchKernelGGL(k_comp_fill, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, L.key1, L.val1, L.head, L.before,
                       comp_of, members, comp_start);
    AD_LAUNCH_CHECK("k_comp_fill");
    hipLaunchKernelGGL(k_comp_chunks, dim3(pgrid(nc + 1)), dim3(PBLOCK), 0, stream, nc, comp_start, L.cnt);
    AD_LAUNCH_CHECK("k_comp_chunks");
    tb = L.temp_bytes;
    AD_RP(rocprim::exclusive_scan(L.temp, tb, L.cnt, chunk_start, (int64_t)0, (size_t)(nc + 1),
                                  rocprim::plus<int64_t>(), stream));
    int64_t nch = 0;
    AD_HIP(hipMemcpyAsync(&nch, chunk_start + nc, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipStreamSynchronize(stream));
    *n_comp_host = nc;
    *n_chunks_host = nch;
    return AD_OK;
}

extern "C" size_t ad_spearman_workspace_size(int64_t n) {
    if (n < 0 || n >= ((int64_t)1 << 31)) return 0;
    return rank_layout(n, nullptr, 0, nullptr);
}

extern "C" ad_status ad_spearman(int64_t n, const double *x, const double *y, double *rho_host, void *ws,
                                 size_t ws_bytes, hipStream_t stream) {
    if (n < 0) return fail(AD_ERR_INVALID_ARG, "negative n");
    if (n >= ((int64_t)1 << 31)) return fail(AD_ERR_UNSUPPORTED, "n must be below 2^31");
    if (n > 0 && (!x || !y)) return fail(AD_ERR_INVALID_ARG, "x or y is NULL");
    if (!rho_host) return fail(AD_ERR_INVALID_ARG, "rho_host is NULL");
    ad_status s = check_ws(ws, rank_layout(n, nullptr, 0, nullptr), ws_bytes);
    if (s != AD_OK) return s;
    RankLayout L;
    if (rank_layout(n, ws, ws_bytes, &L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    *rho_host = 0.0;
    if (n < 2) return AD_OK;
    TraceScope trace("k_spearman", stream);
    const double *src[2] = {x, y};
    int64_t *dst[2] = {L.rx2, L.ry2};
    for (int v = 0; v < 2; ++v) {
        AD_HIP(hipMemcpyAsync(L.keys0, src[v], (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, stream));
        hipLaunchKernelGGL(k_iota, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, L.idx0);
        AD_LAUNCH_CHECK("k_iota");
        size_t tb = L.temp_bytes;
        AD_RP(rocprim::radix_sort_pairs(L.temp, tb, L.keys0, L.keys1, L.idx0, L.idx1, (size_t)n, 0,
                                        8 * (unsigned)sizeof(double), stream));
        hipLaunchKernelGGL(k_mean_ranks, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, L.keys1, L.idx1, dst[v]);
        AD_LAUNCH_CHECK("k_mean_ranks");
    }
    hipLaunchKernelGGL(k_rank_diff2, dim3(PREDUCE_BLOCKS), dim3(PBLOCK), 0, stream, n, L.rx2, L.ry2, L.part);
    AD_LAUNCH_CHECK("k_rank_diff2");
    double part[PREDUCE_BLOCKS];
    AD_HIP(hipMemcpyAsync(part, L.part, sizeof(part), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipStreamSynchronize(stream));
    double sum4 = 0.0;    // sum of (2 p_i)^2
    for (int b = 0; b < PREDUCE_BLOCKS; ++b) sum4 += part[b];
    const double dn = (double)n;
    *rho_host = 1.0 - 6.0 * (sum4 / 4.0) / (dn * (dn * dn - 1.0));
    return AD_OK;
}

// ------------------------------------------------------------ comparison --

namespace ad {

// Degree of every vertex as a double (the score Spearman's formula ranks).
__global__ void k_degree_f64(int64_t n, const int64_t *__restrict__ row_ptr, double *__restrict__ deg) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        deg[i] = (double)(row_ptr[i + 1] - row_ptr[i]);
}

struct CmpLayout {
    int64_t *sub_row_ptr;
    int32_t *sub_col, *sub_eid;
    double *c_o, *c_s, *deg_o, *deg_s;
    void *ws;                 // the largest of the subgraph, properties and Spearman workspaces
    size_t ws_bytes;
};

static size_t cmp_layout(const ad_graph *g, void *ws, size_t ws_bytes, CmpLayout *L) {
    Carver c(ws, ws_bytes);
    const size_t n = (size_t)std::max<int64_t>(1, g->n), nnz = (size_t)std::max<int64_t>(1, 2 * g->m);
    CmpLayout l;
    l.sub_row_ptr = c.take<int64_t>(n + 1);
    l.sub_col = c.take<int32_t>(nnz);
    l.sub_eid = c.take<int32_t>(nnz);
    l.c_o = c.take<double>(n);
    l.c_s = c.take<double>(n);
    l.deg_o = c.take<double>(n);
    l.deg_s = c.take<double>(n);
    ad_graph gu = *g;
    gu.w = nullptr;
    l.ws_bytes = std::max(sub_layout(&gu, nullptr, 0, nullptr),
                          std::max(prop_layout(&gu, nullptr, 0, nullptr), rank_layout(g->n, nullptr, 0, nullptr)));
    l.ws = c.take<char>(l.ws_bytes);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

}  // namespace ad

extern "C" size_t ad_compare_properties_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK || g->n >= ((int64_t)1 << 31) || g->m >= ((int64_t)1 << 31)) return 0;
    return cmp_layout(g, nullptr, 0, nullptr);
}

extern "C" ad_status ad_compare_properties(const ad_graph *g, const uint8_t *keep, double *out_host, void *ws,
                                           size_t ws_bytes, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (!out_host) return fail(AD_ERR_INVALID_ARG, "out_host is NULL");
    if (g->m > 0 && !keep) return fail(AD_ERR_INVALID_ARG, "keep is NULL");
    if (g->n >= ((int64_t)1 << 31) || g->m >= ((int64_t)1 << 31))
        return fail(AD_ERR_UNSUPPORTED, "n and m must be below 2^31");
    s = check_ws(ws, cmp_layout(g, nullptr, 0, nullptr), ws_bytes);
    if (s != AD_OK) return s;
    CmpLayout L;
    if (cmp_layout(g, ws, ws_bytes, &L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    for (int q = 0; q < AD_CMP_FIELDS; ++q) out_host[q] = 0.0;
    const int64_t n = g->n;
    ad_graph go = *g;             // the properties read the structure only
    go.w = nullptr;
    go.col_orig = nullptr;
    int64_t ms = 0;
    s = ad_subgraph(&go, keep, L.sub_row_ptr, L.sub_col, nullptr, L.sub_eid, nullptr, &ms, L.ws, L.ws_bytes, stream);
    if (s != AD_OK) return s;
    ad_graph gs = go;
    gs.m = ms;
    gs.row_ptr = L.sub_row_ptr;
    gs.col = L.sub_col;
    gs.eid = L.sub_eid;
    double sum_o[2] = {0.0, 0.0}, sum_s[2] = {0.0, 0.0};
    s = ad_graph_properties(&go, nullptr, L.c_o, nullptr, sum_o, L.ws, L.ws_bytes, stream);
    if (s != AD_OK) return s;
    s = ad_graph_properties(&gs, nullptr, L.c_s, nullptr, sum_s, L.ws, L.ws_bytes, stream);
    if (s != AD_OK) return s;
    double rho_deg = 0.0, rho_c = 0.0;
    if (n > 0) {
        hipLaunchKernelGGL(k_degree_f64, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, go.row_ptr, L.deg_o);
        AD_LAUNCH_CHECK("k_degree_f64");
        hipLaunchKernelGGL(k_degree_f64, dim3(pgrid(n)), dim3(PBLOCK), 0, stream, n, gs.row_ptr, L.deg_s);
        AD_LAUNCH_CHECK("k_degree_f64");
        s = ad_spearman(n, L.deg_o, L.deg_s, &rho_deg, L.ws, L.ws_bytes, stream);
        if (s != AD_OK) return s;
        s = ad_spearman(n, L.c_o, L.c_s, &rho_c, L.ws, L.ws_bytes, stream);
        if (s != AD_OK) return s;
    }
    out_host[0] = (double)ms;
    out_host[1] = sum_o[0];
    out_host[2] = sum_s[0];
    out_host[3] = sum_o[1];
    out_host[4] = sum_s[1];
    out_host[5] = sum_o[1] > 0.0 ? sum_s[1] / sum_o[1] : 0.0;
    out_host[6] = rho_deg;
    out_host[7] = rho_c;
    return AD_OK;
}
