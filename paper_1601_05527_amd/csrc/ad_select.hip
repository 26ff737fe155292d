// ad_select.hip -- edge distances (Algorithm 1, last steps), per-vertex
// ranking and selection (Algorithm 3) and the retention fit (Section 6.2).
//
// Distances: each upper entry (i, j), j > i, is handled by C lanes that
// hold VEC consecutive values each; the squared scaled differences are
// summed per lane in order and the lanes combined in a fixed tree, so each
// distance has one summation order (the adjoint reproduces it).
//
// Ranking: every stored entry (i, j) gets its position in row i's order
// (rho ascending for LOCAL, descending for GLOBAL; ties by orig_id[j]).
// Keys are unique inside a row, so ranks are well defined.  Rows of degree
// <= 64 are packed several to a wave, one entry per lane, and rank by
// counting through shuffles.  Rows of degree <= 8192 sort in LDS, one
// workgroup per row sized to the row: a radix sort of the distance bits, or,
// for a caller's own 64-bit keys, counting inside one wave (<= 512) and a
// bitonic network (<= 8192).  Longer rows are cut into buckets by a sorted
// sample and rank inside their bucket.  FP64 distances above 64 count
// against keys read from memory.
//
// Selection at fixed e: entry (i, j) selects its edge when rank < budget[d_i];
// keep[e] = 1 is written by any selecting entry (all writers store the same
// value).  Fit: with per-vertex budgets floor(d^e) non-decreasing in e, edge
// e is kept exactly for e >= T_e, T_e the smaller of the two endpoints'
// thresholds; the bisection of Section 6.2 returns the smallest point of its
// 2^-40 grid at or above the K-th smallest T_e (K = fewest kept edges that
// meet the target).  The grid point is located from log-ratio estimates of
// the thresholds by a radix select and then confirmed exactly with budget
// tables built on the host with the C library's pow, as the bisection would
// evaluate them.
#include "ad_internal.h"

#include <math.h>

#include <cmath>

#include <algorithm>
#include <mutex>
#include <thread>
#include <vector>

#include <rocprim/block/block_radix_sort.hpp>

namespace ad {

constexpr int SBLOCK = 256;
constexpr int NCLASS = 8;            // degree classes above 64 (see CLASS_LO)
constexpr int HUB_CLASS = 7;         // FP32 rows of class >= HUB_CLASS take the bucket partition
constexpr int SORT_CAP = 8192;       // longest FP32 row ranked in one wave or one LDS sort
constexpr int DIST_UNROLL = 8;       // entries per slot in flight in the distance pass (FP32 vectors)

// Entries per slot in flight: FP64 vectors hold twice the registers per entry.
template <typename Tx>
constexpr int dist_unroll() { return sizeof(Tx) == 8 ? DIST_UNROLL / 2 : DIST_UNROLL; }

// ---------------------------------------------------------------- distance --

// The value of a butterfly partner at distance off within rows of 16 lanes,
// through DPP: quad permutations for off = 1 and 2 (lane ^ off), the
// half-row mirror for 4 and the row mirror for 8.  The mirrors pair a lane
// with a lane of the other half of its block of 2 * off lanes; after the
// earlier butterfly steps every lane of that half holds the same partial,
// so the sums equal those of lane ^ off.
template <int CTRL>
__device__ __forceinline__ float dpp_take(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_take(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
template <typename A>
__device__ __forceinline__ A butterfly_partner(A v, int off) {
    switch (off) {
        case 1: return dpp_take<0xB1>(v);      // quad_perm [1, 0, 3, 2]
        case 2: return dpp_take<0x4E>(v);      // quad_perm [2, 3, 0, 1]
        case 4: return dpp_take<0x141>(v);     // row_half_mirror
        case 8: return dpp_take<0x140>(v);     // row_mirror
        default: return __shfl_xor(v, off, WAVE);
    }
}

// Sum over the C lanes of one entry's group (lanes base .. base + C - 1):
// a butterfly when C is a power of two, ((c0 + c1) + (c2 + c3)) ..., else
// c0 + c1 + ... in order.  Every lane of the group gets the same value.
template <typename A>
__device__ __forceinline__ A group_sum(A v, int C, int base) {
    if (C == 4) {
        v += dpp_take<0xB1>(v);
        return v + dpp_take<0x4E>(v);
    }
    if (C == 2) return v + dpp_take<0xB1>(v);
    if ((C & (C - 1)) == 0) {
        for (int off = 1; off < C; off <<= 1) v += butterfly_partner(v, off);
        return v;
    }
    A t = shfl(v, base);
    for (int c = 1; c < C; ++c) t += shfl(v, base + c);
    return t;
}

// rho for the upper entries (j > i) of the entries beg .. end - 1 of `row`
// (one lane group of C lanes per slot, SPR slots, U entries per slot in
// flight).  Lane chunk c sums ((x_i - x_j) * inv)^2 over its VEC values in
// order; group_sum adds the chunks.  `len` is the wave's common trip bound.
// With ALL, every entry p of the span gets its value in rho_ent[p] (the
// entry order of the CSR), and the upper ones also in rho[eid[p]]: an edge's
// two entries get equal values, since x_j - x_i = -(x_i - x_j) exactly and
// both are summed in the same order.
template <typename Tx, typename Tr, int VEC, int U, bool ALL = false>
__device__ __forceinline__ void dist_span(const int32_t *__restrict__ col, const int32_t *__restrict__ eid,
                                          const Tx *__restrict__ x, const double *__restrict__ minmax,
                                          Tr *__restrict__ rho, Tr *__restrict__ rho_ent, int R, int C, int SPR,
                                          int slot, int chunk, int base, bool active, int64_t row, int64_t beg,
                                          int64_t end, int64_t len, int64_t gb) {
    typedef typename acc_of<Tx>::type A;
    const int off = chunk * VEC;
    A xi[VEC], iv[VEC];
    if (active) {
        load_vec<VEC>(x + row * R + off, xi);
    } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) xi[q] = (A)0;
    }
    // 1 / (max - min) of this lane's vectors, for the graph of the row
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
        const double lo = minmax[gb + off + q], hi = minmax[gb + R + off + q];
        iv[q] = (hi > lo) ? (A)(1.0 / (hi - lo)) : (A)0;
    }
    for (int64_t k0 = slot; k0 < len; k0 += (int64_t)U * SPR) {
        int32_t jj[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = beg + k0 + (int64_t)u * SPR;
            ok[u] = active && p < end;
            jj[u] = ok[u] ? col[p] : 0;
            if (!ALL) ok[u] = ok[u] && jj[u] > row;
        }
        A part[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            A xj[VEC];
            if (ok[u]) {
                load_vec<VEC>(x + (int64_t)jj[u] * R + off, xj);
            } else {
#pragma unroll
                for (int q = 0; q < VEC; ++q) xj[q] = xi[q];
            }
            A acc = (A)0;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const A d = (xi[q] - xj[q]) * iv[q];
                acc = fma(d, d, acc);
            }
            part[u] = acc;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const A tot = group_sum(part[u], C, base);
            if (ok[u] && chunk == 0) {
                const int64_t p = beg + k0 + (int64_t)u * SPR;
                const Tr r = (Tr)sqrt(tot);
                if (ALL) rho_ent[p] = r;
                if (!ALL || jj[u] > row) rho[eid[p]] = r;
            }
        }
    }
}

// Entries per wave work item of a long row in the distance pass.
constexpr int64_t DIST_SEG = 4096;

// rho for every edge, visited from its upper entry (j > i; the suffix of the
// row after upper_start); with ALL, from both of its entries (whole rows),
// every entry's value also in rho_ent in CSR order.  The first hub_blocks workgroups take the rows
// longer than hub_d, their upper suffix cut into work items of DIST_SEG
// entries (row h of the hub list, segment s < hub_segs; items past the row's
// end are skipped), one wave per item.  The other waves walk the launch plan (first row, rows in the tile,
// log2 rows per wave) as the sweep does, with SPRW / rpw slots per row.
// Every edge's value is computed by the same lane arithmetic on either path.
template <typename Tx, typename Tr, int VEC, int U, bool ALL>
__global__ __launch_bounds__(SBLOCK) void k_edge_dist(
    int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const Tx *__restrict__ x, const double *__restrict__ minmax,
    Tr *__restrict__ rho, Tr *__restrict__ rho_ent, int R, int C, int SPRW, int64_t hub_d, int hub_blocks, int64_t hub_segs,
    const int32_t *__restrict__ hub_list, const unsigned int *__restrict__ hub_count,
    const long long *__restrict__ plan, const unsigned int *__restrict__ plan_count,
    const unsigned int *__restrict__ splits, int xcd_groups, const int32_t *__restrict__ row_graph) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    if ((int)blockIdx.x < hub_blocks) {
        const int group = C * SPRW;
        const int slot = lane / C;
        const int chunk = lane - slot * C;
        const bool active = lane < group;
        const unsigned long long items = (unsigned long long)(*hub_count) * (unsigned long long)hub_segs;
        const unsigned long long stride = (unsigned long long)hub_blocks * (SBLOCK / WAVE);
        for (unsigned long long it = (unsigned long long)blockIdx.x * (SBLOCK / WAVE) + wave; it < items;
             it += stride) {
            const int64_t row = hub_list[it / hub_segs];
            const int64_t re = row_ptr[row + 1];
            const int64_t rb = ALL ? row_ptr[row] : upper_start(col, row_ptr[row], re, row);
            const int64_t b0 = rb + (int64_t)(it % hub_segs) * DIST_SEG;
            if (b0 >= re) continue;                       // uniform across the wave
            const int64_t e0 = min(re, b0 + DIST_SEG);
            const int64_t gb = (int64_t)(row_graph ? row_graph[row] : 0) * 2 * R;
            dist_span<Tx, Tr, VEC, U, ALL>(col, eid, x, minmax, rho, rho_ent, R, C, SPRW, slot, chunk,
                                           lane - chunk, active, row, b0, e0, e0 - b0, gb);
        }
        return;
    }
    const PlanWalk pw = plan_walk(*plan_count, splits, xcd_groups, blockIdx.x - hub_blocks, gridDim.x - hub_blocks,
                                  wave, SBLOCK / WAVE);
    for (unsigned long long pi = pw.first; pi < pw.end; pi += pw.stride) {
        const long long pe = plan[pi];
        const int64_t row0 = pe >> 16;
        const int nrows = (int)((pe >> 8) & 0xff);     // rows of this entry inside its tile
        const int RPW = 1 << (int)(pe & 0xff);
        const int SPR = SPRW / RPW;
        const int group = C * SPR;
        const int rw = lane / group;
        const int sub = lane - rw * group;
        const int slot = sub / C;
        const int chunk = sub - slot * C;
        const int64_t row = row0 + rw;
        bool active = rw < nrows;
        int64_t beg = 0, end = 0;
        if (active) {
            beg = row_ptr[row];
            end = row_ptr[row + 1];
            if (end - beg > hub_d) active = false;        // taken by the hub workgroups
            else if (!ALL) beg = upper_start(col, beg, end, row);
        }
        if (!active) beg = end = 0;
        // uniform trip count across the wave: the longest row of the wave
        int64_t len = end - beg;
        for (int d = WAVE / 2; d >= 1; d >>= 1) len = max(len, shfl_down(len, d));
        len = shfl(len, 0);
        const int64_t gb = (int64_t)(row_graph ? row_graph[row0] : 0) * 2 * R;
        dist_span<Tx, Tr, VEC, U, ALL>(col, eid, x, minmax, rho, rho_ent, R, C, SPR, slot, chunk, lane - chunk,
                                       active, row, beg, end, len, gb);
    }
}

// ------------------------------------------------------------ normalization --

// f_i = the weighted degree s_i in FP64 (or the degree d_i): one wave per row.
__global__ __launch_bounds__(SBLOCK) void k_vertex_weight(int64_t n, const int64_t *__restrict__ row_ptr,
                                                         const float *__restrict__ w, int by_strength,
                                                         double *__restrict__ f) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (SBLOCK / WAVE);
    for (int64_t i = (int64_t)blockIdx.x * (SBLOCK / WAVE) + (threadIdx.x >> 6); i < n; i += nw) {
        const int64_t beg = row_ptr[i], end = row_ptr[i + 1];
        if (!by_strength || !w) {
            if (lane == 0) f[i] = (double)(end - beg);
            continue;
        }
        double acc = 0.0;
        for (int64_t p = beg + lane; p < end; p += WAVE) acc += (double)w[p];
        for (int o = WAVE / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
        if (lane == 0) f[i] = acc;
    }
}

// Row of entry p within rows [lo, hi] (row_ptr[lo] <= p < row_ptr[hi + 1]).
__device__ __forceinline__ int64_t row_of(const int64_t *__restrict__ row_ptr, int64_t lo, int64_t hi, int64_t p) {
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

constexpr int64_t NORM_CHUNK = 4096;     // stored entries per wave work item

// out_e = sqrt(rho_e^2 + eps) * sqrt(f_i f_j), from each edge's upper entry
// (j > i).  Waves take chunks of NORM_CHUNK consecutive stored entries; the
// rows a chunk spans are found by binary search over row_ptr.
template <typename Tr>
__global__ __launch_bounds__(SBLOCK) void k_normalize(int64_t n, int64_t nnz, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const int32_t *__restrict__ eid,
                                                     const double *__restrict__ f, const Tr *rho, double eps,
                                                     Tr *out) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nchunks = ceil_div_dev(nnz, NORM_CHUNK);
    const int64_t nw = (int64_t)gridDim.x * (SBLOCK / WAVE);
    for (int64_t c = (int64_t)blockIdx.x * (SBLOCK / WAVE) + (threadIdx.x >> 6); c < nchunks; c += nw) {
        const int64_t p0 = c * NORM_CHUNK, p1 = min(nnz, p0 + NORM_CHUNK);
        int64_t r = 0;
        if (lane == 0) r = row_of(row_ptr, 0, n - 1, p0);
        if (lane == 1) r = row_of(row_ptr, 0, n - 1, p1 - 1);
        const int64_t r0 = __shfl(r, 0, WAVE), r1 = __shfl(r, 1, WAVE);
        for (int64_t p = p0 + lane; p < p1; p += WAVE) {
            const int64_t i = row_of(row_ptr, r0, r1, p);
            const int64_t j = col[p];
            if (j <= i) continue;
            const int32_t e = eid[p];
            const double v = (double)rho[e];
            out[e] = (Tr)(sqrt(v * v + eps) * sqrt(f[i] * f[j]));
        }
    }
}

// ------------------------------------------------------------------ ranking --

enum { MODE_FIXED = 0, MODE_REC = 1, MODE_REC_L = 2, MODE_REC_G = 3 };

// Original id of the neighbour of entry p (tie-break key): the per-entry
// copy when the graph carries one, else a gather through orig_id.
__device__ __forceinline__ int32_t nbr_id(int64_t p, int32_t j, const int32_t *__restrict__ col_orig,
                                          const int32_t *__restrict__ orig_id) {
    return col_orig ? col_orig[p] : (orig_id ? orig_id[j] : j);
}

// Where ranks go.  MODE_FIXED marks keep[e] when rank < budget[d] (with
// `both`, the LOCAL rank against (budget, keep) and the GLOBAL rank against
// (budget2, keep2); otherwise the rank of `orient`).  MODE_REC stores the
// side record {d, first rank, second rank, 0} at recs[2e + (row > j)]: with
// `both` the LOCAL and the GLOBAL rank, otherwise the rank of `orient` in
// both places; one 16-byte store per entry.  The bucketed rows rank one
// orientation per pass: MODE_REC_L stores {d, rank} in words 0 and 1,
// MODE_REC_G stores d and the rank in words 0 and 2.
struct Emit {
    int mode, orient, both;
    const int32_t *budget, *budget2;
    uint8_t *keep, *keep2;
    uint4 *recs;
};

// Order-preserving 64-bit key of (rho, orig_id) for the row's order
// (FP32 distances); the GLOBAL key is the LOCAL key with the rho half
// inverted, i.e. key ^ KEY_FLIP.
constexpr unsigned long long KEY_FLIP = 0xffffffff00000000ull;
__device__ __forceinline__ unsigned long long sort_key(float r, int32_t id, int orient) {
    uint32_t b = __float_as_uint(r);                 // rho >= 0: bits are monotone
    if (orient == AD_GLOBAL) b = ~b;
    return ((unsigned long long)b << 32) | (unsigned long long)(uint32_t)id;
}

// Key of CSR entry p (edge e, neighbour id `id`): the caller's own 64-bit
// key when `keys` is given (distinct within each row and below ~0; the row
// order is then ascending keys), else the distance key above.
__device__ __forceinline__ unsigned long long entry_key(const unsigned long long *__restrict__ keys,
                                                        const float *__restrict__ rho, int64_t p, int32_t e,
                                                        int32_t id, int orient) {
    return keys ? keys[p] : sort_key(rho[e], id, orient);
}

// Rank of an entry in its row of d entries, in both orders of Algorithm 3:
// LOCAL (rho ascending) and GLOBAL (rho descending), ties by neighbour id
// ascending in both.  With lt = #{rho' < rho}, eq = #{rho' == rho} (itself
// included) and eqlt = #{rho' == rho, id' < id}:
//   rank_local = lt + eqlt,   rank_global = (d - lt - eq) + eqlt.
__device__ __forceinline__ void emit_ranks(const Emit &em, int64_t row, int32_t j, int32_t e, int64_t d,
                                           int64_t rank_local, int64_t rank_global) {
    const int64_t rank_o = em.orient == AD_LOCAL ? rank_local : rank_global;
    if (em.mode == MODE_FIXED) {
        if (em.both) {
            if (rank_local < em.budget[d]) em.keep[e] = 1;
            if (rank_global < em.budget2[d]) em.keep2[e] = 1;
        } else if (rank_o < em.budget[d]) {
            em.keep[e] = 1;
        }
        return;
    }
    uint4 *r = em.recs + 2 * (int64_t)e + (row > j ? 1 : 0);
    if (em.mode == MODE_REC) {
        *r = make_uint4((uint32_t)d, (uint32_t)(em.both ? rank_local : rank_o),
                        (uint32_t)(em.both ? rank_global : rank_o), 0u);
    } else if (em.mode == MODE_REC_L) {
        *reinterpret_cast<uint2 *>(r) = make_uint2((uint32_t)d, (uint32_t)rank_o);
    } else {
        reinterpret_cast<uint32_t *>(r)[0] = (uint32_t)d;
        reinterpret_cast<uint32_t *>(r)[2] = (uint32_t)rank_o;
    }
}

// Rows of degree <= 64, packed: a wave takes consecutive rows whose entries
// fit in its 64 lanes (plan entry: first row << 8 | number of rows), one
// entry per lane; each lane counts the entries of its own row that come
// before it, stepping through its row's lanes (as many steps as the wave's
// longest row).
constexpr int RANK_TILE = 64;

template <typename Tr>
__global__ __launch_bounds__(SBLOCK) void k_rank_packed(
    const long long *__restrict__ plan, const unsigned int *__restrict__ plan_count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id,
    const int32_t *__restrict__ col_orig, const Tr *__restrict__ rho,
    const unsigned long long *__restrict__ keys, Emit em, const float *__restrict__ rho_ent) {
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned int np = *plan_count;
    const unsigned int nwaves = gridDim.x * (SBLOCK / WAVE);
    for (unsigned int pi = blockIdx.x * (SBLOCK / WAVE) + (threadIdx.x >> 6); pi < np; pi += nwaves) {
        const long long pe = plan[pi];
        const int64_t first = pe >> 8;
        const int nrows = (int)(pe & 0xff);
        const int64_t e0 = row_ptr[first];
        const int64_t e1 = row_ptr[first + nrows];
        const int cnt = (int)(e1 - e0);
        // start of row `lane` within the wave's entries (non-decreasing in lane)
        const int st = lane < nrows ? (int)(row_ptr[first + lane] - e0) : cnt;
        const int64_t e = e0 + lane;
        const bool on = lane < cnt;
        // my row: the last row of the wave that starts at or before my entry
        // (binary search over the row starts; empty rows share the next start)
        int k = 0;
        for (int step = WAVE / 2; step >= 1; step >>= 1) {
            const int cand = k + step;
            const int sc = shfl(st, cand < WAVE ? cand : WAVE - 1);
            if (cand < nrows && sc <= lane) k = cand;
        }
        const int s0 = shfl(st, k);
        const int s1 = shfl(st, k + 1 < WAVE ? k + 1 : WAVE - 1);
        const int d = on ? ((k + 1 < nrows) ? s1 : cnt) - s0 : 0;
        Tr my_rho = (Tr)0;
        int32_t my_id = 0, my_j = 0, my_e = 0;
        if (on) {
            my_j = col[e];
            my_e = eid[e];
            if (!keys) my_rho = rho_ent ? (Tr)rho_ent[e] : rho[my_e];
            my_id = nbr_id(e, my_j, col_orig, orig_id);
        }
        // every lane walks its own row: as many steps as the wave's longest row
        int dmax = d;
        for (int o = WAVE / 2; o >= 1; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o, WAVE));
        if (sizeof(Tr) == 4 && !keys) {
            // FP32 distances: count on the 32-bit distance bits (rho >= 0, so
            // the bits order as the values): lt = #{rho' < rho}, eq = #{rho' ==
            // rho}; only when some row of the wave has a tie, a second pass
            // counts the tied neighbours with smaller ids (eqlt)
            const uint32_t mine = __float_as_uint((float)my_rho);
            int lt = 0, eq = 0, eqlt = 0;
            for (int t = 0; t < dmax; ++t) {
                const uint32_t kb = (uint32_t)shfl((int)mine, min(s0 + t, WAVE - 1));
                if (t < d) {
                    lt += (kb < mine) ? 1 : 0;
                    eq += (kb == mine) ? 1 : 0;
                }
            }
            if (__any(on && eq > 1)) {                 // uniform across the wave
                for (int t = 0; t < dmax; ++t) {
                    const int src = min(s0 + t, WAVE - 1);
                    const uint32_t kb = (uint32_t)shfl((int)mine, src);
                    const int32_t id = shfl(my_id, src);
                    if (t < d) eqlt += (kb == mine && id < my_id) ? 1 : 0;
                }
            }
            if (on) emit_ranks(em, first + k, my_j, my_e, d, lt + eqlt, d - lt - eq + eqlt);
        } else if constexpr (sizeof(Tr) == 4) {
            // caller keys: the row orders are those of 64-bit keys
            const unsigned long long key =
                keys ? (on ? keys[e] : 0ull) : sort_key((float)my_rho, my_id, em.both ? AD_LOCAL : em.orient);
            const unsigned long long keyg = key ^ KEY_FLIP;
            int r1 = 0, r2 = 0;
            if (em.both) {
                for (int t = 0; t < dmax; ++t) {
                    const unsigned long long k = shfl(key, min(s0 + t, WAVE - 1));
                    if (t < d) {
                        r1 += (k < key) ? 1 : 0;
                        r2 += ((k ^ KEY_FLIP) < keyg) ? 1 : 0;
                    }
                }
            } else {
                for (int t = 0; t < dmax; ++t) {
                    const unsigned long long k = shfl(key, min(s0 + t, WAVE - 1));
                    if (t < d) r1 += (k < key) ? 1 : 0;
                }
                r2 = r1;
            }
            if (on) emit_ranks(em, first + k, my_j, my_e, d, r1, r2);
        } else {
            int lt = 0, eq = 0, eqlt = 0;
            for (int t = 0; t < dmax; ++t) {
                const int src = min(s0 + t, WAVE - 1);
                const Tr r = shfl(my_rho, src);
                const int32_t id = shfl(my_id, src);
                if (t < d) {
                    lt += (r < my_rho) ? 1 : 0;
                    eq += (r == my_rho) ? 1 : 0;
                    eqlt += (r == my_rho && id < my_id) ? 1 : 0;
                }
            }
            if (on) emit_ranks(em, first + k, my_j, my_e, d, lt + eqlt, d - lt - eq + eqlt);
        }
    }
}

// Packing of rows with 1 <= degree <= 64 per tile of RANK_TILE rows: a wave
// holds consecutive such rows (isolated rows ride along) while their entries
// fit in 64 lanes; a longer row closes the wave.  fill == 0 counts waves per
// tile, fill == 1 writes the plan entries at the scanned offsets.
__global__ void k_rank_plan(int64_t n, const int64_t *__restrict__ row_ptr, int fill,
                            unsigned int *__restrict__ tile_waves, long long *__restrict__ plan) {
    const int64_t ntiles = ceil_div_dev(n, RANK_TILE);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r0 = t * RANK_TILE, r1 = min(n, r0 + RANK_TILE);
        unsigned int waves = 0;
        unsigned int o = fill ? tile_waves[t] : 0;
        int64_t first = -1;
        int cur = 0, nr = 0;
        for (int64_t r = r0; r < r1; ++r) {
            const int64_t d = row_ptr[r + 1] - row_ptr[r];
            const bool small = d <= WAVE;
            if (first >= 0 && (!small || cur + d > WAVE)) {
                if (fill && cur > 0) plan[o++] = ((long long)first << 8) | nr;
                if (cur > 0) ++waves;
                first = -1;
            }
            if (!small) continue;
            if (first < 0) {
                first = r;
                cur = 0;
                nr = 0;
            }
            cur += (int)d;
            ++nr;
        }
        if (first >= 0 && cur > 0) {
            if (fill) plan[o++] = ((long long)first << 8) | nr;
            ++waves;
        }
        if (!fill) tile_waves[t] = waves;
    }
}

// Rows with degree > 64 into per-class lists (class c holds rows with
// lo[c] < d <= lo[c + 1]); one pass, atomic slots per class.
struct ClassBounds {
    int64_t lo[NCLASS + 1];
    int64_t off[NCLASS];
};

__global__ void k_classify(int64_t n, const int64_t *__restrict__ row_ptr, ClassBounds cb,
                           int32_t *__restrict__ lists, unsigned int *__restrict__ counts) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n_pad = ceil_div_dev(n, stride) * stride;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += stride) {
        int c = -1;
        if (i < n) {
            const int64_t d = row_ptr[i + 1] - row_ptr[i];
            if (d > cb.lo[0]) {
                c = 0;
                while (c + 1 < NCLASS && d > cb.lo[c + 1]) ++c;
            }
        }
        if (!__any(c >= 0)) continue;       // uniform across the wave
        for (int k = 0; k < NCLASS; ++k) {
            const unsigned int at = wave_append(c == k, &counts[k]);
            if (c == k) lists[cb.off[k] + at] = (int32_t)i;
        }
    }
}


// Listed rows with 32 * KPL < d <= 64 * KPL (FP32 distances): one wave per row,
// KPL keys per lane; each key's rank counts the row's smaller keys (and,
// for both orders, the smaller GLOBAL keys), broadcast one lane at a time.
template <int KPL>
__global__ __launch_bounds__(SBLOCK) void k_rank_wave(
    const int32_t *__restrict__ list, const unsigned int *__restrict__ count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id,
    const int32_t *__restrict__ col_orig, const float *__restrict__ rho,
    const unsigned long long *__restrict__ keys, Emit em) {
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned int nr = *count;
    const unsigned int waves = gridDim.x * (SBLOCK / WAVE);
    const int orient = em.both ? AD_LOCAL : em.orient;
    for (unsigned int h = blockIdx.x * (SBLOCK / WAVE) + (threadIdx.x >> 6); h < nr; h += waves) {
        const int64_t row = list[h];
        const int64_t beg = row_ptr[row];
        const int d = (int)(row_ptr[row + 1] - beg);
        unsigned long long key[KPL];
        int32_t jj[KPL], ee[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
            const int q = t * WAVE + lane;
            if (q < d) {
                jj[t] = col[beg + q];
                ee[t] = eid[beg + q];
                key[t] = entry_key(keys, rho, beg + q, ee[t], nbr_id(beg + q, jj[t], col_orig, orig_id), orient);
            } else {
                jj[t] = 0;
                ee[t] = 0;
                key[t] = ~0ull;
            }
        }
        int r1[KPL], r2[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) r1[t] = r2[t] = 0;
        if (em.both) {
            unsigned long long keyg[KPL];
#pragma unroll
            for (int t = 0; t < KPL; ++t) keyg[t] = key[t] ^ KEY_FLIP;
#pragma unroll
            for (int ts = 0; ts < KPL; ++ts) {
                if (ts * WAVE >= d) break;                 // uniform across the wave
                const int lim = min(WAVE, d - ts * WAVE);
                for (int src = 0; src < lim; ++src) {
                    const unsigned long long k = shfl(key[ts], src);
                    const unsigned long long kg = k ^ KEY_FLIP;
#pragma unroll
                    for (int t = 0; t < KPL; ++t) {
                        r1[t] += (k < key[t]) ? 1 : 0;
                        r2[t] += (kg < keyg[t]) ? 1 : 0;
                    }
                }
            }
        } else {
#pragma unroll
            for (int ts = 0; ts < KPL; ++ts) {
                if (ts * WAVE >= d) break;
                const int lim = min(WAVE, d - ts * WAVE);
                for (int src = 0; src < lim; ++src) {
                    const unsigned long long k = shfl(key[ts], src);
#pragma unroll
                    for (int t = 0; t < KPL; ++t) r1[t] += (k < key[t]) ? 1 : 0;
                }
            }
#pragma unroll
            for (int t = 0; t < KPL; ++t) r2[t] = r1[t];
        }
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
            const int q = t * WAVE + lane;
            if (q < d) emit_ranks(em, row, jj[t], ee[t], d, r1[t], r2[t]);
        }
    }
}

// Listed rows with P_MAX/2 < d <= P_MAX (FP32 distances): bitonic sort in
// LDS by a TB-thread workgroup.
template <int P_MAX, int TB>
__global__ __launch_bounds__(TB) void k_rank_bitonic(
    const int32_t *__restrict__ list, const unsigned int *__restrict__ count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id,
    const int32_t *__restrict__ col_orig, const float *__restrict__ rho,
    const unsigned long long *__restrict__ keys, Emit em) {
    __shared__ unsigned long long key[P_MAX];
    __shared__ uint16_t idx[P_MAX];
    const unsigned int nr = *count;
    const int orient = em.both ? AD_LOCAL : em.orient;
    for (unsigned int h = blockIdx.x; h < nr; h += gridDim.x) {
        const int64_t row = list[h];
        const int64_t beg = row_ptr[row];
        const int d = (int)(row_ptr[row + 1] - beg);
        int P = 1;
        while (P < d) P <<= 1;
        for (int t = threadIdx.x; t < P; t += TB) {
            if (t < d) {
                int32_t j = col[beg + t];
                key[t] = entry_key(keys, rho, beg + t, eid[beg + t], nbr_id(beg + t, j, col_orig, orig_id), orient);
            } else {
                key[t] = ~0ull;
            }
            idx[t] = (uint16_t)t;
        }
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = threadIdx.x; t < (P >> 1); t += TB) {
                    int a = 2 * t - (t & (stride - 1));
                    int b = a + stride;
                    bool up = ((a & size) == 0);
                    unsigned long long ka = key[a], kb = key[b];
                    if ((ka > kb) == up) {
                        key[a] = kb;
                        key[b] = ka;
                        uint16_t ia = idx[a];
                        idx[a] = idx[b];
                        idx[b] = ia;
                    }
                }
                __syncthreads();
            }
        }
        for (int t = threadIdx.x; t < d; t += TB) {
            const int64_t p = beg + idx[t];
            int64_t rank_global = t;
            if (em.both) {
                // sorted LOCAL: the run [a, b) of equal rho holds t; GLOBAL puts the
                // d - b larger distances first, then the run in the same id order
                const unsigned long long hb = key[t] >> 32;
                int a = 0, hi = d;
                while (a < hi) {
                    const int mid = (a + hi) >> 1;
                    if ((key[mid] >> 32) < hb) a = mid + 1;
                    else hi = mid;
                }
                int b = a;
                hi = d;
                while (b < hi) {
                    const int mid = (b + hi) >> 1;
                    if ((key[mid] >> 32) <= hb) b = mid + 1;
                    else hi = mid;
                }
                rank_global = (int64_t)(d - b) + (t - a);
            }
            emit_ranks(em, row, col[p], eid[p], d, t, rank_global);
        }
        __syncthreads();
    }
}

// Listed rows with d <= TB * IPT (FP32 distances, no caller keys): one
// workgroup per row sorts the row's distance bits (rho >= 0, so the bits
// order as the values) with the entry's place in the row as payload, by a
// block radix sort in LDS (8-bit digits, four passes).  A distance shared by
// several entries forms a run [a, b) of the sorted row; its entries take
// their order inside the run from the neighbour ids (distinct within a row),
// counted against the run.  LOCAL rank = a + place in run, GLOBAL rank =
// (d - b) + place in run, as Algorithm 3 orders the row both ways.
// Largest sort key of a real entry: padding (0xffffffff) must sort after
// every entry, so the one bit pattern that could equal it (a negative NaN)
// is clamped below it; valid distances (>= 0) are far below.
constexpr uint32_t KEY_LAST = 0xfffffffeu;

template <int TB, int IPT>
__global__ __launch_bounds__(TB) void k_rank_radix(
    const int32_t *__restrict__ list, const unsigned int *__restrict__ count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id,
    const int32_t *__restrict__ col_orig, const float *__restrict__ rho, const float *__restrict__ rho_ent, Emit em,
    int slice, int nslices) {
    constexpr int P = TB * IPT;
    static_assert(P <= 65536, "places are 16-bit");
    using Sorter = rocprim::block_radix_sort<uint32_t, TB, IPT, uint16_t>;
    __shared__ union {
        typename Sorter::storage_type sort;
        struct {
            uint32_t key[P];
            uint32_t rank[P];                        // both ranks of entry q of the row, 16 bits each
            uint16_t place[P];
        } row;
    } sh;
    const unsigned int nr = *count;
    // this launch takes rows slice, slice + nslices, ... of the list
    for (unsigned int h = blockIdx.x * nslices + slice; h < nr; h += gridDim.x * nslices) {
        const int64_t row = list[h];
        const int64_t beg = row_ptr[row];
        const int d = (int)(row_ptr[row + 1] - beg);
        // striped load (item s of thread t is entry s * TB + t); places past d
        // carry the largest key and sort last
        uint32_t k[IPT];
        uint16_t v[IPT];
        if (rho_ent) {                               // distances in entry order: contiguous
#pragma unroll
            for (int s = 0; s < IPT; ++s) {
                const int q = s * TB + (int)threadIdx.x;
                k[s] = q < d ? min(__float_as_uint(rho_ent[beg + q]), KEY_LAST) : 0xffffffffu;
                v[s] = (uint16_t)q;
            }
        } else {
            int32_t e[IPT];
#pragma unroll
            for (int s = 0; s < IPT; ++s) {
                const int q = s * TB + (int)threadIdx.x;
                e[s] = q < d ? eid[beg + q] : 0;
            }
#pragma unroll
            for (int s = 0; s < IPT; ++s) {
                const int q = s * TB + (int)threadIdx.x;
                k[s] = q < d ? min(__float_as_uint(rho[e[s]]), KEY_LAST) : 0xffffffffu;
                v[s] = (uint16_t)q;
            }
        }
        Sorter().sort(k, v, sh.sort);                // blocked: thread t holds sorted places t * IPT + s
        __syncthreads();
#pragma unroll
        for (int s = 0; s < IPT; ++s) {
            const int q = (int)threadIdx.x * IPT + s;
            sh.row.key[q] = k[s];
            sh.row.place[q] = v[s];
        }
        __syncthreads();
        // both ranks of sorted place q (each below d <= 65536: 16 bits each),
        // stored at the entry's place in the row, so that the records are
        // written by consecutive entries of the row (its upper entries hold
        // consecutive edge ids)
#pragma unroll
        for (int s = 0; s < IPT; ++s) {
            const int q = (int)threadIdx.x * IPT + s;
            if (q >= d) continue;
            uint32_t rk = (uint32_t)q | ((uint32_t)(d - 1 - q) << 16);
            const uint32_t key = k[s];
            const bool tie = (q > 0 && sh.row.key[q - 1] == key) || (q + 1 < d && sh.row.key[q + 1] == key);
            if (tie) {
                int a = 0, hi = q;                        // first place with this key
                while (a < hi) {
                    const int mid = (a + hi) >> 1;
                    if (sh.row.key[mid] < key) a = mid + 1;
                    else hi = mid;
                }
                int b = q + 1;                            // first place past the run
                hi = d;
                while (b < hi) {
                    const int mid = (b + hi) >> 1;
                    if (sh.row.key[mid] <= key) b = mid + 1;
                    else hi = mid;
                }
                const int64_t p = beg + v[s];
                const int32_t id = nbr_id(p, col[p], col_orig, orig_id);
                int before = 0;
                for (int r = a; r < b; ++r) {
                    const int64_t pr = beg + sh.row.place[r];
                    before += nbr_id(pr, col[pr], col_orig, orig_id) < id ? 1 : 0;
                }
                rk = (uint32_t)(a + before) | ((uint32_t)(d - b + before) << 16);
            }
            sh.row.rank[v[s]] = rk;
        }
        __syncthreads();
#pragma unroll 2
        for (int s = 0; s < IPT; ++s) {
            const int q = s * TB + (int)threadIdx.x;
            if (q < d) {
                const uint32_t r = sh.row.rank[q];
                emit_ranks(em, row, col[beg + q], eid[beg + q], d, r & 0xffffu, r >> 16);
            }
        }
        __syncthreads();
    }
}

// Listed rows ranked by counting against keys read from memory (FP64
// distances with d > 64).
template <typename Tr>
__global__ __launch_bounds__(SBLOCK) void k_rank_count(
    const int32_t *__restrict__ list, const unsigned int *__restrict__ count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id,
    const int32_t *__restrict__ col_orig, const Tr *__restrict__ rho, Emit em) {
    const unsigned int nr = *count;
    for (unsigned int h = blockIdx.x; h < nr; h += gridDim.x) {
        const int64_t row = list[h];
        const int64_t beg = row_ptr[row];
        const int64_t d = row_ptr[row + 1] - beg;
        for (int64_t t = threadIdx.x; t < d; t += SBLOCK) {
            const int32_t j = col[beg + t];
            const int32_t e = eid[beg + t];
            const Tr r = rho[e];
            const int32_t id = nbr_id(beg + t, j, col_orig, orig_id);
            int64_t lt = 0, eq = 0, eqlt = 0;
            for (int64_t u = 0; u < d; ++u) {
                const int32_t ju = col[beg + u];
                const Tr ru = rho[eid[beg + u]];
                const int32_t iu = nbr_id(beg + u, ju, col_orig, orig_id);
                lt += (ru < r) ? 1 : 0;
                eq += (ru == r) ? 1 : 0;
                eqlt += (ru == r && iu < id) ? 1 : 0;
            }
            emit_ranks(em, row, j, e, d, lt + eqlt, d - lt - eq + eqlt);
        }
    }
}

// Rows longer than SORT_CAP (FP32 distances): bucket partition, then one
// wave per bucket.  A workgroup per row sorts a regular sample of the row's
// keys in LDS; runs of consecutive sorted samples delimit the buckets,
// whose sizes are counted and scanned, and the row's entries are scattered
// to their bucket's range of a scratch copy (key and offset in the row).  An
// entry's rank is its bucket's offset plus its rank among the bucket's keys.
// Keys are unique within a row (the neighbour id breaks ties), so the order
// the scatter leaves inside a bucket does not matter.  A key with u samples
// <= it goes to bucket floor(u * B / S): every bucket spans S / B samples.
constexpr int HUB_TB = 1024;
constexpr int HUB_SAMPLE = 16384;       // largest sample (128 KiB of keys in LDS)
constexpr int HUB_BUCKET = 256;         // target bucket size
constexpr int HUB_MIN_SP = 4;           // fewest samples per bucket
constexpr int HUB_MAX_B = HUB_SAMPLE / HUB_MIN_SP;
constexpr int HUB_KPL = 8;              // bucket keys per lane held in registers
constexpr uint32_t HUB_EMITTED = 0x80000000u;  // place already emitted (above any rank: d < 2^31)

struct HubScratch {
    unsigned long long *key;   // [2m] bucketed keys, at the row's own entry range (32-bit
                               // distance keys: key << 32 | offset of the entry in its row)
    uint32_t *pos;             // [2m] offset in the row of each bucketed 64-bit key (32-bit
                               // keys: each entry's key at its own place between the passes,
                               // then its LOCAL rank or HUB_EMITTED)
    int32_t *bk_row;           // [cap] the bucket's row
    uint32_t *bk_off;          // [cap] bucket offset within its row
    uint32_t *bk_cnt;          // [cap] bucket size
    unsigned int *nbk;         // [1] buckets written
    int64_t cap;
};

// In-place exclusive scan of a[0 .. B) (B <= 4 * HUB_TB) by the workgroup.
__device__ void hub_scan(uint32_t *a, int B, uint32_t *wsum) {
    const int t = threadIdx.x, lane = t & (WAVE - 1), w = t >> 6;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = 4 * t + i;
        v[i] = q < B ? a[q] : 0u;
        s += v[i];
    }
    uint32_t inc = s;
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, WAVE);
        if (lane >= o) inc += y;
    }
    if (lane == WAVE - 1) wsum[w] = inc;
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (int i = 0; i < HUB_TB / WAVE; ++i) {
            const uint32_t x = wsum[i];
            wsum[i] = run;
            run += x;
        }
    }
    __syncthreads();
    uint32_t b = wsum[w] + inc - s;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = 4 * t + i;
        if (q < B) a[q] = b;
        b += v[i];
    }
    __syncthreads();
}

// Number of samples <= k in the sorted samp[0 .. S).
template <typename K>
__device__ __forceinline__ int hub_upper(const K *samp, int S, K k) {
    int lo = 0, hi = S;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (samp[mid] <= k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Key of entry p for the bucket partition: 64-bit (rho, id) or caller keys
// of one orientation, or, with K = uint32_t, the 32-bit distance bits alone
// (both orientations from one partition: equal distances share a bucket).
template <typename K>
__device__ __forceinline__ K hub_key(const unsigned long long *__restrict__ keys, const float *__restrict__ rho,
                                     const float *__restrict__ rho_ent, int64_t p, const int32_t *__restrict__ eid,
                                     const int32_t *__restrict__ col, const int32_t *__restrict__ col_orig,
                                     const int32_t *__restrict__ orig_id, int orient) {
    if constexpr (sizeof(K) == 4) return __float_as_uint(rho_ent ? rho_ent[p] : rho[eid[p]]);
    else return entry_key(keys, rho, p, eid[p], nbr_id(p, col[p], col_orig, orig_id), orient);
}

template <typename K>
__global__ __launch_bounds__(HUB_TB) void k_hub_partition(
    const int32_t *__restrict__ list, const unsigned int *__restrict__ count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id,
    const int32_t *__restrict__ col_orig, const float *__restrict__ rho, const float *__restrict__ rho_ent,
    const unsigned long long *__restrict__ keys, int orient, HubScratch hs) {
    __shared__ K samp[HUB_SAMPLE];
    __shared__ uint32_t cnt[HUB_MAX_B];
    __shared__ uint32_t wsum[HUB_TB / WAVE];
    __shared__ uint32_t base_s;
    const unsigned int nr = *count;
    for (unsigned int h = blockIdx.x; h < nr; h += gridDim.x) {
        const int64_t row = list[h];
        const int64_t beg = row_ptr[row];
        const int64_t d = row_ptr[row + 1] - beg;
        // a power-of-two sample of about d / 16 keys (1024 .. HUB_SAMPLE), at
        // distinct, evenly spaced entries (S < d: S = 1024 < SORT_CAP < d, or S <= d / 8)
        int S = 1024;
        while (S < HUB_SAMPLE && (int64_t)S * 16 < d) S <<= 1;
        const int B = (int)min((int64_t)(S / HUB_MIN_SP), (d + HUB_BUCKET - 1) / HUB_BUCKET);
        for (int t = threadIdx.x; t < S; t += HUB_TB) {
            const int64_t p = beg + ((int64_t)t * d) / S;
            samp[t] = hub_key<K>(keys, rho, rho_ent, p, eid, col, col_orig, orig_id, orient);
        }
        for (int b = threadIdx.x; b < B; b += HUB_TB) cnt[b] = 0;
        __syncthreads();
        for (int size = 2; size <= S; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = threadIdx.x; t < (S >> 1); t += HUB_TB) {
                    const int a = 2 * t - (t & (stride - 1));
                    const int b = a + stride;
                    const bool up = ((a & size) == 0);
                    const K ka = samp[a], kb = samp[b];
                    if ((ka > kb) == up) {
                        samp[a] = kb;
                        samp[b] = ka;
                    }
                }
                __syncthreads();
            }
        }
        for (int64_t q = threadIdx.x; q < d; q += HUB_TB) {
            const int64_t p = beg + q;
            const K k = hub_key<K>(keys, rho, rho_ent, p, eid, col, col_orig, orig_id, orient);
            atomicAdd(&cnt[min(B - 1, hub_upper(samp, S, k) * B / S)], 1u);
            // 32-bit keys: kept at the entry's own place for the scatter pass
            // (one gather of the distance per entry instead of two)
            if constexpr (sizeof(K) == 4) hs.pos[p] = k;
        }
        __syncthreads();
        if (threadIdx.x == 0) base_s = atomicAdd(hs.nbk, (unsigned int)B);
        __syncthreads();
        const int64_t base = base_s;
        const bool fits = base + B <= hs.cap;              // holds by the workspace bound
        if (fits) {
            for (int b = threadIdx.x; b < B; b += HUB_TB) {
                hs.bk_row[base + b] = (int32_t)row;
                hs.bk_cnt[base + b] = cnt[b];
            }
        }
        __syncthreads();
        hub_scan(cnt, B, wsum);
        if (fits) {
            for (int b = threadIdx.x; b < B; b += HUB_TB) hs.bk_off[base + b] = cnt[b];
        }
        __syncthreads();
        for (int64_t q = threadIdx.x; q < d; q += HUB_TB) {
            const int64_t p = beg + q;
            if constexpr (sizeof(K) == 4) {
                // bucketed as (key << 32 | place in row): one 8-byte entry
                const uint32_t k = hs.pos[p];
                const uint32_t at = atomicAdd(&cnt[min(B - 1, hub_upper(samp, S, k) * B / S)], 1u);
                hs.key[beg + at] = ((unsigned long long)k << 32) | (uint32_t)q;
            } else {
                const K k = hub_key<K>(keys, rho, rho_ent, p, eid, col, col_orig, orig_id, orient);
                const uint32_t at = atomicAdd(&cnt[min(B - 1, hub_upper(samp, S, k) * B / S)], 1u);
                hs.key[beg + at] = (unsigned long long)k;
                hs.pos[beg + at] = (uint32_t)q;
            }
        }
        __syncthreads();
    }
}

// One wave per bucket: each key's rank among the bucket's keys, counted
// against all of them broadcast 64 at a time; HUB_KPL * 64 own keys per pass.
// `em` names one orientation (the one the keys were built for).
__global__ __launch_bounds__(SBLOCK) void k_hub_rank(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const int32_t *__restrict__ eid,
    Emit em, HubScratch hs) {
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned int nb = (unsigned int)min((int64_t)(*hs.nbk), hs.cap);
    const unsigned int waves = gridDim.x * (SBLOCK / WAVE);
    for (unsigned int w = blockIdx.x * (SBLOCK / WAVE) + (threadIdx.x >> 6); w < nb; w += waves) {
        const int64_t row = hs.bk_row[w];
        const int64_t beg = row_ptr[row];
        const int64_t d = row_ptr[row + 1] - beg;
        const uint32_t off = hs.bk_off[w], c = hs.bk_cnt[w];
        const unsigned long long *bk = hs.key + beg + off;
        const uint32_t *bp = hs.pos + beg + off;
        for (uint32_t c0 = 0; c0 < c; c0 += HUB_KPL * WAVE) {
            unsigned long long key[HUB_KPL];
            int rank[HUB_KPL];
#pragma unroll
            for (int t = 0; t < HUB_KPL; ++t) {
                const uint32_t q = c0 + t * WAVE + lane;
                key[t] = q < c ? bk[q] : ~0ull;
                rank[t] = 0;
            }
            for (uint32_t s0 = 0; s0 < c; s0 += WAVE) {
                const unsigned long long mine = (s0 + lane < c) ? bk[s0 + lane] : ~0ull;
                const int lim = (int)min((uint32_t)WAVE, c - s0);
                for (int src = 0; src < lim; ++src) {
                    const unsigned long long k = shfl(mine, src);
#pragma unroll
                    for (int t = 0; t < HUB_KPL; ++t) rank[t] += (k < key[t]) ? 1 : 0;
                }
            }
#pragma unroll
            for (int t = 0; t < HUB_KPL; ++t) {
                const uint32_t q = c0 + t * WAVE + lane;
                if (q < c) {
                    const int64_t p = beg + bp[q];
                    const int64_t r = (int64_t)off + rank[t];
                    emit_ranks(em, row, col[p], eid[p], d, r, r);
                }
            }
        }
    }
}

// One wave per bucket (of more than c_min entries) of a partition on 32-bit
// distance bits: every entry's ranks in both orders from counts inside its bucket (equal distances share
// a bucket, so every entry of an earlier bucket is smaller and of a later
// one larger): LOCAL = off + smaller + tied with smaller id, GLOBAL = d - off -
// smaller - equal + tied with smaller id.  The ids are read only when the
// wave's keys have a tie in their bucket.
__global__ __launch_bounds__(SBLOCK) void k_hub_rank32(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const int32_t *__restrict__ eid,
    const int32_t *__restrict__ orig_id, const int32_t *__restrict__ col_orig, Emit em, HubScratch hs,
    uint32_t c_min) {
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned int nb = (unsigned int)min((int64_t)(*hs.nbk), hs.cap);
    const unsigned int waves = gridDim.x * (SBLOCK / WAVE);
    for (unsigned int w = blockIdx.x * (SBLOCK / WAVE) + (threadIdx.x >> 6); w < nb; w += waves) {
        const uint32_t c = hs.bk_cnt[w];
        if (c <= c_min) continue;                    // sorted by k_hub_sort
        const int64_t row = hs.bk_row[w];
        const int64_t beg = row_ptr[row];
        const int64_t d = row_ptr[row + 1] - beg;
        const uint32_t off = hs.bk_off[w];
        const unsigned long long *bk = hs.key + beg + off;
        for (uint32_t c0 = 0; c0 < c; c0 += HUB_KPL * WAVE) {
            uint32_t key[HUB_KPL];
            int lt[HUB_KPL], eq[HUB_KPL], eqlt[HUB_KPL];
#pragma unroll
            for (int t = 0; t < HUB_KPL; ++t) {
                const uint32_t q = c0 + t * WAVE + lane;
                key[t] = q < c ? (uint32_t)(bk[q] >> 32) : 0u;
                lt[t] = eq[t] = eqlt[t] = 0;
            }
            for (uint32_t s0 = 0; s0 < c; s0 += WAVE) {
                const uint32_t mine = (s0 + lane < c) ? (uint32_t)(bk[s0 + lane] >> 32) : 0u;
                const int lim = (int)min((uint32_t)WAVE, c - s0);
                for (int src = 0; src < lim; ++src) {
                    const uint32_t kb = (uint32_t)shfl((int)mine, src);
#pragma unroll
                    for (int t = 0; t < HUB_KPL; ++t) {
                        lt[t] += (kb < key[t]) ? 1 : 0;
                        eq[t] += (kb == key[t]) ? 1 : 0;
                    }
                }
            }
            bool tie = false;
#pragma unroll
            for (int t = 0; t < HUB_KPL; ++t) tie = tie || (c0 + t * WAVE + lane < c && eq[t] > 1);
            if (__any(tie)) {                          // uniform across the wave
                int32_t id[HUB_KPL];
#pragma unroll
                for (int t = 0; t < HUB_KPL; ++t) {
                    const uint32_t q = c0 + t * WAVE + lane;
                    id[t] = 0;
                    if (q < c) {
                        const int64_t p = beg + (uint32_t)bk[q];
                        id[t] = nbr_id(p, col[p], col_orig, orig_id);
                    }
                }
                for (uint32_t s0 = 0; s0 < c; s0 += WAVE) {
                    uint32_t mine = 0u;
                    int32_t mid = 0;
                    if (s0 + lane < c) {
                        const unsigned long long kp = bk[s0 + lane];
                        mine = (uint32_t)(kp >> 32);
                        const int64_t p = beg + (uint32_t)kp;
                        mid = nbr_id(p, col[p], col_orig, orig_id);
                    }
                    const int lim = (int)min((uint32_t)WAVE, c - s0);
                    for (int src = 0; src < lim; ++src) {
                        const uint32_t kb = (uint32_t)shfl((int)mine, src);
                        const int32_t ib = shfl(mid, src);
#pragma unroll
                        for (int t = 0; t < HUB_KPL; ++t) eqlt[t] += (kb == key[t] && ib < id[t]) ? 1 : 0;
                    }
                }
            }
            // an untied entry's LOCAL rank goes to its place in the row (its
            // GLOBAL rank is d - 1 - LOCAL) for k_hub_emit, which writes the
            // records in row order; tied entries are emitted here
#pragma unroll
            for (int t = 0; t < HUB_KPL; ++t) {
                const uint32_t q = c0 + t * WAVE + lane;
                if (q < c) {
                    const int64_t p = beg + (uint32_t)bk[q];
                    const int64_t rl = (int64_t)off + lt[t] + eqlt[t];
                    if (eq[t] > 1) {
                        const int64_t rg = d - (int64_t)off - lt[t] - eq[t] + eqlt[t];
                        emit_ranks(em, row, col[p], eid[p], d, rl, rg);
                        hs.pos[p] = HUB_EMITTED;
                    } else {
                        hs.pos[p] = (uint32_t)rl;
                    }
                }
            }
        }
    }
}

// Buckets of c_lo < c <= 64 * IPT entries of a partition on 32-bit distance
// bits, one per one-wave workgroup: the bucket's keys sorted by a block radix
// sort in LDS (bucket index as payload), so that an untied key's LOCAL rank is
// the bucket offset + its sorted place.  Tied keys (adjacent after the sort)
// take their order inside the run from the neighbour ids, as in k_rank_radix,
// and are emitted here.
template <int IPT>
__global__ __launch_bounds__(WAVE) void k_hub_sort(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const int32_t *__restrict__ eid,
    const int32_t *__restrict__ orig_id, const int32_t *__restrict__ col_orig, Emit em, HubScratch hs,
    uint32_t c_lo) {
    constexpr int P = WAVE * IPT;
    using Sorter = rocprim::block_radix_sort<uint32_t, WAVE, IPT, uint16_t>;
    __shared__ union {
        typename Sorter::storage_type sort;
        struct {
            uint32_t key[P];
            uint32_t place[P];                       // offset in the row of sorted place q
        } b;
    } sh;
    const unsigned int nb = (unsigned int)min((int64_t)(*hs.nbk), hs.cap);
    for (unsigned int w = blockIdx.x; w < nb; w += gridDim.x) {
        const uint32_t c = hs.bk_cnt[w];
        if (c <= c_lo || c > (uint32_t)P) continue;  // uniform over the workgroup
        const int64_t row = hs.bk_row[w];
        const int64_t beg = row_ptr[row];
        const int64_t d = row_ptr[row + 1] - beg;
        const uint32_t off = hs.bk_off[w];
        const unsigned long long *bk = hs.key + beg + off;
        uint32_t k[IPT];
        uint16_t v[IPT];
#pragma unroll
        for (int s = 0; s < IPT; ++s) {
            const uint32_t q = (uint32_t)(s * WAVE) + threadIdx.x;
            k[s] = q < c ? min((uint32_t)(bk[q] >> 32), KEY_LAST) : 0xffffffffu;
            v[s] = (uint16_t)q;
        }
        Sorter().sort(k, v, sh.sort);                // blocked: thread t holds sorted places t * IPT + s
        __syncthreads();
#pragma unroll
        for (int s = 0; s < IPT; ++s) {
            const uint32_t q = threadIdx.x * IPT + s;
            sh.b.key[q] = k[s];
            sh.b.place[q] = q < c ? (uint32_t)bk[v[s]] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < IPT; ++s) {
            const int q = (int)(threadIdx.x * IPT + s);
            if (q >= (int)c) continue;
            const uint32_t key = k[s];
            const int64_t p = beg + sh.b.place[q];
            const bool tie = (q > 0 && sh.b.key[q - 1] == key) || (q + 1 < (int)c && sh.b.key[q + 1] == key);
            if (!tie) {
                hs.pos[p] = off + (uint32_t)q;
                continue;
            }
            int a = 0, hi = q;                            // first place with this key
            while (a < hi) {
                const int mid = (a + hi) >> 1;
                if (sh.b.key[mid] < key) a = mid + 1;
                else hi = mid;
            }
            int b = q + 1;                                // first place past the run
            hi = (int)c;
            while (b < hi) {
                const int mid = (b + hi) >> 1;
                if (sh.b.key[mid] <= key) b = mid + 1;
                else hi = mid;
            }
            const int32_t j = col[p];
            const int32_t id = nbr_id(p, j, col_orig, orig_id);
            int before = 0;
            for (int r = a; r < b; ++r) {
                const int64_t pr = beg + sh.b.place[r];
                before += nbr_id(pr, col[pr], col_orig, orig_id) < id ? 1 : 0;
            }
            emit_ranks(em, row, j, eid[p], d, (int64_t)off + a + before, d - (int64_t)off - b + before);
            hs.pos[p] = HUB_EMITTED;
        }
        __syncthreads();
    }
}

// Records of the untied entries of the partitioned rows, in row order: the
// buckets' offsets and sizes tile each row's places [0, d) into consecutive
// ranges, one wave per range.
__global__ __launch_bounds__(SBLOCK) void k_hub_emit(const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ eid, Emit em, HubScratch hs) {
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned int nb = (unsigned int)min((int64_t)(*hs.nbk), hs.cap);
    const unsigned int waves = gridDim.x * (SBLOCK / WAVE);
    for (unsigned int w = blockIdx.x * (SBLOCK / WAVE) + (threadIdx.x >> 6); w < nb; w += waves) {
        const int64_t row = hs.bk_row[w];
        const int64_t beg = row_ptr[row];
        const int64_t d = row_ptr[row + 1] - beg;
        const int64_t a = beg + hs.bk_off[w], b = a + hs.bk_cnt[w];
        for (int64_t p = a + lane; p < b; p += WAVE) {
            const uint32_t r = hs.pos[p];
            if (r != HUB_EMITTED) emit_ranks(em, row, col[p], eid[p], d, r, d - 1 - (int64_t)r);
        }
    }
}

// Block-wide sum of per-thread counts, valid in thread 0.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long c) {
    __shared__ unsigned long long part[SBLOCK / WAVE];
    for (int d = WAVE / 2; d >= 1; d >>= 1) c += shfl_down(c, d);
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < SBLOCK / WAVE; ++w) t += part[w];
    return t;
}

// Block-wide sum of per-thread counts; thread 0 adds it to *out (one atomic
// per block; integer addition, so the total does not depend on order).
// Atomics on one address from many blocks serialise at the memory side, so
// grids that use it stay small.
__device__ __forceinline__ void block_add(unsigned long long c, unsigned long long *out) {
    const unsigned long long t = block_sum(c);
    if (threadIdx.x == 0 && t) atomicAdd(out, t);
}

constexpr int COUNT_BLOCKS = 2048;
constexpr int SUM_BLOCKS = 256;    // grids that end in block_add
constexpr int HIST_BLOCKS = 2048;

// Sum of a byte mask into a 64-bit device counter.
__global__ __launch_bounds__(SBLOCK) void k_count_bytes(int64_t m, const uint8_t *__restrict__ keep,
                                                       unsigned long long *out) {
    unsigned long long c = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
         q += (int64_t)gridDim.x * blockDim.x)
        c += keep[q];
    block_add(c, out);
}

// ---------------------------------------------------------------------- fit --

constexpr int DIGIT = 11;
constexpr int NBINS = 1 << DIGIT;
constexpr double GRID = 1099511627776.0;   // 2^40

// The select's digits of a grid index (at most 2^40, so 41 bits), most
// significant first: 11 + 11 + 11 + 8 bits.
constexpr int NPASS = 4;
constexpr int DIGIT_SHIFT[NPASS] = {30, 19, 8, 0};
constexpr int DIGIT_WIDTH[NPASS] = {11, 11, 11, 8};
static_assert(DIGIT_SHIFT[0] + DIGIT_WIDTH[0] == 41 && (1ull << 40) >> DIGIT_SHIFT[0] < NBINS,
              "the first digit holds the top bits of every grid index");

// Edges per thread per step of the fit's grid-stride loops (loads issued
// together).
constexpr int FIT_U = 4;
constexpr int FIT_LDS_TB = 1024;   // threads of the grid pass with the log tables in LDS

// Two grid indices in one 16-byte load.
struct alignas(16) U64x2 {
    unsigned long long a, b;
};

// logs[v] = log(v) for v = 1 .. count - 1 (logs[0] unused), and
// logs[count + v] = 1 / log(v) for v >= 2.
__global__ void k_log_table(int64_t count, double *__restrict__ logs) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < count;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double l = v > 0 ? log((double)v) : 0.0;
        logs[v] = l;
        logs[count + v] = v > 1 ? 1.0 / l : 0.0;
    }
}

// Estimated grid index of a side's threshold (0: kept at every e): the side
// (d, r) selects once d^e >= r + 1, i.e. e >= log(r + 1) / log(d); inv_ld =
// 1 / log(d) from the table.  The estimate is within a small fraction of a
// grid step of the index the exact check finds (see FIT_MARGIN).
__device__ __forceinline__ unsigned long long side_grid(uint32_t d, uint32_t r, double inv_ld,
                                                        const double *__restrict__ logs) {
    if (r == 0 || d < 2) return 0ull;
    const double gi = ceil(logs[r + 1] * inv_ld * GRID);
    return gi <= 0.0 ? 0ull : (unsigned long long)gi;
}

// Rank of fitted orientation o in a side record: the first rank, or the
// second when both orientations are fitted.
__device__ __forceinline__ uint32_t rec_rank(const uint4 &v, int o) { return o == 0 ? v.y : v.z; }

// Per fitted orientation (at most two): the edges' grid indices and the
// current radix histogram.
struct FitArrays {
    unsigned long long *G[2];
    unsigned int *hist[2];
};

// Histogram of a thread's sequence of bins: runs of equal bins are added at once.
struct BinRun {
    int last = -1;
    unsigned int run = 0;
    __device__ __forceinline__ void add(unsigned int *h, int bin) {
        if (bin == last) {
            ++run;
        } else {
            if (run) atomicAdd(&h[last], run);
            last = bin;
            run = 1;
        }
    }
    __device__ __forceinline__ void flush(unsigned int *h) {
        if (run) atomicAdd(&h[last], run);
    }
};

// G_o[e] = the smaller of edge e's two sides' grid indices, and the
// histogram of the first radix digit of G_o (its bits from DIGIT_SHIFT[0]
// up), for every fitted orientation o < nfit from one read of the side
// records.  hist must be zero on entry.  LDS_TAB: the log tables (2 * nlogs
// doubles) are first copied into dynamic LDS, one workgroup per compute unit
// (six random table reads per edge cost more from the caches than the
// records' stream; the values read are the same).
template <int TB, bool LDS_TAB>
__global__ __launch_bounds__(TB) void k_fit_grid(int64_t m, const uint4 *__restrict__ recs,
                                                const double *__restrict__ logs, int64_t nlogs, int nfit,
                                                FitArrays fa) {
    extern __shared__ double tab_lds[];
    __shared__ unsigned int h[2][NBINS];
    if (LDS_TAB)
        for (int64_t i = threadIdx.x; i < 2 * nlogs; i += TB) tab_lds[i] = logs[i];
    const double *tab = LDS_TAB ? tab_lds : logs;
    for (int b = threadIdx.x; b < 2 * NBINS; b += TB) h[b / NBINS][b % NBINS] = 0;
    __syncthreads();
    BinRun run[2];
    constexpr int64_t STEP = (int64_t)TB * FIT_U;
    for (int64_t b0 = (int64_t)blockIdx.x * STEP; b0 < m; b0 += (int64_t)gridDim.x * STEP) {
        uint4 a[FIT_U] = {}, b[FIT_U] = {};
#pragma unroll
        for (int u = 0; u < FIT_U; ++u) {
            const int64_t e = b0 + u * TB + threadIdx.x;
            if (e < m) {
                a[u] = recs[2 * e];
                b[u] = recs[2 * e + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < FIT_U; ++u) {
            const int64_t e = b0 + u * TB + threadIdx.x;
            if (e >= m) continue;
            const double ia = tab[nlogs + a[u].x], ib = tab[nlogs + b[u].x];
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                if (o >= nfit) break;
                const unsigned long long ga = side_grid(a[u].x, rec_rank(a[u], o), ia, tab);
                const unsigned long long gb = side_grid(b[u].x, rec_rank(b[u], o), ib, tab);
                const unsigned long long g = ga < gb ? ga : gb;
                fa.G[o][e] = g;
                run[o].add(h[o], (int)((g >> DIGIT_SHIFT[0]) & (NBINS - 1)));
            }
        }
    }
#pragma unroll
    for (int o = 0; o < 2; ++o)
        if (o < nfit) run[o].flush(h[o]);
    __syncthreads();
    for (int o = 0; o < nfit; ++o)
        for (int b = threadIdx.x; b < NBINS; b += TB)
            if (h[o][b]) atomicAdd(&fa.hist[o][b], h[o][b]);
}

// Values of G_o matching the select's first digit, gathered by the second
// pass so that the last two passes read only them.  n[o] counts every
// match; when it exceeds cap the list is incomplete and the later passes
// read G_o again.
struct CandArrays {
    unsigned long long *v[2];   // [cap] per fitted orientation
    unsigned long long *n;      // [2]
    int64_t cap;
};

// Zero the histograms, the candidate counts and the first check's six
// counters; state[2o] = prefix of selected digits, state[2o + 1] = rank
// still to skip (1-based inside the prefix), for o < nfit.  One block.
__global__ __launch_bounds__(SBLOCK) void k_select_init(unsigned long long *state, unsigned long long K, int nfit,
                                                       unsigned int *hist, unsigned long long *cand_n,
                                                       unsigned long long *counts) {
    for (int b = threadIdx.x; b < 2 * NBINS; b += SBLOCK) hist[b] = 0;
    if (threadIdx.x < 2) cand_n[threadIdx.x] = 0;
    if (threadIdx.x < 6) counts[threadIdx.x] = 0;
    if (threadIdx.x == 0)
        for (int o = 0; o < nfit; ++o) {
            state[2 * o] = 0;
            state[2 * o + 1] = K;
        }
}

constexpr int STAGE = 2048;   // LDS staging of a block's candidates (entries)

// Append the block's staged candidates to the global list (one reservation
// per block and flush).  Every thread calls it, after a barrier that follows
// the last staging write.
template <typename T>
__device__ __forceinline__ void stage_flush(const T *stage, unsigned int *n_stage, unsigned long long *base_sh,
                                            T *dst, unsigned long long *dst_n, int64_t cap) {
    const unsigned int ns = *n_stage;
    if (threadIdx.x == 0 && ns) *base_sh = atomicAdd(dst_n, (unsigned long long)ns);
    __syncthreads();
    if (ns) {
        const unsigned long long base = *base_sh;
        for (unsigned int i = threadIdx.x; i < ns; i += SBLOCK)
            if (base + i < (unsigned long long)cap) dst[base + i] = stage[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) *n_stage = 0;
    __syncthreads();
}

// Histogram of the digit at `shift` (`width` bits) of G_o among the values
// whose higher digits equal the selected prefix; orientation o = blockIdx.y.
// COMPACT (the second digit's pass) also appends those values to the
// candidate list; the later passes read the list instead of G_o when it is
// complete.
template <bool COMPACT>
__global__ __launch_bounds__(SBLOCK) void k_radix_hist(int64_t m, FitArrays fa, CandArrays cs, int shift,
                                                      int width, const unsigned long long *__restrict__ state) {
    __shared__ unsigned int h[NBINS];
    __shared__ unsigned long long stage[COMPACT ? STAGE : 1];
    __shared__ unsigned int n_stage;
    __shared__ unsigned long long base_sh;
    const int o = blockIdx.y;
    const unsigned long long *__restrict__ src = fa.G[o];
    int64_t count = m;
    if (!COMPACT) {
        const unsigned long long nc = cs.n[o];
        if (nc <= (unsigned long long)cs.cap) {
            src = cs.v[o];
            count = (int64_t)nc;
        }
    }
    for (int b = threadIdx.x; b < NBINS; b += SBLOCK) h[b] = 0;
    if (threadIdx.x == 0) n_stage = 0;
    __syncthreads();
    const unsigned long long prefix = state[2 * o];
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned long long below = lane ? (~0ull >> (WAVE - lane)) : 0ull;
    BinRun run;
    constexpr int64_t STEP = (int64_t)SBLOCK * FIT_U;
    for (int64_t b0 = (int64_t)blockIdx.x * STEP; b0 < count; b0 += (int64_t)gridDim.x * STEP) {
        unsigned long long v[FIT_U];
#pragma unroll
        for (int u = 0; u < FIT_U; ++u) {
            const int64_t e = b0 + u * SBLOCK + threadIdx.x;
            v[u] = e < count ? src[e] : ~0ull;     // ~0 matches no prefix (prefixes stay below 2^33)
        }
#pragma unroll
        for (int u = 0; u < FIT_U; ++u) {
            const bool match = (v[u] >> (shift + width)) == prefix;
            if (match) run.add(h, (int)((v[u] >> shift) & (NBINS - 1)));
            if (COMPACT) {
                const unsigned long long mask = __ballot(match);
                if (mask) {
                    const int leader = __ffsll((long long)mask) - 1;
                    unsigned int off = 0;
                    if (lane == leader) off = atomicAdd(&n_stage, (unsigned int)__popcll(mask));
                    off = __shfl(off, leader, WAVE);
                    if (match) stage[off + (unsigned int)__popcll(mask & below)] = v[u];
                }
            }
        }
        if (COMPACT) {
            __syncthreads();
            if (n_stage > STAGE - STEP) stage_flush(stage, &n_stage, &base_sh, cs.v[o], &cs.n[o], cs.cap);
        }
    }
    run.flush(h);
    if (COMPACT) {
        __syncthreads();
        stage_flush(stage, &n_stage, &base_sh, cs.v[o], &cs.n[o], cs.cap);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NBINS; b += SBLOCK)
        if (h[b]) atomicAdd(&fa.hist[o][b], h[b]);
}

// The bin holding the state's rank, appended (`width` bits) to the prefix,
// and the histogram cleared for the next pass; orientation o = blockIdx.x.
__global__ __launch_bounds__(SBLOCK) void k_radix_pick(FitArrays fa, unsigned long long *state_all, int width) {
    __shared__ unsigned long long part[SBLOCK];
    constexpr int PER = NBINS / SBLOCK;
    unsigned int *hist = fa.hist[blockIdx.x];
    unsigned long long *state = state_all + 2 * blockIdx.x;
    unsigned long long c = 0;
    for (int q = 0; q < PER; ++q) c += hist[threadIdx.x * PER + q];
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long need = state[1];   // 1-based rank inside the current prefix
        unsigned long long run = 0;
        int chunk = 0;
        while (chunk < SBLOCK - 1 && run + part[chunk] < need) run += part[chunk++];
        int bin = chunk * PER;
        while (bin < chunk * PER + PER - 1 && run + hist[bin] < need) run += hist[bin++];
        state[0] = (state[0] << width) | (unsigned long long)bin;
        state[1] = need - run;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NBINS; b += SBLOCK) hist[b] = 0;
}

// The exact check of a candidate grid point g_hi per orientation (and of
// g_hi - 1 when use_lo): budget tables from the host at both points.
struct CountArgs {
    const int32_t *tab_hi[2], *tab_lo[2];
    const unsigned long long *G[2];
    unsigned long long g_hi[2];
    int use_lo[2], active[2];
    int keep_aligned[2];          // keep[o] is 4-byte aligned
    uint8_t *keep[2];
    uint32_t *list[2];            // edges left to the tables (LIST form), per orientation
    unsigned long long *list_n;   // [2]: their number (all of them, also beyond list_cap)
    int64_t list_cap;
};

// An edge is kept at grid point p exactly when its threshold index is <= p.
// G holds that index estimated from the log ratio in FP64, within a small
// fraction of one grid step of the index the host's pow tables give; edges
// whose estimate lies more than FIT_MARGIN steps from both candidate points
// are classified by the estimate, the rest by the budget tables.
constexpr unsigned long long FIT_MARGIN = 1ull << 16;

// Exact kept counts at the two grid points of every active orientation (per
// block, into part[4 * block ..]), and keep[] at the upper point.  A thread takes four consecutive edges at a
// time (two 16-byte loads of G per orientation, one 4-byte store of keep when
// keep is 4-byte aligned).  LIST form (launched before the budget tables
// reach the device): an edge whose estimate does not settle it is not counted
// but listed for k_fit_margin (ids staged in LDS, one global reservation per
// block and flush), and its keep flag is left for that kernel to store.
constexpr int STAGE_M = 4096;   // LDS staging of listed edges per orientation

template <bool LIST>
__global__ __launch_bounds__(SBLOCK) void k_fit_count(int64_t m, const uint4 *__restrict__ recs, int nfit,
                                                     CountArgs ca, unsigned long long *__restrict__ part) {
    __shared__ uint32_t stage[LIST ? 2 : 1][LIST ? STAGE_M : 1];
    __shared__ unsigned int n_stage[2];
    __shared__ unsigned long long base_sh;
    unsigned long long c[2][2] = {{0, 0}, {0, 0}};
    constexpr int QU = FIT_U / 2;                      // quads per thread per step
    const int64_t nq = (m + 3) / 4;
    constexpr int64_t STEP = (int64_t)SBLOCK * QU;
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned long long below = lane ? (~0ull >> (WAVE - lane)) : 0ull;
    if (LIST) {
        if (threadIdx.x < 2) n_stage[threadIdx.x] = 0;
        __syncthreads();
    }
    for (int64_t q0 = (int64_t)blockIdx.x * STEP; q0 < nq; q0 += (int64_t)gridDim.x * STEP) {
        unsigned long long gv[2][QU][4];
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            if (o >= nfit || !ca.active[o]) continue;
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int64_t q = q0 + u * SBLOCK + threadIdx.x;
                const int64_t e0 = 4 * q;
                if (e0 + 3 < m) {
                    const U64x2 *G2 = reinterpret_cast<const U64x2 *>(ca.G[o] + e0);
                    const U64x2 x = G2[0], y = G2[1];
                    gv[o][u][0] = x.a;
                    gv[o][u][1] = x.b;
                    gv[o][u][2] = y.a;
                    gv[o][u][3] = y.b;
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) gv[o][u][t] = e0 + t < m ? ca.G[o][e0 + t] : 0ull;
                }
            }
        }
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            if (o >= nfit || !ca.active[o]) continue;
            const unsigned long long hi = ca.g_hi[o];
            const unsigned long long lo = hi > 0 ? hi - 1 : 0;
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int64_t q = q0 + u * SBLOCK + threadIdx.x;
                const int64_t e0 = 4 * q;
                uint32_t kb = 0;                       // keep bytes, little-endian
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int64_t e = e0 + t;
                    const bool valid = e < m;
                    const unsigned long long g = gv[o][u][t];
                    bool k_hi = false, k_lo = false, listed = false;
                    if (!valid || g > hi + FIT_MARGIN) {
                        // past the end, or kept at neither point
                    } else if (g + FIT_MARGIN < lo) {
                        k_hi = k_lo = true;
                    } else if (LIST) {
                        listed = true;
                    } else {
                        const uint4 a = recs[2 * e], b = recs[2 * e + 1];
                        const uint32_t ra = rec_rank(a, o), rb = rec_rank(b, o);
                        k_hi = ra < (uint32_t)ca.tab_hi[o][a.x] || rb < (uint32_t)ca.tab_hi[o][b.x];
                        k_lo = ca.use_lo[o] &&
                               (ra < (uint32_t)ca.tab_lo[o][a.x] || rb < (uint32_t)ca.tab_lo[o][b.x]);
                    }
                    kb |= (k_hi ? 1u : 0u) << (8 * t);
                    c[o][0] += k_hi;
                    if (ca.use_lo[o]) c[o][1] += k_lo;
                    if (LIST) {
                        const unsigned long long mask = __ballot(listed);
                        if (mask) {
                            const int leader = __ffsll((long long)mask) - 1;
                            unsigned int off = 0;
                            if (lane == leader) off = atomicAdd(&n_stage[o], (unsigned int)__popcll(mask));
                            off = __shfl(off, leader, WAVE);
                            if (listed) stage[LIST ? o : 0][off + (unsigned int)__popcll(mask & below)] = (uint32_t)e;
                        }
                    }
                }
                if (e0 >= m) continue;
                if (ca.keep_aligned[o] && e0 + 3 < m) {
                    *reinterpret_cast<uint32_t *>(ca.keep[o] + e0) = kb;
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (e0 + t < m) ca.keep[o][e0 + t] = (uint8_t)(kb >> (8 * t));
                }
            }
        }
        if (LIST) {
            __syncthreads();
#pragma unroll
            for (int o = 0; o < 2; ++o)
                if (o < nfit && ca.active[o] && n_stage[o] > STAGE_M - SBLOCK * QU * 4)
                    stage_flush(stage[LIST ? o : 0], &n_stage[o], &base_sh, ca.list[o], &ca.list_n[o], ca.list_cap);
        }
    }
    if (LIST) {
        __syncthreads();
#pragma unroll
        for (int o = 0; o < 2; ++o)
            if (o < nfit && ca.active[o])
                stage_flush(stage[LIST ? o : 0], &n_stage[o], &base_sh, ca.list[o], &ca.list_n[o], ca.list_cap);
    }
    // the block's four counts to its own slots (k_sum_counts adds them up)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned long long t = block_sum(c[k >> 1][k & 1]);
        if (threadIdx.x == 0) part[4 * (int64_t)blockIdx.x + k] = t;
        __syncthreads();
    }
}

// counts[k] += the sum over nblocks blocks of part[4 * b + k], k < 4.  One
// block; wave k sums count k.
static_assert(SBLOCK / WAVE == 4, "one wave per count");
__global__ __launch_bounds__(SBLOCK) void k_sum_counts(const unsigned long long *__restrict__ part, int nblocks,
                                                      unsigned long long *__restrict__ counts) {
    const int k = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    unsigned long long c = 0;
    for (int b = lane; b < nblocks; b += WAVE) c += part[4 * (int64_t)b + k];
    for (int d = WAVE / 2; d >= 1; d >>= 1) c += shfl_down(c, d);
    if (lane == 0) counts[k] += c;
}

// The listed edges of orientation o = blockIdx.y against the budget tables:
// counts added, keep flags stored.  Does nothing for an orientation whose
// list overflowed (the host then counts it again in one full pass).
__global__ __launch_bounds__(SBLOCK) void k_fit_margin(const uint4 *__restrict__ recs, CountArgs ca,
                                                      unsigned long long *__restrict__ counts) {
    const int o = blockIdx.y;
    if (!ca.active[o]) return;
    const unsigned long long n = ca.list_n[o];
    if (n > (unsigned long long)ca.list_cap) return;
    unsigned long long c_hi = 0, c_lo = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = ca.list[o][i];
        const uint4 a = recs[2 * e], b = recs[2 * e + 1];
        const uint32_t ra = rec_rank(a, o), rb = rec_rank(b, o);
        const bool k_hi = ra < (uint32_t)ca.tab_hi[o][a.x] || rb < (uint32_t)ca.tab_hi[o][b.x];
        const bool k_lo = ca.use_lo[o] && (ra < (uint32_t)ca.tab_lo[o][a.x] || rb < (uint32_t)ca.tab_lo[o][b.x]);
        ca.keep[o][e] = k_hi ? 1 : 0;
        c_hi += k_hi;
        c_lo += k_lo;
    }
    block_add(c_hi, &counts[2 * o]);
    __syncthreads();
    block_add(c_lo, &counts[2 * o + 1]);
}

// dst[i] = src[i] for i < count; src is host memory mapped for the device.
__global__ __launch_bounds__(SBLOCK) void k_copy_mapped(int32_t *__restrict__ dst, const int32_t *__restrict__ src,
                                                       int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_store_count(const unsigned long long *__restrict__ c, int64_t *__restrict__ out) {
    *out = (int64_t)c[0];
}

// ------------------------------------------------------------------- host --

struct SelLayout {
    int32_t *lists;               // rows of degree > 64, by class
    unsigned int *cnt;            // [NCLASS]
    ClassBounds cb;
    long long *plan;              // packed small-row waves
    unsigned int *tile_waves, *plan_count;
    ScanScratch scan;
    uint4 *recs;                  // [2m] side records (Emit, MODE_REC*)
    unsigned long long *G, *G2;   // [m] grid indices per fitted orientation (G2 when both)
    unsigned long long *cand, *cand2, *cand_n;   // select candidates (CandArrays), per orientation
    unsigned long long *fit_part;                // [COUNT_BLOCKS][4]: the count pass's per-block counts
    int64_t cand_cap;
    unsigned int *hist;           // [2][NBINS]
    unsigned long long *state;    // [4]: two words per fitted orientation
    unsigned long long *counts;   // [6]: counts at the upper and lower grid point per orientation, then
                                  // the listed edges per orientation (k_fit_count LIST form)
    int32_t *tabs;                // [4][d_max + 1]: upper and lower budget tables, per orientation
    double *logs;                 // [2][d_max + 2]: log(v), then 1 / log(v)
    HubScratch hub;               // rows longer than SORT_CAP (d_max > SORT_CAP only)
};

// Degree classes above 64: wave counting with 2/4/8 keys per lane, bitonic
// sorts in LDS of 1024/2048/4096/8192 keys, then the bucket partition (FP32;
// FP64 rows above 64 are counted from memory).
static const int64_t CLASS_LO[NCLASS + 1] = {64, 128, 256, 512, 1024, 2048, 4096, 8192, (int64_t)1 << 62};

static size_t sel_layout(const ad_graph *g, void *ws, size_t ws_bytes, SelLayout *L, bool both = false) {
    Carver c(ws, ws_bytes);
    const int64_t n = std::max<int64_t>(1, g->n), m = std::max<int64_t>(1, g->m);
    const int64_t ntiles = std::max<int64_t>(1, ceil_div(g->n, RANK_TILE));
    SelLayout l;
    int64_t total = 0;
    for (int k = 0; k <= NCLASS; ++k) l.cb.lo[k] = CLASS_LO[k];
    for (int k = 0; k < NCLASS; ++k) {
        // rows in class k have degree > lo[k]: at most 2m / (lo[k] + 1) of them
        const int64_t cap = std::min<int64_t>(n, ceil_div(2 * m, CLASS_LO[k] + 1));
        l.cb.off[k] = total;
        total += cap;
    }
    l.lists = c.take<int32_t>(total);
    l.cnt = c.take<unsigned int>(NCLASS);
    l.plan = c.take<long long>(n + ntiles);
    l.tile_waves = c.take<unsigned int>(ntiles);
    l.plan_count = c.take<unsigned int>(1);
    const size_t nblk = scan_scratch_blocks(ntiles);
    l.scan.blk_v = c.take<unsigned int>(nblk);
    l.scan.blk_w = c.take<unsigned long long>(nblk);
    l.scan.total_w = c.take<unsigned long long>(1);
    l.recs = c.take<uint4>(2 * m);
    l.G = c.take<unsigned long long>(m);
    l.G2 = both ? c.take<unsigned long long>(m) : nullptr;
    l.cand_cap = std::min<int64_t>(m, std::max<int64_t>(1 << 16, m / 16));
    l.cand = c.take<unsigned long long>(l.cand_cap);
    l.cand2 = both ? c.take<unsigned long long>(l.cand_cap) : nullptr;
    l.cand_n = c.take<unsigned long long>(2);
    l.fit_part = c.take<unsigned long long>(4 * (size_t)COUNT_BLOCKS);
    l.hist = c.take<unsigned int>(2 * NBINS);
    l.state = c.take<unsigned long long>(4);
    l.counts = c.take<unsigned long long>(6);
    l.tabs = c.take<int32_t>(4 * ((size_t)g->d_max + 1));
    l.logs = c.take<double>(2 * ((size_t)g->d_max + 2));
    l.hub = HubScratch{};
    if (g->d_max > SORT_CAP) {
        // at most 2m entries lie in long rows; a row of degree d has at most
        // ceil(d / HUB_BUCKET) buckets, and there are at most 2m / (SORT_CAP + 1) such rows
        l.hub.cap = ceil_div(2 * m, HUB_BUCKET) + ceil_div(2 * m, SORT_CAP + 1) + 1;
        l.hub.key = c.take<unsigned long long>(2 * m);
        l.hub.pos = c.take<uint32_t>(2 * m);
        l.hub.bk_row = c.take<int32_t>(l.hub.cap);
        l.hub.bk_off = c.take<uint32_t>(l.hub.cap);
        l.hub.bk_cnt = c.take<uint32_t>(l.hub.cap);
        l.hub.nbk = c.take<unsigned int>(1);
    }
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

// Budget of a vertex of degree d (Algorithm 3): floor(d^e), at least 1 and
// at most d.
static inline int64_t budget_of(int64_t d, double e) {
    const double p = floor(pow((double)d, e));
    int64_t c = (int64_t)p;
    if (c < 1) c = 1;
    if (c > d) c = d;
    return c;
}

// budget_of for d = 0 .. d_max (0 for d = 0).  The budget is a
// non-decreasing step function of d (pow(d, e) is increasing in d, and for
// the degrees and exponents at which the budget can change the steps of
// pow's argument are far above its rounding), so the table is filled step
// by step: the end of the step at value c is predicted from (c + 1)^(1/e)
// and confirmed with budget_of itself around the prediction.  Every entry
// equals budget_of(d, e) under that monotonicity.
static void budget_fill(int32_t d_max, double e, int32_t *t) {
    t[0] = 0;
    int64_t d = 1;
    int64_t c = d_max >= 1 ? budget_of(1, e) : 0;
    while (d <= d_max) {
        int64_t last = d, next = -1;          // next: budget_of(last + 1) when already known
        if (c < d && e > 0.0) {
            const double edge = pow((double)(c + 1), 1.0 / e);
            int64_t guess = edge >= (double)d_max ? (int64_t)d_max : (int64_t)edge;
            if (guess < d) guess = d;
            if (budget_of(guess, e) == c) {
                last = guess;
                while (last < d_max) {
                    const int64_t b = budget_of(last + 1, e);
                    if (b != c) {
                        next = b;
                        break;
                    }
                    ++last;
                }
            } else {
                last = guess - 1;
                while (last > d && budget_of(last, e) != c) --last;
            }
        } else if (c < d) {                 // e == 0: every budget is 1
            last = d_max;
        }
        for (int64_t q = d; q <= last; ++q) t[q] = (int32_t)c;
        d = last + 1;
        if (d <= d_max) c = next >= 0 ? next : budget_of(d, e);
    }
}

static void budget_table(int32_t d_max, double e, std::vector<int32_t> &t) {
    t.assign((size_t)d_max + 1, 0);
    budget_fill(d_max, e, t.data());
}

// Rank every entry of every row and emit per `em`.
// Helper streams for the ranking classes.  The classes rank disjoint rows
// (their outputs are distinct side records or set-only keep flags), and the long
// classes are latency-bound (one workgroup sorts one row), so outside stream
// capture they run beside the short rows on three more streams of the same
// (default) priority, forked from and joined back into the caller's stream
// with events.  Created once per device; the mutex keeps one fork/join
// sequence's records and waits together when several host threads rank.
struct RankFork {
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
    bool ok = false;
    std::mutex mu;
};

static RankFork *rank_fork() {
    static RankFork forks[MAX_DEVICES];
    static std::once_flag once[MAX_DEVICES];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    RankFork *f = &forks[dev];
    std::call_once(once[dev], [f]() {
        bool ok = hipEventCreateWithFlags(&f->fork, hipEventDisableTiming) == hipSuccess;
        for (int h = 0; h < 3 && ok; ++h) {
            ok = hipStreamCreateWithFlags(&f->side[h], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&f->join[h], hipEventDisableTiming) == hipSuccess;
        }
        if (!ok) (void)hipGetLastError();
        f->ok = ok;
    });
    return f->ok ? f : nullptr;
}

template <typename Tr>
static ad_status rank_all(const ad_graph *g, const Tr *rho, const Emit &em, const SelLayout &L, hipStream_t st,
                          const unsigned long long *keys = nullptr, const float *rho_ent = nullptr) {
    const int64_t n = g->n;
    if (n <= 0 || g->m <= 0) return AD_OK;
    TraceScope trace("k_rank", st);
    ad_status s;
    // FP32 rows above 64: classify first, then fork the classes off
    RankFork *fk = nullptr;
    std::unique_lock<std::mutex> hold;
    hipStream_t cls[3] = {st, st, st};
    if (sizeof(Tr) == 4 && g->d_max > 64) {
        s = fill_i32((int32_t *)L.cnt, 0, NCLASS, st);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_classify, dim3(grid_for(n, SBLOCK)), dim3(SBLOCK), 0, st, n, g->row_ptr, L.cb, L.lists,
                           L.cnt);
        AD_LAUNCH_CHECK("k_classify");
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone) fk = rank_fork();
        else (void)hipGetLastError();
        if (fk) {
            hold = std::unique_lock<std::mutex>(fk->mu);
            AD_HIP(hipEventRecord(fk->fork, st));
            for (int h = 0; h < 3; ++h) {
                AD_HIP(hipStreamWaitEvent(fk->side[h], fk->fork, 0));
                cls[h] = fk->side[h];
            }
        }
    }
    // rows of degree <= 64, packed into waves
    const int64_t ntiles = ceil_div(n, RANK_TILE);
    hipLaunchKernelGGL(k_rank_plan, dim3(grid_for(ntiles, SBLOCK)), dim3(SBLOCK), 0, st, n, g->row_ptr, 0,
                       L.tile_waves, L.plan);
    AD_LAUNCH_CHECK("k_rank_plan");
    s = scan_exclusive(ntiles, L.tile_waves, nullptr, L.plan_count, nullptr, L.scan, st);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_rank_plan, dim3(grid_for(ntiles, SBLOCK)), dim3(SBLOCK), 0, st, n, g->row_ptr, 1,
                       L.tile_waves, L.plan);
    AD_LAUNCH_CHECK("k_rank_plan");
    const unsigned packed_blocks = (unsigned)std::min<int64_t>(4096, ceil_div(n, SBLOCK / WAVE));
    hipLaunchKernelGGL((k_rank_packed<Tr>), dim3(packed_blocks), dim3(SBLOCK), 0, st, L.plan, L.plan_count,
                       g->row_ptr, g->col, g->eid, g->orig_id, g->col_orig, rho, keys, em, rho_ent);
    AD_LAUNCH_CHECK("k_rank_packed");
    if (g->d_max <= 64) return AD_OK;

    if (sizeof(Tr) != 4) {
        s = fill_i32((int32_t *)L.cnt, 0, NCLASS, st);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_classify, dim3(grid_for(n, SBLOCK)), dim3(SBLOCK), 0, st, n, g->row_ptr, L.cb, L.lists,
                           L.cnt);
        AD_LAUNCH_CHECK("k_classify");
    }
    const unsigned grid = (unsigned)std::min<int64_t>(2048, n);
    const int32_t *lst[NCLASS];
    for (int k = 0; k < NCLASS; ++k) lst[k] = L.lists + L.cb.off[k];
    if (sizeof(Tr) == 4) {
        const float *rf = (const float *)rho;
#define AD_RANK_ARGS_F g->row_ptr, g->col, g->eid, g->orig_id, g->col_orig, rf, keys, em
        // the longest rows first on their streams: their latency is the tail.
        // Distance keys: radix sorts of the 32-bit distance bits; the caller's
        // own 64-bit keys: bitonic sorts of the keys.
        if (!keys) {
            // one-wave workgroups for rows up to 512: more of them in flight
            const unsigned grid_w = (unsigned)std::min<int64_t>(8192, n);
#define AD_RANK_ARGS_R g->row_ptr, g->col, g->eid, g->orig_id, g->col_orig, rf, rho_ent, em
            // The classes' costs follow their entry counts, which differ by
            // graph (a power-law graph holds most long-row entries in its few
            // hundred longest rows, R-MAT spreads them over every class).  The
            // longest sorted class is split in two slices on two streams (its
            // 512-thread workgroups need most of a compute unit and wait for
            // room beside the other classes' work), and the rest spread so that
            // neither kind of graph piles its work on one stream; the bucket
            // partition follows the packed short rows on the caller's stream.
            if (g->d_max > 4096) {
                hipLaunchKernelGGL((k_rank_radix<512, 16>), dim3(grid), dim3(512), 0, cls[0], lst[6], &L.cnt[6],
                                   AD_RANK_ARGS_R, 0, 2);
                hipLaunchKernelGGL((k_rank_radix<512, 16>), dim3(grid), dim3(512), 0, cls[1], lst[6], &L.cnt[6],
                                   AD_RANK_ARGS_R, 1, 2);
            }
            if (g->d_max > 2048)
                hipLaunchKernelGGL((k_rank_radix<512, 8>), dim3(grid), dim3(512), 0, cls[2], lst[5], &L.cnt[5],
                                   AD_RANK_ARGS_R, 0, 1);
            if (g->d_max > 1024)
                hipLaunchKernelGGL((k_rank_radix<256, 8>), dim3(grid), dim3(256), 0, cls[0], lst[4], &L.cnt[4],
                                   AD_RANK_ARGS_R, 0, 1);
            if (g->d_max > 64)
                hipLaunchKernelGGL((k_rank_radix<64, 2>), dim3(grid_w), dim3(64), 0, cls[1], lst[0], &L.cnt[0],
                                   AD_RANK_ARGS_R, 0, 1);
            if (g->d_max > 512)
                hipLaunchKernelGGL((k_rank_radix<256, 4>), dim3(grid), dim3(256), 0, cls[2], lst[3], &L.cnt[3],
                                   AD_RANK_ARGS_R, 0, 1);
            if (g->d_max > 256)
                hipLaunchKernelGGL((k_rank_radix<64, 8>), dim3(grid_w), dim3(64), 0, cls[2], lst[2], &L.cnt[2],
                                   AD_RANK_ARGS_R, 0, 1);
            // 128..256 after the first half of the longest class, or, with no
            // rows for the bucket partition, after the short rows on the
            // caller's stream
            if (g->d_max > 128)
                hipLaunchKernelGGL((k_rank_radix<64, 4>), dim3(grid_w), dim3(64), 0,
                                   g->d_max > SORT_CAP ? cls[0] : st, lst[1], &L.cnt[1], AD_RANK_ARGS_R, 0, 1);
            AD_LAUNCH_CHECK("k_rank_radix");
#undef AD_RANK_ARGS_R
        } else {
            if (g->d_max > 4096)
                hipLaunchKernelGGL((k_rank_bitonic<8192, 1024>), dim3(grid), dim3(1024), 0, cls[0], lst[6], &L.cnt[6],
                                   AD_RANK_ARGS_F);
            if (g->d_max > 2048)
                hipLaunchKernelGGL((k_rank_bitonic<4096, 512>), dim3(grid), dim3(512), 0, cls[1], lst[5], &L.cnt[5],
                                   AD_RANK_ARGS_F);
            if (g->d_max > 1024)
                hipLaunchKernelGGL((k_rank_bitonic<2048, 256>), dim3(grid), dim3(256), 0, cls[2], lst[4], &L.cnt[4],
                                   AD_RANK_ARGS_F);
            if (g->d_max > 512)
                hipLaunchKernelGGL((k_rank_bitonic<1024, 256>), dim3(grid), dim3(256), 0, cls[1], lst[3], &L.cnt[3],
                                   AD_RANK_ARGS_F);
            AD_LAUNCH_CHECK("k_rank_bitonic");
            if (g->d_max > 256)
                hipLaunchKernelGGL((k_rank_wave<8>), dim3(grid), dim3(SBLOCK), 0, cls[2], lst[2], &L.cnt[2],
                                   AD_RANK_ARGS_F);
            if (g->d_max > 128)
                hipLaunchKernelGGL((k_rank_wave<4>), dim3(grid), dim3(SBLOCK), 0, cls[0], lst[1], &L.cnt[1],
                                   AD_RANK_ARGS_F);
            if (g->d_max > 64)
                hipLaunchKernelGGL((k_rank_wave<2>), dim3(grid), dim3(SBLOCK), 0, cls[2], lst[0], &L.cnt[0],
                                   AD_RANK_ARGS_F);
            AD_LAUNCH_CHECK("k_rank_wave");
        }
        // rows above SORT_CAP: the bucket partition (for caller keys once per
        // orientation, on a helper stream; for distance keys once, on the caller's stream)
        static_assert(HUB_CLASS == 7 && SORT_CAP == 8192, "bitonic classes end where the bucket partition starts");
#undef AD_RANK_ARGS_F
        if (g->d_max > SORT_CAP && !keys) {
            // distance keys: one partition on the 32-bit distance bits serves both orders
            s = fill_i32((int32_t *)L.hub.nbk, 0, 1, st);
            if (s != AD_OK) return s;
            for (int k = HUB_CLASS; k < NCLASS; ++k) {
                if (g->d_max <= CLASS_LO[k]) break;
                hipLaunchKernelGGL(k_hub_partition<uint32_t>, dim3(512), dim3(HUB_TB), 0, st, lst[k], &L.cnt[k],
                                   g->row_ptr, g->col, g->eid, g->orig_id, g->col_orig, rf, rho_ent, keys, em.orient,
                                   L.hub);
                AD_LAUNCH_CHECK("k_hub_partition");
            }
            // buckets of up to 256 / 512 entries by sorts, larger ones by counting
            hipLaunchKernelGGL((k_hub_sort<4>), dim3(8192), dim3(WAVE), 0, st, g->row_ptr, g->col, g->eid,
                               g->orig_id, g->col_orig, em, L.hub, 0u);
            hipLaunchKernelGGL((k_hub_sort<8>), dim3(8192), dim3(WAVE), 0, st, g->row_ptr, g->col, g->eid,
                               g->orig_id, g->col_orig, em, L.hub, 4u * WAVE);
            AD_LAUNCH_CHECK("k_hub_sort");
            hipLaunchKernelGGL(k_hub_rank32, dim3(2048), dim3(SBLOCK), 0, st, g->row_ptr, g->col, g->eid,
                               g->orig_id, g->col_orig, em, L.hub, 8u * WAVE);
            AD_LAUNCH_CHECK("k_hub_rank32");
            hipLaunchKernelGGL(k_hub_emit, dim3(2048), dim3(SBLOCK), 0, st, g->row_ptr, g->col, g->eid, em, L.hub);
            AD_LAUNCH_CHECK("k_hub_emit");
        } else if (g->d_max > SORT_CAP) {
            // caller keys carry one orientation: one partition per orientation asked for
            for (int pass = 0; pass < (em.both ? 2 : 1); ++pass) {
                Emit one = em;
                one.both = 0;
                if (em.both) {
                    one.orient = pass == 0 ? AD_LOCAL : AD_GLOBAL;
                    if (pass == 1) {
                        one.budget = em.budget2;
                        one.keep = em.keep2;
                    }
                }
                if (em.mode != MODE_FIXED) one.mode = (em.both && pass == 1) ? MODE_REC_G : MODE_REC_L;
                s = fill_i32((int32_t *)L.hub.nbk, 0, 1, cls[2]);
                if (s != AD_OK) return s;
                for (int k = HUB_CLASS; k < NCLASS; ++k) {
                    if (g->d_max <= CLASS_LO[k]) break;
                    hipLaunchKernelGGL(k_hub_partition<unsigned long long>, dim3(512), dim3(HUB_TB), 0, cls[2], lst[k], &L.cnt[k],
                                       g->row_ptr, g->col, g->eid, g->orig_id, g->col_orig, rf, nullptr, keys,
                                       one.orient, L.hub);
                    AD_LAUNCH_CHECK("k_hub_partition");
                }
                hipLaunchKernelGGL(k_hub_rank, dim3(2048), dim3(SBLOCK), 0, cls[2], g->row_ptr, g->col, g->eid, one,
                                   L.hub);
                AD_LAUNCH_CHECK("k_hub_rank");
            }
        }
        if (fk) {
            // join: the caller's stream waits for the three class streams
            for (int h = 0; h < 3; ++h) {
                AD_HIP(hipEventRecord(fk->join[h], fk->side[h]));
                AD_HIP(hipStreamWaitEvent(st, fk->join[h], 0));
            }
        }
    } else {
        for (int k = 0; k < NCLASS; ++k) {
            if (g->d_max <= CLASS_LO[k]) break;
            hipLaunchKernelGGL((k_rank_count<Tr>), dim3(grid), dim3(SBLOCK), 0, st, lst[k], &L.cnt[k],
                               g->row_ptr, g->col, g->eid, g->orig_id, g->col_orig, rho, em);
            AD_LAUNCH_CHECK("k_rank_count");
        }
    }
    return AD_OK;
}

static Emit emit_single(int mode, int orient, const int32_t *budget, uint8_t *keep, uint4 *recs) {
    Emit em{};
    em.mode = mode;
    em.orient = orient;
    em.both = 0;
    em.budget = budget;
    em.keep = keep;
    em.recs = recs;
    return em;
}

static ad_status check_sel_args(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                                uint8_t *keep, int64_t *n_kept, void *ws, size_t ws_bytes, SelLayout *L,
                                bool both = false) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (rho_dtype != AD_F32 && rho_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "rho must be F32 or F64");
    if (orient != AD_LOCAL && orient != AD_GLOBAL) return fail(AD_ERR_INVALID_ARG, "unknown orientation");
    if (g->m > 0 && (!rho || !keep)) return fail(AD_ERR_INVALID_ARG, "rho or keep is NULL");
    if (!n_kept) return fail(AD_ERR_INVALID_ARG, "n_kept is NULL");
    if (g->m > 0 && g->d_max <= 0) return fail(AD_ERR_INVALID_ARG, "d_max must be set for selection");
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (sel_layout(g, ws, ws_bytes, L, both) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    return AD_OK;
}

}  // namespace ad

using namespace ad;

namespace ad {

// Rows longer than this are cut into DIST_SEG-entry work items.
constexpr int64_t DIST_HUB = 4096;

static SweepShape dist_shape(int R, ad_dtype x_dtype, int64_t d_max, bool whole_rows) {
    // the sweep's lane layout for this vector width, rows per wave sized by
    // the upper entries (or the whole rows); rows longer than DIST_HUB (when
    // the graph has any) go to the hub workgroups
    SweepShape sh = sweep_shape(R, x_dtype == AD_F64 ? 8 : 4, 0, 0);
    sh.hub_d = (d_max > DIST_HUB) ? DIST_HUB : ((int64_t)1 << 62);
    sh.upper_only = whole_rows ? 0 : 1;
    return sh;
}

size_t edge_dist_segs_workspace(const ad_graph *g, const Segs &sg) {
    return sweep_plan_bytes(g->n, sg.tile_off ? sg.ntiles : ceil_div(g->n, PLAN_TILE));
}

ad_status edge_dist_segs(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x, const double *minmax,
                         ad_dtype rho_dtype, void *rho, void *ws, size_t ws_bytes, const Segs &sg,
                         hipStream_t stream, float *rho_ent) {
    Carver c(ws, ws_bytes);
    SweepPlan pl;
    sweep_plan_carve(c, g->n, sg.tile_off ? sg.ntiles : ceil_div(g->n, PLAN_TILE), pl);
    if (!c.ok()) return fail(AD_ERR_WORKSPACE, "workspace too small");
    if (g->n <= 0 || g->m <= 0) return AD_OK;
    // FP64 vectors with FP32 distances (the FP64 tail of FP32 storage) take
    // the FP32 lane layout: four values, 32 bytes, per lane
    if (rho_ent && rho_dtype != AD_F32) return fail(AD_ERR_INTERNAL, "entry-ordered distances are FP32");
    pl.sh = dist_shape(R, (x_dtype == AD_F64 && rho_dtype == AD_F32) ? AD_F32 : x_dtype, g->d_max, rho_ent != nullptr);
    const bool hubs = g->d_max > DIST_HUB;
    ad_status s = sweep_plan_build(g, pl, hubs, sg, stream);
    if (s != AD_OK) return s;
    // hub work items: (rows longer than DIST_HUB) x (segments of the longest row)
    int64_t hub_segs = 1, hub_blocks = 0;
    if (hubs) {
        hub_segs = ceil_div(g->d_max, DIST_SEG);
        const int64_t busy = ceil_div(2 * g->m, DIST_SEG) + ceil_div(2 * g->m, DIST_HUB + 1);
        hub_blocks = round_up_xcds(std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(busy, SBLOCK / WAVE))));
    }
    const unsigned nb = (unsigned)(std::min<int64_t>(4096, ceil_div(g->n, SBLOCK / WAVE)) + hub_blocks);
    TraceScope trace("k_edge_dist", stream);
#define AD_DIST_ALL(TX, TR, V, ALL)                                                                         \
    hipLaunchKernelGGL((k_edge_dist<TX, TR, V, dist_unroll<TX>(), ALL>), dim3(nb), dim3(SBLOCK), 0, stream,  \
                       g->n, g->row_ptr, g->col, g->eid, (const TX *)x, minmax, (TR *)rho, (TR *)rho_ent, R,  \
                       pl.sh.C, pl.sh.SPRW, pl.sh.hub_d, (int)hub_blocks, hub_segs, pl.hub_list, pl.hub_count, \
                       pl.plan, pl.plan_count, pl.splits, pl.xcd_groups, sg.row_graph)
#define AD_DIST(TX, TR, V)                   \
    do {                                     \
        if (rho_ent) AD_DIST_ALL(TX, TR, V, true); \
        else AD_DIST_ALL(TX, TR, V, false);  \
    } while (0)
    if (x_dtype == AD_F64 && rho_dtype == AD_F64) {
        if (pl.sh.vec == 2) AD_DIST_ALL(double, double, 2, false);   // rho_ent is FP32 only
        else AD_DIST_ALL(double, double, 1, false);
    } else if (x_dtype == AD_F64) {
        // FP64 vectors (the FP64 tail of FP32 storage), FP64 arithmetic, FP32 rho
        if (pl.sh.vec == 4) AD_DIST(double, float, 4);
        else if (pl.sh.vec == 2) AD_DIST(double, float, 2);
        else AD_DIST(double, float, 1);
    } else {
        if (pl.sh.vec == 4) AD_DIST(float, float, 4);
        else if (pl.sh.vec == 2) AD_DIST(float, float, 2);
        else AD_DIST(float, float, 1);
    }
#undef AD_DIST
#undef AD_DIST_ALL
    AD_LAUNCH_CHECK("k_edge_dist");
    return AD_OK;
}

// Algorithm 3 at fixed budgets: keep[] (zeroed first) for every edge of the
// (possibly packed) graph; no count.
ad_status sparsify_fixed(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                         const int32_t *budget, uint8_t *keep, void *ws, size_t ws_bytes, hipStream_t stream) {
    SelLayout L;
    if (sel_layout(g, ws, ws_bytes, &L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    if (g->m <= 0) return AD_OK;
    ad_status s = fill_u8(keep, 0, g->m, stream);
    if (s != AD_OK) return s;
    const Emit em = emit_single(MODE_FIXED, orient, budget, keep, nullptr);
    if (rho_dtype == AD_F32) return rank_all<float>(g, (const float *)rho, em, L, stream);
    return rank_all<double>(g, (const double *)rho, em, L, stream);
}

size_t sparsify_workspace(const ad_graph *g) { return sel_layout(g, nullptr, 0, nullptr); }

}  // namespace ad

using namespace ad;

extern "C" size_t ad_edge_dist_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK) return 0;
    return edge_dist_segs_workspace(g, Segs());
}

extern "C" ad_status ad_edge_dist(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                                  const double *minmax, ad_dtype rho_dtype, void *rho, void *ws, size_t ws_bytes,
                                  hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (R < 1 || R > 64) return fail(AD_ERR_INVALID_ARG, "R must be in [1, 64]");
    if (x_dtype != AD_F32 && x_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "x must be F32 or F64");
    if (rho_dtype != AD_F32 && rho_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "rho must be F32 or F64");
    if (rho_dtype == AD_F64 && x_dtype != AD_F64) return fail(AD_ERR_UNSUPPORTED, "FP64 rho needs FP64 x");
    if (g->m > 0 && (!x || !minmax || !rho)) return fail(AD_ERR_INVALID_ARG, "x, minmax or rho is NULL");
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    return edge_dist_segs(g, R, x_dtype, x, minmax, rho_dtype, rho, ws, ws_bytes, Segs(), stream);
}

extern "C" size_t ad_normalize_dist_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK) return 0;
    return (size_t)std::max<int64_t>(1, g->n) * sizeof(double) + 256;
}

extern "C" ad_status ad_normalize_dist(const ad_graph *g, ad_dtype rho_dtype, const void *rho, int32_t by_strength,
                                       double eps, void *rho_out, void *ws, size_t ws_bytes, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (rho_dtype != AD_F32 && rho_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "rho must be F32 or F64");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(AD_ERR_INVALID_ARG, "eps must be finite and >= 0");
    if (g->m > 0 && (!rho || !rho_out)) return fail(AD_ERR_INVALID_ARG, "rho or rho_out is NULL");
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < ad_normalize_dist_workspace_size(g)) return fail(AD_ERR_WORKSPACE, "workspace too small");
    if (g->n <= 0 || g->m <= 0) return AD_OK;
    double *f = (double *)ws;
    hipLaunchKernelGGL(k_vertex_weight, dim3(grid_for(ceil_div(g->n, SBLOCK / WAVE), 1)), dim3(SBLOCK), 0, stream,
                       g->n, g->row_ptr, g->w, by_strength ? 1 : 0, f);
    AD_LAUNCH_CHECK("k_vertex_weight");
    const int64_t nnz = 2 * g->m;
    const unsigned nb = grid_for(ceil_div(ceil_div(nnz, NORM_CHUNK), SBLOCK / WAVE), 1);
    if (rho_dtype == AD_F32)
        hipLaunchKernelGGL((k_normalize<float>), dim3(nb), dim3(SBLOCK), 0, stream, g->n, nnz, g->row_ptr, g->col,
                           g->eid, f, (const float *)rho, eps, (float *)rho_out);
    else
        hipLaunchKernelGGL((k_normalize<double>), dim3(nb), dim3(SBLOCK), 0, stream, g->n, nnz, g->row_ptr, g->col,
                           g->eid, f, (const double *)rho, eps, (double *)rho_out);
    AD_LAUNCH_CHECK("k_normalize");
    return AD_OK;
}

extern "C" ad_status ad_budget_table(int32_t d_max, double e, int32_t *budget_host) {
    if (d_max < 0) return fail(AD_ERR_INVALID_ARG, "negative d_max");
    if (!(e >= 0.0 && e <= 1.0)) return fail(AD_ERR_INVALID_ARG, "e must be in [0, 1]");
    if (!budget_host) return fail(AD_ERR_INVALID_ARG, "budget_host is NULL");
    std::vector<int32_t> t;
    budget_table(d_max, e, t);
    std::copy(t.begin(), t.end(), budget_host);
    return AD_OK;
}

extern "C" size_t ad_sparsify_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK) return 0;
    return sel_layout(g, nullptr, 0, nullptr);
}

// Algorithm 3 at fixed budgets with the count (ad_sparsify's work); rho_ent,
// when given, holds the FP32 distances in CSR entry order.
static ad_status sparsify_count(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                                const int32_t *budget, uint8_t *keep, int64_t *n_kept, const SelLayout &L,
                                hipStream_t stream, const float *rho_ent = nullptr) {
    ad_status s = fill_u64(L.counts, 0, 1, stream);
    if (s != AD_OK) return s;
    if (g->m > 0) {
        s = fill_u8(keep, 0, g->m, stream);
        if (s != AD_OK) return s;
        const Emit em = emit_single(MODE_FIXED, orient, budget, keep, nullptr);
        if (rho_dtype == AD_F32)
            s = rank_all<float>(g, (const float *)rho, em, L, stream, nullptr, rho_ent);
        else
            s = rank_all<double>(g, (const double *)rho, em, L, stream);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_count_bytes, dim3((unsigned)std::min<int64_t>(SUM_BLOCKS, ceil_div(g->m, SBLOCK))),
                           dim3(SBLOCK), 0, stream, g->m, keep,
                           L.counts);
        AD_LAUNCH_CHECK("k_count_bytes");
    }
    hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, stream, L.counts, n_kept);
    AD_LAUNCH_CHECK("k_store_count");
    return AD_OK;
}

extern "C" ad_status ad_sparsify(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                                 const int32_t *budget, uint8_t *keep, int64_t *n_kept, void *ws,
                                 size_t ws_bytes, hipStream_t stream) {
    SelLayout L;
    ad_status s = check_sel_args(g, rho_dtype, rho, orient, keep, n_kept, ws, ws_bytes, &L);
    if (s != AD_OK) return s;
    if (g->m > 0 && !budget) return fail(AD_ERR_INVALID_ARG, "budget is NULL");
    return sparsify_count(g, rho_dtype, rho, orient, budget, keep, n_kept, L, stream);
}

// Fewest kept edges meeting the target, in the bisection's own test
// (kept / m >= target).
static int64_t fit_count_target(int64_t m, double target) {
    int64_t K = (int64_t)ceil(target * (double)m);
    if (K < 1) K = 1;
    if (K > m) K = m;
    while (K > 1 && (double)(K - 1) / (double)m >= target) --K;
    while (K < m && (double)K / (double)m < target) ++K;
    return K;
}

namespace ad {

// Pinned host staging for the fit's read-backs (the first STAGE_RB 32-bit
// words) and budget tables (grown on demand, kept for the life of the
// process; one fit at a time uses it).  Mapped into the device's address
// space, so that a kernel copies the tables in stream order.
constexpr size_t STAGE_RB = 32;
static std::mutex g_stage_mu;
static int32_t *g_stage = nullptr;
static size_t g_stage_cap = 0;

static ad_status stage_reserve(size_t count) {
    if (count <= g_stage_cap) return AD_OK;
    if (g_stage) AD_HIP(hipHostFree(g_stage));
    g_stage = nullptr;
    g_stage_cap = 0;
    AD_HIP(hipHostMalloc((void **)&g_stage, count * sizeof(int32_t), hipHostMallocMapped));
    g_stage_cap = count;
    return AD_OK;
}

// From the side records (nfit <= 2 fitted orientations: the first rank, and
// the second when both are fitted): the per-edge threshold grid index, the
// radix select of the K-th smallest, and the exact confirmation with budget
// tables (count at the grid point >= K, count one grid step lower < K).  The
// orientations share every launch and every read-back: one after the
// selects, one per confirmation round.  Writes keep[o], the device counts
// n_kept[o] and the exponents.  L.logs must hold the log table.
static ad_status fit_from_recs(const ad_graph *g, const SelLayout &L, int nfit, int64_t K, uint8_t *const *keep,
                               int64_t *n_kept, double *e_used_host, hipStream_t stream) {
    const int64_t m = g->m;
    const size_t tl = (size_t)g->d_max + 1;
    ad_status s;
    const unsigned hist_blocks = (unsigned)std::min<int64_t>(HIST_BLOCKS, ceil_div(m, (int64_t)SBLOCK * FIT_U));
    const unsigned count_blocks = (unsigned)std::min<int64_t>(COUNT_BLOCKS, ceil_div(m, (int64_t)SBLOCK * 2 * FIT_U));
    const FitArrays fa{{L.G, L.G2}, {L.hist, L.hist + NBINS}};
    const CandArrays cs{{L.cand, L.cand2}, L.cand_n, L.cand_cap};
    std::lock_guard<std::mutex> lock(g_stage_mu);
    s = stage_reserve(STAGE_RB + 4 * tl);
    if (s != AD_OK) return s;
    unsigned long long *const rb = reinterpret_cast<unsigned long long *>(g_stage);   // read-backs
    int32_t *const tabs_h = g_stage + STAGE_RB;
    int32_t *stage_dev = nullptr;
    AD_HIP(hipHostGetDevicePointer((void **)&stage_dev, g_stage, 0));
    const int32_t *const tabs_mapped = stage_dev + STAGE_RB;   // tabs_h as the device sees it
    hipLaunchKernelGGL(k_select_init, dim3(1), dim3(SBLOCK), 0, stream, L.state, (unsigned long long)K, nfit,
                       L.hist, L.cand_n, L.counts);
    AD_LAUNCH_CHECK("k_select_init");
    const int64_t nlogs = (int64_t)g->d_max + 2;
    int dev = 0, lds_max = 0, n_cu = 0;
    const bool lds_tab = hipGetDevice(&dev) == hipSuccess &&
                         hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                         hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                         (int64_t)lds_max >= 2 * nlogs * (int64_t)sizeof(double) + 2 * NBINS * 4 + 1024;
    if (lds_tab) {
        const unsigned blocks = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>(n_cu, ceil_div(m, (int64_t)FIT_LDS_TB * FIT_U)));
        hipLaunchKernelGGL((k_fit_grid<FIT_LDS_TB, true>), dim3(blocks), dim3(FIT_LDS_TB),
                           (size_t)(2 * nlogs) * sizeof(double), stream, m, L.recs, L.logs, nlogs, nfit, fa);
    } else {
        hipLaunchKernelGGL((k_fit_grid<SBLOCK, false>), dim3(hist_blocks), dim3(SBLOCK), 0, stream, m, L.recs,
                           L.logs, nlogs, nfit, fa);
    }
    AD_LAUNCH_CHECK("k_fit_grid");
    hipLaunchKernelGGL(k_radix_pick, dim3(nfit), dim3(SBLOCK), 0, stream, fa, L.state, DIGIT_WIDTH[0]);
    AD_LAUNCH_CHECK("k_radix_pick");
    for (int pass = 1; pass < NPASS; ++pass) {
        if (pass == 1)
            hipLaunchKernelGGL(k_radix_hist<true>, dim3(hist_blocks, nfit), dim3(SBLOCK), 0, stream, m, fa, cs,
                               DIGIT_SHIFT[pass], DIGIT_WIDTH[pass], L.state);
        else
            hipLaunchKernelGGL(k_radix_hist<false>, dim3(hist_blocks, nfit), dim3(SBLOCK), 0, stream, m, fa, cs,
                               DIGIT_SHIFT[pass], DIGIT_WIDTH[pass], L.state);
        AD_LAUNCH_CHECK("k_radix_hist");
        hipLaunchKernelGGL(k_radix_pick, dim3(nfit), dim3(SBLOCK), 0, stream, fa, L.state, DIGIT_WIDTH[pass]);
        AD_LAUNCH_CHECK("k_radix_pick");
    }
    AD_HIP(hipMemcpyAsync(rb, L.state, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipStreamSynchronize(stream));
    const unsigned long long GMAX = 1ull << 40;
    long long g_try[2];
    bool done[2] = {false, false};
    for (int o = 0; o < nfit; ++o) g_try[o] = (long long)std::min(rb[2 * o], GMAX);
    // The first check splits the count: the edges that the estimate settles are
    // counted while the host builds the budget tables, the listed rest after
    // the tables arrive.  Later checks (a moved grid point, or a list that
    // overflowed) count in one pass with the tables.
    bool split = true;
    const unsigned margin_blocks = (unsigned)std::min<int64_t>(64, ceil_div(2 * L.cand_cap, SBLOCK));
    for (int attempt = 0; attempt < 64; ++attempt) {
        // budget tables at the candidate grid point and one step below, filled
        // in the pinned staging buffer (one host thread per table for long rows)
        CountArgs ca{};
        std::vector<std::pair<int32_t *, double>> fills;
        for (int o = 0; o < nfit; ++o) {
            ca.tab_hi[o] = L.tabs + (2 * o) * tl;
            ca.tab_lo[o] = L.tabs + (2 * o + 1) * tl;
            ca.G[o] = o == 0 ? L.G : L.G2;
            ca.g_hi[o] = (unsigned long long)g_try[o];
            ca.keep[o] = keep[o];
            ca.keep_aligned[o] = ((uintptr_t)keep[o] & 3) == 0 ? 1 : 0;
            ca.active[o] = done[o] ? 0 : 1;
            ca.use_lo[o] = g_try[o] > 0 ? 1 : 0;
            ca.list[o] = reinterpret_cast<uint32_t *>(o == 0 ? L.cand : L.cand2);
            if (done[o]) continue;
            fills.emplace_back(tabs_h + (2 * o) * tl, (double)g_try[o] / GRID);
            if (g_try[o] > 0) fills.emplace_back(tabs_h + (2 * o + 1) * tl, (double)(g_try[o] - 1) / GRID);
        }
        ca.list_n = L.counts + 4;
        ca.list_cap = 2 * L.cand_cap;
        if (!split) {                        // the first check's counts were zeroed by k_select_init
            s = fill_u64(L.counts, 0, 6, stream);
            if (s != AD_OK) return s;
        }
        if (split) {
            hipLaunchKernelGGL(k_fit_count<true>, dim3(count_blocks), dim3(SBLOCK), 0, stream, m, L.recs, nfit, ca,
                               L.fit_part);
            AD_LAUNCH_CHECK("k_fit_count");
            hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(SBLOCK), 0, stream, L.fit_part, (int)count_blocks,
                               L.counts);
            AD_LAUNCH_CHECK("k_sum_counts");
        }
        std::vector<std::thread> th;
        size_t started = 0;                  // tables 1 .. started on their own threads
        if (g->d_max >= (1 << 16)) {
            try {
                while (started + 1 < fills.size()) {
                    const auto &f = fills[started + 1];
                    th.emplace_back(budget_fill, g->d_max, f.second, f.first);
                    ++started;
                }
            } catch (...) {                  // no thread: the rest on this one
            }
        }
        for (size_t f = 0; f < fills.size(); ++f)
            if (f == 0 || f > started) budget_fill(g->d_max, fills[f].second, fills[f].first);
        for (auto &x : th) x.join();
        // the tables to the device by a kernel reading the mapped staging (a
        // host-side copy call would wait for the stream's earlier work)
        const int64_t tab_words = (int64_t)(2 * nfit * tl);
        hipLaunchKernelGGL(k_copy_mapped, dim3(grid_for(tab_words, SBLOCK)), dim3(SBLOCK), 0, stream, L.tabs,
                           tabs_mapped, tab_words);
        AD_LAUNCH_CHECK("k_copy_mapped");
        if (split) {
            hipLaunchKernelGGL(k_fit_margin, dim3(margin_blocks, nfit), dim3(SBLOCK), 0, stream, L.recs, ca,
                               L.counts);
            AD_LAUNCH_CHECK("k_fit_margin");
        } else {
            hipLaunchKernelGGL(k_fit_count<false>, dim3(count_blocks), dim3(SBLOCK), 0, stream, m, L.recs, nfit, ca,
                               L.fit_part);
            AD_LAUNCH_CHECK("k_fit_count");
            hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(SBLOCK), 0, stream, L.fit_part, (int)count_blocks,
                               L.counts);
            AD_LAUNCH_CHECK("k_sum_counts");
        }
        unsigned long long *const hc = rb + 4;
        AD_HIP(hipMemcpyAsync(hc, L.counts, 6 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
        AD_HIP(hipStreamSynchronize(stream));
        bool overflow = false;
        for (int o = 0; o < nfit; ++o)
            if (split && !done[o] && hc[4 + o] > (unsigned long long)ca.list_cap) overflow = true;
        split = false;
        if (overflow) continue;              // the same points again, in one full pass
        bool all = true;
        for (int o = 0; o < nfit; ++o) {
            if (done[o]) continue;
            const bool hi_ok = (int64_t)hc[2 * o] >= K;
            const bool lo_ok = g_try[o] == 0 || (int64_t)hc[2 * o + 1] < K;
            if (hi_ok && lo_ok) {
                hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, stream, L.counts + 2 * o, n_kept + o);
                AD_LAUNCH_CHECK("k_store_count");
                e_used_host[o] = (double)g_try[o] / GRID;
                done[o] = true;
                continue;
            }
            all = false;
            if (!hi_ok) {
                if (g_try[o] >= (long long)GMAX) return fail(AD_ERR_INTERNAL, "retention fit found no grid point");
                ++g_try[o];
            } else {
                --g_try[o];
            }
        }
        if (all) return AD_OK;
    }
    return fail(AD_ERR_INTERNAL, "retention fit did not settle on a grid point");
}

// Both halves of the fitted sparsify: rank (one or both orientations) into
// side records, then the fits.
static ad_status sparsify_fit_impl(const ad_graph *g, ad_dtype rho_dtype, const void *rho, int orient, bool both,
                                   double target, uint8_t *keep, uint8_t *keep2, int64_t *n_kept,
                                   double *e_used_host, const SelLayout &L, hipStream_t stream,
                                   const float *rho_ent = nullptr) {
    const int64_t m = g->m;
    const int nfit = both ? 2 : 1;
    ad_status s;
    if (m == 0) {
        s = fill_u64(L.counts, 0, 4, stream);
        if (s != AD_OK) return s;
        for (int o = 0; o < nfit; ++o) {
            hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, stream, L.counts, n_kept + o);
            AD_LAUNCH_CHECK("k_store_count");
            e_used_host[o] = 0.0;
        }
        AD_HIP(hipStreamSynchronize(stream));
        return AD_OK;
    }
    const int64_t K = fit_count_target(m, target);
    Emit em = emit_single(MODE_REC, orient, nullptr, nullptr, L.recs);
    if (both) {
        em.orient = AD_LOCAL;
        em.both = 1;
    }
    if (rho_dtype == AD_F32)
        s = rank_all<float>(g, (const float *)rho, em, L, stream, nullptr, rho_ent);
    else
        s = rank_all<double>(g, (const double *)rho, em, L, stream);
    if (s != AD_OK) return s;
    TraceScope trace_fit("k_fit_select", stream);
    hipLaunchKernelGGL(k_log_table, dim3(grid_for((int64_t)g->d_max + 2, SBLOCK)), dim3(SBLOCK), 0, stream,
                       (int64_t)g->d_max + 2, L.logs);
    AD_LAUNCH_CHECK("k_log_table");
    uint8_t *kp[2] = {keep, keep2};
    return fit_from_recs(g, L, nfit, K, kp, n_kept, e_used_host, stream);
}

}  // namespace ad

extern "C" ad_status ad_sparsify_fit(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                                     double target, uint8_t *keep, int64_t *n_kept, double *e_used_host,
                                     void *ws, size_t ws_bytes, hipStream_t stream) {
    SelLayout L;
    ad_status s = check_sel_args(g, rho_dtype, rho, orient, keep, n_kept, ws, ws_bytes, &L);
    if (s != AD_OK) return s;
    if (!(target > 0.0 && target <= 1.0)) return fail(AD_ERR_INVALID_ARG, "target must be in (0, 1]");
    if (!e_used_host) return fail(AD_ERR_INVALID_ARG, "e_used_host is NULL");
    return sparsify_fit_impl(g, rho_dtype, rho, orient, false, target, keep, nullptr, n_kept, e_used_host, L,
                             stream);
}

extern "C" size_t ad_sparsify_fit_both_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK) return 0;
    return sel_layout(g, nullptr, 0, nullptr, true);
}

extern "C" ad_status ad_sparsify_fit_both(const ad_graph *g, ad_dtype rho_dtype, const void *rho, double target,
                                          uint8_t *keep_local, uint8_t *keep_global, int64_t *n_kept,
                                          double *e_used_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    SelLayout L;
    ad_status s = check_sel_args(g, rho_dtype, rho, AD_LOCAL, keep_local, n_kept, ws, ws_bytes, &L, true);
    if (s != AD_OK) return s;
    if (g->m > 0 && !keep_global) return fail(AD_ERR_INVALID_ARG, "keep_global is NULL");
    if (!(target > 0.0 && target <= 1.0)) return fail(AD_ERR_INVALID_ARG, "target must be in (0, 1]");
    if (!e_used_host) return fail(AD_ERR_INVALID_ARG, "e_used_host is NULL");
    return sparsify_fit_impl(g, rho_dtype, rho, AD_LOCAL, true, target, keep_local, keep_global, n_kept,
                             e_used_host, L, stream);
}

// ------------------------------------------- distance and selection, fused --
// One call for Algorithm 1's distances and Algorithm 3's selection: the
// distance pass visits whole rows and writes every CSR entry's distance in
// entry order beside rho (each edge's two entries get equal values), and the
// ranking reads its keys from that array, contiguously, instead of gathering
// rho by edge id.  Workspace: the distance plan, the entry-ordered distances
// and the selection workspace of both orders, each 256-byte aligned.
struct FusedLayout {
    void *dist_ws = nullptr;
    size_t dist_bytes = 0;
    float *rho_ent = nullptr;
    void *sel_ws = nullptr;
    size_t sel_bytes = 0;
};

static size_t fused_layout(const ad_graph *g, void *ws, FusedLayout *F) {
    const size_t dist = edge_dist_segs_workspace(g, Segs());
    const size_t ent = (size_t)std::max<int64_t>(1, 2 * g->m) * sizeof(float);
    const size_t sel = sel_layout(g, nullptr, 0, nullptr, true);
    if (dist == 0 || sel == 0) return 0;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t o1 = up(dist), o2 = up(o1 + ent);
    if (F) {
        F->dist_ws = ws;
        F->dist_bytes = dist;
        F->rho_ent = (float *)((char *)ws + o1);
        F->sel_ws = (char *)ws + o2;
        F->sel_bytes = sel;
    }
    return o2 + sel;
}

static ad_status check_fused_args(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                                  const double *minmax, void *rho, uint8_t *keep, int64_t *n_kept, void *ws,
                                  size_t ws_bytes, FusedLayout *F, SelLayout *L) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (R < 1 || R > 64) return fail(AD_ERR_INVALID_ARG, "R must be in [1, 64]");
    if (x_dtype != AD_F32 && x_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "x must be F32 or F64");
    if (g->m > 0 && (!x || !minmax || !rho || !keep)) return fail(AD_ERR_INVALID_ARG, "x, minmax, rho or keep is NULL");
    if (!n_kept) return fail(AD_ERR_INVALID_ARG, "n_kept is NULL");
    if (g->m > 0 && g->d_max <= 0) return fail(AD_ERR_INVALID_ARG, "d_max must be set for selection");
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    const size_t need = fused_layout(g, ws, F);
    if (need == 0 || ws_bytes < need) return fail(AD_ERR_WORKSPACE, "workspace too small");
    if (sel_layout(g, F->sel_ws, F->sel_bytes, L, true) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    return AD_OK;
}

extern "C" size_t ad_edge_dist_select_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK) return 0;
    return fused_layout(g, nullptr, nullptr);
}

extern "C" ad_status ad_edge_dist_sparsify(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                                           const double *minmax, float *rho, ad_orient orient,
                                           const int32_t *budget, uint8_t *keep, int64_t *n_kept, void *ws,
                                           size_t ws_bytes, hipStream_t stream) {
    FusedLayout F;
    SelLayout L;
    ad_status s = check_fused_args(g, R, x_dtype, x, minmax, rho, keep, n_kept, ws, ws_bytes, &F, &L);
    if (s != AD_OK) return s;
    if (orient != AD_LOCAL && orient != AD_GLOBAL) return fail(AD_ERR_INVALID_ARG, "unknown orientation");
    if (g->m > 0 && !budget) return fail(AD_ERR_INVALID_ARG, "budget is NULL");
    s = edge_dist_segs(g, R, x_dtype, x, minmax, AD_F32, rho, F.dist_ws, F.dist_bytes, Segs(), stream, F.rho_ent);
    if (s != AD_OK) return s;
    return sparsify_count(g, AD_F32, rho, orient, budget, keep, n_kept, L, stream, F.rho_ent);
}

extern "C" ad_status ad_edge_dist_fit_both(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                                           const double *minmax, float *rho, double target, uint8_t *keep_local,
                                           uint8_t *keep_global, int64_t *n_kept, double *e_used_host, void *ws,
                                           size_t ws_bytes, hipStream_t stream) {
    FusedLayout F;
    SelLayout L;
    ad_status s = check_fused_args(g, R, x_dtype, x, minmax, rho, keep_local, n_kept, ws, ws_bytes, &F, &L);
    if (s != AD_OK) return s;
    if (g->m > 0 && !keep_global) return fail(AD_ERR_INVALID_ARG, "keep_global is NULL");
    if (!(target > 0.0 && target <= 1.0)) return fail(AD_ERR_INVALID_ARG, "target must be in (0, 1]");
    if (!e_used_host) return fail(AD_ERR_INVALID_ARG, "e_used_host is NULL");
    s = edge_dist_segs(g, R, x_dtype, x, minmax, AD_F32, rho, F.dist_ws, F.dist_bytes, Segs(), stream, F.rho_ent);
    if (s != AD_OK) return s;
    return sparsify_fit_impl(g, AD_F32, rho, AD_LOCAL, true, target, keep_local, keep_global, n_kept, e_used_host,
                             L, stream, F.rho_ent);
}

// ---------------------------------------------------------------------------
// Sparsify with binning (Algorithm 4, SparsifyB; bin rule of Section 4).
//
// Readings (shared with the oracle, which is written separately):
//   - the values binned are the per-edge distances handed in; sigma is their
//     population standard deviation over N_i (two passes in double, rounded
//     to single precision so that the bins do not depend on summation
//     order), min and max are exact;
//   - h = (3.5 sigma) / cbrt(d_i) in double, with cbrt from the host's C
//     library (a table by degree); B_i = max(1, ceil((max - min) / h)) bins
//     (1 when h == 0); entry q falls in bin min(B_i - 1, floor((rho_q -
//     min) / h));
//   - random order: vertex i's 32-bit key K_i is the low half of word 0 of
//     Philox4x64-10 with key (seed, graph_id) and counter (orig_id[i], 0, 1,
//     0); neighbour j's priority is fmix32(orig_id[j] ^ K_i), fmix32 being
//     the 32-bit finalizer of MurmurHash3 (a bijection: priorities within a
//     row are distinct);
//   - selection: rounds r = 0, 1, ...; in each round the non-empty bins, in
//     increasing order of their smallest priority, give up their unselected
//     edge of smallest priority, until c_i = budget(d_i, e) edges are taken;
//     an edge is kept when either endpoint takes it.
//
// On the device the rounds become two rankings of 64-bit keys per row: first
// (bin, priority), whose rank p of an entry minus the rank of its bin's
// first entry is the entry's round r (the bins' first entries are read off
// the row laid out in that order); then (r, smallest priority of the bin),
// whose rank is the entry's place in the selection order.  The rank
// kernels of Algorithm 3 do both; the budget and the retention fit then
// apply unchanged (the selected sets grow with e).
// ---------------------------------------------------------------------------

namespace ad {

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Rows of degree <= BIN_SHORT_ROW are handled by groups of BIN_SHORT_G
// consecutive lanes (neighbouring lanes read neighbouring entries), longer
// rows by one wave each: every kernel below runs its row body over the
// short rows with groups of BIN_SHORT_G lanes, then over the long rows with
// groups of WAVE lanes (rows strided over the grid's groups, then its waves).
constexpr int64_t BIN_SHORT_ROW = 32;
constexpr int BIN_SHORT_G = 16;

template <int G>
__device__ __forceinline__ double group_sum(double v) {
    for (int o = G / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return __shfl(v, (int)(threadIdx.x & (WAVE - 1)) & ~(G - 1), WAVE);   // one value for the group
}
template <int G>
__device__ __forceinline__ double group_min(double v) {
    for (int o = G / 2; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, WAVE));
    return v;
}
template <int G>
__device__ __forceinline__ double group_max(double v) {
    for (int o = G / 2; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Runs body.template run<G>(row, lane in group) for every row with d >= 1:
// short rows with G = BIN_SHORT_G, long rows with G = WAVE.  All lanes of a
// wave take part in both passes (rows past n or of the other kind idle
// through the group's loops), so the group shuffles see full waves.
template <typename Body>
__device__ __forceinline__ void for_bin_rows(int64_t n, const int64_t *__restrict__ row_ptr, const Body &body) {
    constexpr int GS = BIN_SHORT_G;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & (WAVE - 1);
    // short rows: the wave's groups take rows g, g + ngroups, ... in lockstep
    for (int64_t base = (tid / WAVE) * (WAVE / GS); base < n; base += (nt / WAVE) * (WAVE / GS)) {
        const int64_t i = base + lane / GS;
        const int64_t d = i < n ? row_ptr[i + 1] - row_ptr[i] : 0;
        body.template run<GS>(i, lane % GS, d >= 1 && d <= BIN_SHORT_ROW);
    }
    for (int64_t i = tid / WAVE; i < n; i += nt / WAVE) {
        const int64_t d = row_ptr[i + 1] - row_ptr[i];
        if (d > BIN_SHORT_ROW) body.template run<WAVE>(i, lane, true);
    }
}

// Per row: bins by Scott's rule and the first key (bin << 32 | priority) of
// every entry.
template <typename Tr>
struct BinKeys {
    const int64_t *row_ptr;
    const int32_t *col, *eid, *orig_id, *col_orig;
    const Tr *rho;
    const double *cbrt_tab;
    int64_t d_max;
    uint64_t seed, graph_id;
    unsigned long long *keys;
    template <int G>
    __device__ __forceinline__ void run(int64_t i, int lane, bool on) const {
        const int64_t beg = on ? row_ptr[i] : 0, d = on ? row_ptr[i + 1] - beg : 0;
        double mn = INFINITY, mx = -INFINITY, sum = 0.0;
        for (int64_t q = lane; q < d; q += G) {
            const double v = (double)rho[eid[beg + q]];
            mn = fmin(mn, v);
            mx = fmax(mx, v);
            sum += v;
        }
        mn = group_min<G>(mn);
        mx = group_max<G>(mx);
        sum = group_sum<G>(sum);
        const double mean = d > 0 ? sum / (double)d : 0.0;
        double ss = 0.0;
        for (int64_t q = lane; q < d; q += G) {
            const double t = (double)rho[eid[beg + q]] - mean;
            ss += t * t;
        }
        ss = group_sum<G>(ss);
        if (!on) return;
        const double sigma = (double)(float)sqrt(ss / (double)d);
        // (rows longer than d_max break the graph's contract; they are kept in bounds)
        const double h = (3.5 * sigma) / (d <= d_max ? cbrt_tab[d] : cbrt((double)d));
        int64_t nb = 1;
        if (h > 0.0) {
            const double k = ceil((mx - mn) / h);
            nb = k < 1.0 ? 1 : (int64_t)k;
            if (nb > d) nb = d;    // never binds: (max - min) / sigma <= sqrt(2 d)
        }
        uint64_t words[4];
        philox4x64_10((uint64_t)(uint32_t)(orig_id ? orig_id[i] : (int32_t)i), 0, 1, 0, seed, graph_id, words);
        const uint32_t K = (uint32_t)words[0];
        for (int64_t q = lane; q < d; q += G) {
            const int64_t p = beg + q;
            const double v = (double)rho[eid[p]];
            int64_t b = 0;
            if (h > 0.0) {
                b = (int64_t)floor((v - mn) / h);
                if (b > nb - 1) b = nb - 1;
            }
            const uint32_t u = fmix32((uint32_t)nbr_id(p, col[p], col_orig, orig_id) ^ K);
            keys[p] = ((unsigned long long)b << 32) | u;
        }
    }
};

template <typename Tr>
__global__ __launch_bounds__(SBLOCK) void k_bin_keys(int64_t n, BinKeys<Tr> body) {
    for_bin_rows(n, body.row_ptr, body);
}

// Rank in the (bin, priority) order of an entry, from the side records
// written by the first ranking (word 1 of recs[2e + (i > j)]).
__device__ __forceinline__ uint32_t side_rank(const uint4 *__restrict__ recs, int32_t e, int64_t i, int32_t j) {
    return recs[2 * (int64_t)e + (i > j ? 1 : 0)].y;
}

// The row in (bin, priority) order: order[beg + rank] = entry offset, and
// every entry's rank.
struct BinOrder {
    const int64_t *row_ptr;
    const int32_t *col, *eid;
    const uint4 *recs;
    uint32_t *order, *rank;
    template <int G>
    __device__ __forceinline__ void run(int64_t i, int lane, bool on) const {
        if (!on) return;
        const int64_t beg = row_ptr[i], d = row_ptr[i + 1] - beg;
        for (int64_t q = lane; q < d; q += G) {
            const uint32_t r = side_rank(recs, eid[beg + q], i, col[beg + q]);
            order[beg + r] = (uint32_t)q;
            rank[beg + q] = r;
        }
    }
};

// Each bin's first entry in that order: its rank (first_pos) and priority
// (first_u), at the row's bin slots [beg, beg + B_i).
struct BinFirsts {
    const int64_t *row_ptr;
    const unsigned long long *keys;
    const uint32_t *order;
    uint32_t *first_u, *first_pos;
    template <int G>
    __device__ __forceinline__ void run(int64_t i, int lane, bool on) const {
        if (!on) return;
        const int64_t beg = row_ptr[i], d = row_ptr[i + 1] - beg;
        for (int64_t t = lane; t < d; t += G) {
            const unsigned long long k = keys[beg + order[beg + t]];
            const uint32_t b = (uint32_t)(k >> 32);
            if (t == 0 || (uint32_t)(keys[beg + order[beg + t - 1]] >> 32) != b) {
                first_pos[beg + b] = (uint32_t)t;
                first_u[beg + b] = (uint32_t)k;
            }
        }
    }
};

// Per entry: its round r (rank minus the rank of its bin's first entry) and
// the second key (r << 32 | the bin's smallest priority), in place of the first.
struct BinRounds {
    const int64_t *row_ptr;
    unsigned long long *keys;
    const uint32_t *rank, *first_u, *first_pos;
    template <int G>
    __device__ __forceinline__ void run(int64_t i, int lane, bool on) const {
        if (!on) return;
        const int64_t beg = row_ptr[i], d = row_ptr[i + 1] - beg;
        for (int64_t q = lane; q < d; q += G) {
            const int64_t p = beg + q;
            const int64_t b = (int64_t)(keys[p] >> 32);
            const uint32_t r = rank[p] - first_pos[beg + b];
            keys[p] = ((unsigned long long)r << 32) | first_u[beg + b];
        }
    }
};

template <typename Body>
__global__ __launch_bounds__(SBLOCK) void k_bin_rows(int64_t n, Body body) {
    for_bin_rows(n, body.row_ptr, body);
}

struct BinLayout {
    SelLayout sel;                // recs hold the first ranking's ranks, then the second's
    unsigned long long *keys;     // [2m]
    uint32_t *first_u, *first_pos;  // [2m]: per-row bin slots
    uint32_t *order, *rank;         // [2m]: the row in the first order, and each entry's rank in it
    double *cbrt_tab;             // [d_max + 1]
    int32_t *budget;              // [d_max + 1]
};

static size_t bin_layout(const ad_graph *g, void *ws, size_t ws_bytes, BinLayout *B) {
    const size_t sel = sel_layout(g, ws, ws_bytes, B ? &B->sel : nullptr, true);
    if (ws && sel == 0) return 0;
    const size_t sel_bytes = sel_layout(g, nullptr, 0, nullptr, true);
    Carver c(ws ? (char *)ws + sel_bytes : nullptr, ws ? ws_bytes - std::min(ws_bytes, sel_bytes) : 0);
    const int64_t nnz = std::max<int64_t>(1, 2 * g->m);
    BinLayout l;
    l.keys = c.take<unsigned long long>(nnz);
    l.first_u = c.take<uint32_t>(nnz);
    l.first_pos = c.take<uint32_t>(nnz);
    l.order = c.take<uint32_t>(nnz);
    l.rank = c.take<uint32_t>(nnz);
    l.cbrt_tab = c.take<double>((size_t)g->d_max + 1);
    l.budget = c.take<int32_t>((size_t)g->d_max + 1);
    if (B) {
        l.sel = B->sel;
        *B = l;
    }
    if (ws && !c.ok()) return 0;
    return sel_bytes + c.used;
}

static ad_status sparsify_binned_impl(const ad_graph *g, ad_dtype rho_dtype, const void *rho, uint64_t seed,
                                      uint64_t graph_id, double e, double target, uint8_t *keep, int64_t *n_kept,
                                      double *e_used_host, const BinLayout &B, hipStream_t stream) {
    const SelLayout &L = B.sel;
    const int64_t n = g->n, m = g->m;
    ad_status s;
    if (m == 0) {
        s = fill_u64(L.counts, 0, 1, stream);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, stream, L.counts, n_kept);
        AD_LAUNCH_CHECK("k_store_count");
        if (e_used_host) {
            *e_used_host = target > 0.0 ? 0.0 : e;
            AD_HIP(hipStreamSynchronize(stream));
        }
        return AD_OK;
    }
    // host tables by degree (the C library's cbrt and pow), copied to the device
    std::vector<double> cb((size_t)g->d_max + 1);
    for (int64_t d = 0; d <= g->d_max; ++d) cb[(size_t)d] = cbrt((double)d);
    AD_HIP(hipMemcpyAsync(B.cbrt_tab, cb.data(), cb.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    std::vector<int32_t> bt;
    if (!(target > 0.0)) {
        budget_table(g->d_max, e, bt);
        AD_HIP(hipMemcpyAsync(B.budget, bt.data(), bt.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    }
    // a group of lanes per short row, a wave per long row
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(n, SBLOCK / BIN_SHORT_G)));
    {
        TraceScope trace("k_bin", stream);
        if (rho_dtype == AD_F32) {
            const BinKeys<float> bk{g->row_ptr, g->col, g->eid, g->orig_id, g->col_orig, (const float *)rho,
                                    B.cbrt_tab, (int64_t)g->d_max, seed, graph_id, B.keys};
            hipLaunchKernelGGL((k_bin_keys<float>), dim3(grid), dim3(SBLOCK), 0, stream, n, bk);
        } else {
            const BinKeys<double> bk{g->row_ptr, g->col, g->eid, g->orig_id, g->col_orig, (const double *)rho,
                                     B.cbrt_tab, (int64_t)g->d_max, seed, graph_id, B.keys};
            hipLaunchKernelGGL((k_bin_keys<double>), dim3(grid), dim3(SBLOCK), 0, stream, n, bk);
        }
        AD_LAUNCH_CHECK("k_bin_keys");
    }
    // first ranking: (bin, priority); ranks into the side records
    s = rank_all<float>(g, nullptr, emit_single(MODE_REC, AD_LOCAL, nullptr, nullptr, L.recs), L, stream, B.keys);
    if (s != AD_OK) return s;
    {
        TraceScope trace("k_bin", stream);
        hipLaunchKernelGGL(k_bin_rows<BinOrder>, dim3(grid), dim3(SBLOCK), 0, stream, n,
                           BinOrder{g->row_ptr, g->col, g->eid, L.recs, B.order, B.rank});
        AD_LAUNCH_CHECK("k_bin_order");
        hipLaunchKernelGGL(k_bin_rows<BinFirsts>, dim3(grid), dim3(SBLOCK), 0, stream, n,
                           BinFirsts{g->row_ptr, B.keys, B.order, B.first_u, B.first_pos});
        AD_LAUNCH_CHECK("k_bin_firsts");
        hipLaunchKernelGGL(k_bin_rows<BinRounds>, dim3(grid), dim3(SBLOCK), 0, stream, n,
                           BinRounds{g->row_ptr, B.keys, B.rank, B.first_u, B.first_pos});
        AD_LAUNCH_CHECK("k_bin_rounds");
    }
    if (target > 0.0) {
        // second ranking (round, bin order) over the first's records, then the retention fit
        s = rank_all<float>(g, nullptr, emit_single(MODE_REC, AD_LOCAL, nullptr, nullptr, L.recs), L, stream,
                            B.keys);
        if (s != AD_OK) return s;
        TraceScope trace_fit("k_fit_select", stream);
        hipLaunchKernelGGL(k_log_table, dim3(grid_for((int64_t)g->d_max + 2, SBLOCK)), dim3(SBLOCK), 0, stream,
                           (int64_t)g->d_max + 2, L.logs);
        AD_LAUNCH_CHECK("k_log_table");
        uint8_t *kp[1] = {keep};
        return fit_from_recs(g, L, 1, fit_count_target(m, target), kp, n_kept, e_used_host, stream);
    }
    // second ranking straight into keep at the fixed exponent
    s = fill_u64(L.counts, 0, 1, stream);
    if (s != AD_OK) return s;
    s = fill_u8(keep, 0, m, stream);
    if (s != AD_OK) return s;
    s = rank_all<float>(g, nullptr, emit_single(MODE_FIXED, AD_LOCAL, B.budget, keep, nullptr), L, stream, B.keys);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_count_bytes, dim3((unsigned)std::min<int64_t>(SUM_BLOCKS, ceil_div(m, SBLOCK))),
                       dim3(SBLOCK), 0, stream, m, keep, L.counts);
    AD_LAUNCH_CHECK("k_count_bytes");
    hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, stream, L.counts, n_kept);
    AD_LAUNCH_CHECK("k_store_count");
    // the host tables must outlive their copies
    AD_HIP(hipStreamSynchronize(stream));
    if (e_used_host) *e_used_host = e;
    return AD_OK;
}

}  // namespace ad

extern "C" size_t ad_sparsify_binned_workspace_size(const ad_graph *g) {
    if (check_graph_args(g) != AD_OK) return 0;
    return bin_layout(g, nullptr, 0, nullptr);
}

extern "C" ad_status ad_sparsify_binned(const ad_graph *g, ad_dtype rho_dtype, const void *rho, uint64_t seed,
                                        uint64_t graph_id, double e, double target, uint8_t *keep,
                                        int64_t *n_kept, double *e_used_host, void *ws, size_t ws_bytes,
                                        hipStream_t stream) {
    SelLayout L;
    ad_status s = check_sel_args(g, rho_dtype, rho, AD_LOCAL, keep, n_kept, ws, ws_bytes, &L, true);
    if (s != AD_OK) return s;
    if (target > 0.0) {
        if (!(target <= 1.0)) return fail(AD_ERR_INVALID_ARG, "target must be in (0, 1]");
        if (!e_used_host) return fail(AD_ERR_INVALID_ARG, "e_used_host is NULL (a fit reports its exponent)");
    } else {
        if (target != 0.0) return fail(AD_ERR_INVALID_ARG, "target must be 0 (fixed e) or in (0, 1]");
        if (!(e >= 0.0 && e <= 1.0)) return fail(AD_ERR_INVALID_ARG, "e must be in [0, 1]");
    }
    if ((size_t)g->d_max + 1 > ((size_t)1 << 31)) return fail(AD_ERR_UNSUPPORTED, "d_max too large");
    BinLayout B;
    B.sel = L;
    if (bin_layout(g, ws, ws_bytes, &B) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    return sparsify_binned_impl(g, rho_dtype, rho, seed, graph_id, e, target, keep, n_kept, e_used_host, B, stream);
}
