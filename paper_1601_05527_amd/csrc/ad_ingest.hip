// Ingest: an undirected edge list into the symmetric CSR that every other
// call reads (the graph model of Section 2: undirected, no self-loops, no
// repeated pairs), optionally with the vertices stored by decreasing degree.
//
// Readings (shared with the oracle, which is written separately): (u, v) and
// (v, u) name the same edge; self-loops are dropped; repeated pairs become
// one edge whose weight is the exact sum of the listed weights rounded once
// to single precision (listed weights must be finite and positive, as the
// graph model requires); edge ids enumerate the edges
// in (smaller endpoint, larger endpoint) order, the CSR order of their upper
// entries; rows list neighbours in ascending order; the decreasing-degree
// order breaks ties by listed id, and orig_id names the listed vertex.  The
// reverse Cuthill-McKee order: components by increasing smallest id, each
// searched breadth first from its vertex of least (degree, id), the
// neighbours of a dequeued vertex queued by increasing (degree, id), the
// whole order reversed.
//
// The pipeline: canonical 64-bit pair keys, a stable radix sort (rocPRIM) of
// (key, list index), run heads and their scan (edge ids), run bounds, and
// the exact weight sum of every run (one thread per short run, one wave per
// long run); for
// the degree order a sort of (degree, id) vertex keys and a second pair sort
// under the new labels (for reverse Cuthill-McKee, the graph placed under
// the listed ids, its components, and a level-by-level search with two
// sorts per level, then the same relabelling); then per-row counts from the run lengths of the
// sorted endpoints (no atomics, so hub vertices cost nothing extra), their
// scans and the placement of the upper entries (edge order) and of the
// lower entries (a stable sort of the edges by larger endpoint).
#include "ad_internal.h"

#include <cstring>    // before rocPRIM: its host code calls memset

#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <cfloat>
#include <cstdint>

namespace ad {

constexpr int IBLOCK = 256;
constexpr unsigned long long NO_PAIR = ~0ull;

static unsigned bits_for(int64_t n) {
    unsigned b = 1;
    while (b < 32 && ((int64_t)1 << b) < n) ++b;
    return b;
}

// Pair key (smaller << 32 | larger), NO_PAIR for self-loops; endpoints out
// of [0, n) raise the error flag (and sort last).
__global__ void k_pair_keys(int64_t m_in, int64_t n, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                            const float *__restrict__ w, unsigned long long *__restrict__ key,
                            uint32_t *__restrict__ idx, unsigned int *__restrict__ err) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m_in; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = u[q], b = v[q];
        unsigned long long k = NO_PAIR;
        if (w && !(w[q] > 0.0f && w[q] <= FLT_MAX)) atomicOr(err, 2u);
        if (a < 0 || a >= n || b < 0 || b >= n) {
            atomicOr(err, 1u);
        } else if (a != b) {
            const uint64_t lo = (uint64_t)(a < b ? a : b), hi = (uint64_t)(a < b ? b : a);
            k = (lo << 32) | hi;
        }
        key[q] = k;
        idx[q] = (uint32_t)q;
    }
}

// 1 at the first entry of every run of equal pair keys.
__global__ void k_run_heads(int64_t count, const unsigned long long *__restrict__ key, uint32_t *__restrict__ head) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x)
        head[q] = (key[q] != NO_PAIR && (q == 0 || key[q] != key[q - 1])) ? 1u : 0u;
}

// Bounds [start, end) of every run of equal pair keys, by edge id (edge_of
// is the exclusive scan of the run heads).
__global__ void k_run_bounds(int64_t count, const unsigned long long *__restrict__ key,
                             const uint32_t *__restrict__ head, const uint32_t *__restrict__ edge_of,
                             uint2 *__restrict__ bounds) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = key[q];
        if (k == NO_PAIR) continue;
        const uint32_t e = head[q] ? edge_of[q] : edge_of[q] - 1u;
        if (head[q]) bounds[e].x = (uint32_t)q;
        if (q + 1 == count || key[q + 1] != k) bounds[e].y = (uint32_t)(q + 1);
    }
}

// Merged weights: the exact sum of a run's listed weights, rounded once to
// single precision (to nearest, ties to even), so no order of additions
// matters and a run can be summed by many lanes.  A positive finite float
// x is mant * 2^(shift - 149) with mant < 2^24 and 0 <= shift <= 253.  When
// every value of a run lies within 53 bits of one another (the bit span of
// the set plus the bits its count adds), every partial sum is exact in
// double and the double sum, rounded to float, is the answer; otherwise the
// run is summed as an integer count of 2^-149 in XDIG base-2^32 digits with
// deferred carries.
constexpr uint32_t MERGE_SHORT = 16;     // runs up to this length are summed by one thread,
constexpr uint32_t MERGE_WAVE = 4096;    // up to this one by one wave, longer ones by a workgroup
constexpr int MERGE_TB = 1024;           // threads of a long run's workgroup
constexpr int XDIG = 11;                 // 352 bits: 2^31 floats below 2^277 units each

__device__ __forceinline__ void f32_split(float x, uint32_t &mant, int &shift) {
    const uint32_t b = __float_as_uint(x);
    const uint32_t ex = (b >> 23) & 0xffu, fr = b & 0x7fffffu;
    mant = ex ? (fr | 0x800000u) : fr;
    shift = ex ? (int)ex - 1 : 0;
}

__device__ __forceinline__ int ceil_log2_u32(uint32_t c) { return c <= 1 ? 0 : 32 - __clz((int)(c - 1)); }

// Digits hold values below 2^63 for fewer than 2^31 added floats.
__device__ __forceinline__ void digits_add(unsigned long long (&acc)[XDIG], float x) {
    uint32_t mant;
    int shift;
    f32_split(x, mant, shift);
    const int k = shift >> 5;
    const unsigned long long add = (unsigned long long)mant << (shift & 31);
    const unsigned long long lo = add & 0xffffffffull, hi = add >> 32;
#pragma unroll
    for (int d = 0; d < XDIG; ++d) {
        acc[d] += (d == k) ? lo : 0ull;
        acc[d] += (d == k + 1) ? hi : 0ull;
    }
}

// The float nearest to acc * 2^-149 (ties to even; +inf past the range).
__device__ float digits_round(const unsigned long long (&acc)[XDIG]) {
    uint32_t dg[XDIG];
    unsigned long long carry = 0;
#pragma unroll
    for (int d = 0; d < XDIG; ++d) {
        const unsigned long long t = acc[d] + carry;
        dg[d] = (uint32_t)t;
        carry = t >> 32;
    }
    int top = -1;
#pragma unroll
    for (int d = XDIG - 1; d >= 0; --d)
        if (top < 0 && dg[d] != 0u) top = 32 * d + 31 - __clz((int)dg[d]);
    if (top < 0) return 0.0f;
    if (top <= 23) return ldexpf((float)dg[0], -149);       // below 2^24 units: exact
    // bits [top - 24, top] from the digits k .. k + 2, and whether any bit below is set
    const int low = top - 24, k = low >> 5, o = low & 31;
    uint32_t d0 = 0, d1 = 0, d2 = 0;
    bool sticky = false;
#pragma unroll
    for (int d = 0; d < XDIG; ++d) {
        d0 = (d == k) ? dg[d] : d0;
        d1 = (d == k + 1) ? dg[d] : d1;
        d2 = (d == k + 2) ? dg[d] : d2;
        sticky |= (d < k) && dg[d] != 0u;
    }
    sticky |= o != 0 && (d0 & ((1u << o) - 1u)) != 0u;
    unsigned long long win = ((unsigned long long)d1 << 32) | d0;
    if (o) win = (win >> o) | ((unsigned long long)d2 << (64 - o));
    uint32_t mant = (uint32_t)(win >> 1) & 0xffffffu;
    const bool rnd = (win & 1ull) != 0ull;
    if (rnd && (sticky || (mant & 1u))) {
        ++mant;
        if (mant == (1u << 24)) {
            mant >>= 1;
            ++top;
        }
    }
    if (top - 149 > 127) return __int_as_float(0x7f800000);
    return ldexpf((float)mant, top - 23 - 149);
}

// One thread per run: the edge's endpoints and, for a short run, its
// weight.  Longer runs go to lists for k_merge_long and k_merge_big.
__global__ void k_merge_runs(int64_t m, const uint2 *__restrict__ bounds, const unsigned long long *__restrict__ key,
                             const uint32_t *__restrict__ idx, const float *__restrict__ w, int32_t *__restrict__ ea,
                             int32_t *__restrict__ eb, float *__restrict__ ew, uint32_t *__restrict__ long_list,
                             unsigned int *__restrict__ long_count, uint32_t *__restrict__ big_list,
                             unsigned int *__restrict__ big_count) {
    // the loop bound is uniform per wave (blocks are whole waves), so every
    // lane reaches the wave-wide append
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t m_pad = ceil_div_dev(m, stride) * stride;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m_pad; e += stride) {
        bool defer = false, big = false;
        if (e < m) {
            const uint2 b = bounds[e];
            const unsigned long long k = key[b.x];
            ea[e] = (int32_t)(k >> 32);
            eb[e] = (int32_t)(k & 0xffffffffull);
            const uint32_t len = b.y - b.x;
            if (w && len == 1) {
                ew[e] = w[idx[b.x]];
            } else if (w && len <= MERGE_SHORT) {
                int lo = 1 << 20, hi = -1;
                double sum = 0.0;
                for (uint32_t r = b.x; r < b.y; ++r) {
                    const float x = w[idx[r]];
                    uint32_t mant;
                    int shift;
                    f32_split(x, mant, shift);
                    lo = min(lo, shift);
                    hi = max(hi, shift + 24);
                    sum += (double)x;
                }
                if (hi + ceil_log2_u32(len) - lo <= 53) {
                    ew[e] = (float)sum;
                } else {
                    unsigned long long acc[XDIG] = {};
                    for (uint32_t r = b.x; r < b.y; ++r) digits_add(acc, w[idx[r]]);
                    ew[e] = digits_round(acc);
                }
            } else if (w) {
                defer = true;
                big = len > MERGE_WAVE;
            }
        }
        const bool to_long = defer && !big, to_big = defer && big;
        const unsigned int at = wave_append(to_long, long_count);
        if (to_long) long_list[at] = (uint32_t)e;
        const unsigned int bt = wave_append(to_big, big_count);
        if (to_big) big_list[bt] = (uint32_t)e;
    }
}

// One wave per run of MERGE_SHORT < length <= MERGE_WAVE: every lane sums
// its share (double partial sums when the whole run spans at most 53 bits,
// digits otherwise), then the wave combines them; both are exact, so the
// order does not matter.
constexpr int MERGE_LOADS = 4;           // weights each lane loads per step

__global__ __launch_bounds__(IBLOCK) void k_merge_long(const unsigned int *__restrict__ long_count,
                                                       const uint32_t *__restrict__ long_list,
                                                       const uint2 *__restrict__ bounds,
                                                       const uint32_t *__restrict__ idx, const float *__restrict__ w,
                                                       float *__restrict__ ew) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (IBLOCK / WAVE);
    const int64_t count = *long_count;
    for (int64_t q = (int64_t)blockIdx.x * (IBLOCK / WAVE) + (threadIdx.x >> 6); q < count; q += nw) {
        const uint32_t e = long_list[q];
        const uint2 b = bounds[e];
        int lo = 1 << 20, hi = -1;
        double sum = 0.0;
        for (uint32_t base = b.x; base < b.y; base += WAVE * MERGE_LOADS) {
            float x[MERGE_LOADS];
#pragma unroll
            for (int t = 0; t < MERGE_LOADS; ++t) {
                const uint32_t r = base + (uint32_t)(t * WAVE + lane);
                x[t] = r < b.y ? w[idx[r]] : 0.0f;
            }
#pragma unroll
            for (int t = 0; t < MERGE_LOADS; ++t) {
                if (x[t] == 0.0f) continue;                  // past the run's end
                uint32_t mant;
                int shift;
                f32_split(x[t], mant, shift);
                lo = min(lo, shift);
                hi = max(hi, shift + 24);
                sum += (double)x[t];
            }
        }
        for (int o = WAVE / 2; o >= 1; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o, WAVE));
            hi = max(hi, __shfl_xor(hi, o, WAVE));
            sum += __shfl_xor(sum, o, WAVE);
        }
        if (hi + ceil_log2_u32(b.y - b.x) - lo <= 53) {
            if (lane == 0) ew[e] = (float)sum;
            continue;
        }
        unsigned long long acc[XDIG] = {};
        for (uint32_t r = b.x + (uint32_t)lane; r < b.y; r += WAVE) digits_add(acc, w[idx[r]]);
#pragma unroll
        for (int d = 0; d < XDIG; ++d)
            for (int o = WAVE / 2; o >= 1; o >>= 1) acc[d] += __shfl_xor(acc[d], o, WAVE);
        if (lane == 0) ew[e] = digits_round(acc);
    }
}

// One workgroup of MERGE_TB threads per run longer than MERGE_WAVE: digits
// always (exact at any length), MERGE_LOADS weights per thread in flight.
__global__ __launch_bounds__(MERGE_TB) void k_merge_big(const unsigned int *__restrict__ big_count,
                                                        const uint32_t *__restrict__ big_list,
                                                        const uint2 *__restrict__ bounds,
                                                        const uint32_t *__restrict__ idx, const float *__restrict__ w,
                                                        float *__restrict__ ew) {
    __shared__ unsigned long long part[MERGE_TB / WAVE][XDIG];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
    const unsigned int count = *big_count;
    for (unsigned int q = blockIdx.x; q < count; q += gridDim.x) {
        const uint32_t e = big_list[q];
        const uint2 b = bounds[e];
        unsigned long long acc[XDIG] = {};
        for (uint32_t base = b.x; base < b.y; base += MERGE_TB * MERGE_LOADS) {
            float x[MERGE_LOADS];
#pragma unroll
            for (int t = 0; t < MERGE_LOADS; ++t) {
                const uint32_t r = base + (uint32_t)(t * MERGE_TB) + threadIdx.x;
                x[t] = r < b.y ? w[idx[r]] : 0.0f;
            }
#pragma unroll
            for (int t = 0; t < MERGE_LOADS; ++t) digits_add(acc, x[t]);     // a zero adds nothing
        }
#pragma unroll
        for (int d = 0; d < XDIG; ++d) {
            for (int o = WAVE / 2; o >= 1; o >>= 1) acc[d] += __shfl_xor(acc[d], o, WAVE);
            if (lane == 0) part[wv][d] = acc[d];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int d = 0; d < XDIG; ++d) {
                unsigned long long t = 0;
                for (int k = 0; k < MERGE_TB / WAVE; ++k) t += part[k][d];
                acc[d] = t;
            }
            ew[e] = digits_round(acc);
        }
        __syncthreads();
    }
}

// Run ends of a sorted key array: start[k] = first position, cnt[k] = end
// (both zero beforehand); k_count_finish turns them into counts.
__global__ void k_count_marks(int64_t m, const int32_t *__restrict__ keys, uint32_t *__restrict__ start,
                              uint32_t *__restrict__ cnt) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = keys[t];
        if (t == 0 || keys[t - 1] != k) start[k] = (uint32_t)t;
        if (t + 1 == m || keys[t + 1] != k) cnt[k] = (uint32_t)(t + 1);
    }
}

// cnt[i] -= start[i]; deg[i] = cnt[i] + other[i] when deg is given.
__global__ void k_count_finish(int64_t n, const uint32_t *__restrict__ start, uint32_t *__restrict__ cnt,
                               const uint32_t *__restrict__ other, uint32_t *__restrict__ deg) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cnt[i] - start[i];
        cnt[i] = c;
        if (deg) deg[i] = c + other[i];
    }
}

__global__ void k_degree_max(int64_t n, const uint32_t *__restrict__ deg, unsigned int *__restrict__ dmax) {
    unsigned int mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mx = max(mx, deg[i]);
    for (int o = WAVE / 2; o >= 1; o >>= 1) mx = max(mx, (unsigned int)__shfl_xor((int)mx, o, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0) atomicMax(dmax, mx);
}

// Storage-order key of vertex i: decreasing degree, then increasing listed id.
__global__ void k_vertex_keys(int64_t n, const uint32_t *__restrict__ deg, unsigned long long *__restrict__ vkey,
                              uint32_t *__restrict__ vid) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        vkey[i] = ((unsigned long long)(0xffffffffu - deg[i]) << 32) | (unsigned long long)i;
        vid[i] = (uint32_t)i;
    }
}

__global__ void k_new_ids(int64_t n, const uint32_t *__restrict__ vid_sorted, uint32_t *__restrict__ new_of,
                          const int32_t *__restrict__ orig_in, int32_t *__restrict__ orig_out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = vid_sorted[r];
        new_of[i] = (uint32_t)r;
        orig_out[r] = orig_in ? orig_in[i] : (int32_t)i;
    }
}

__global__ void k_orig_identity(int64_t n, const int32_t *__restrict__ orig_in, int32_t *__restrict__ orig_out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        orig_out[i] = orig_in ? orig_in[i] : (int32_t)i;
}

// Edge keys under the new labels (no repeats remain), payload the old edge id.
__global__ void k_relabel_keys(int64_t m, const int32_t *__restrict__ ea, const int32_t *__restrict__ eb,
                               const uint32_t *__restrict__ new_of, unsigned long long *__restrict__ key,
                               uint32_t *__restrict__ idx) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = new_of[ea[e]], y = new_of[eb[e]];
        key[e] = ((x < y ? x : y) << 32) | (x < y ? y : x);
        idx[e] = (uint32_t)e;
    }
}

__global__ void k_unpack_edges(int64_t m, const unsigned long long *__restrict__ key,
                               const uint32_t *__restrict__ idx, const float *__restrict__ ew_old,
                               int32_t *__restrict__ ea, int32_t *__restrict__ eb, float *__restrict__ ew) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        ea[e] = (int32_t)(key[e] >> 32);
        eb[e] = (int32_t)(key[e] & 0xffffffffull);
        if (ew_old) ew[e] = ew_old[idx[e]];
    }
}

// Upper entry of edge e = (a, b): after row a's lower entries, at e's place
// among the edges that start at a (edge ids are in (a, b) order).
__global__ void k_place_upper(int64_t m, const int32_t *__restrict__ ea, const int32_t *__restrict__ eb,
                              const float *__restrict__ ew, const int64_t *__restrict__ row_ptr,
                              const uint32_t *__restrict__ lower_cnt, const uint64_t *__restrict__ upper_start,
                              int32_t *__restrict__ col, float *__restrict__ w_out, int32_t *__restrict__ eid) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = ea[e];
        const int64_t pos = row_ptr[a] + lower_cnt[a] + (e - (int64_t)upper_start[a]);
        col[pos] = eb[e];
        eid[pos] = (int32_t)e;
        if (w_out) w_out[pos] = ew[e];
    }
}

// Lower entry of edge e = (a, b), from the edges sorted by b (stably, so by a
// within each b): at its place among the edges that end at b.
__global__ void k_place_lower(int64_t m, const uint32_t *__restrict__ b_sorted, const uint32_t *__restrict__ e_sorted,
                              const int32_t *__restrict__ ea, const float *__restrict__ ew,
                              const int64_t *__restrict__ row_ptr, const uint64_t *__restrict__ lower_start,
                              int32_t *__restrict__ col, float *__restrict__ w_out, int32_t *__restrict__ eid) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t b = b_sorted[t], e = e_sorted[t];
        const int64_t pos = row_ptr[b] + (t - (int64_t)lower_start[b]);
        col[pos] = ea[e];
        eid[pos] = (int32_t)e;
        if (w_out) w_out[pos] = ew[e];
    }
}

__global__ void k_edge_b(int64_t m, const int32_t *__restrict__ eb, uint32_t *__restrict__ bkey,
                         uint32_t *__restrict__ eidx) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        bkey[e] = (uint32_t)eb[e];
        eidx[e] = (uint32_t)e;
    }
}

__global__ void k_u32_to_u64(int64_t n, const uint32_t *__restrict__ a, uint64_t *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// ------------------------------------------------ reverse Cuthill-McKee --
// The order of the oracle's reading, built level by level: a breadth-first
// search visits a level in queue order, and each vertex of the next level
// is queued by its first-visited neighbour in the level, its siblings in
// increasing (degree, id) order, so the next level is the set of unplaced
// neighbours ordered by (smallest place among their placed neighbours,
// degree, id).  Every component is searched at once, each in its own range
// of places (components in increasing order of their smallest id, each
// starting at its vertex of least (degree, id)).
constexpr uint32_t RC_UNSET = 0xffffffffu;

__global__ void k_rc_init(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ root,
                          uint32_t *__restrict__ size, unsigned long long *__restrict__ start,
                          uint32_t *__restrict__ pos, uint32_t *__restrict__ par) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = root[i];
        const unsigned long long d = (unsigned long long)(row_ptr[i + 1] - row_ptr[i]);
        atomicAdd(&size[r], 1u);
        atomicMin(&start[r], (d << 32) | (unsigned long long)i);
        pos[i] = RC_UNSET;
        par[i] = RC_UNSET;
    }
}

// Each component's start takes the component's first place and joins the
// first frontier.
__global__ void k_rc_seed(int64_t n, const uint32_t *__restrict__ size, const uint32_t *__restrict__ off,
                          const unsigned long long *__restrict__ start, uint32_t *__restrict__ pos,
                          uint32_t *__restrict__ fill, uint32_t *__restrict__ front, unsigned int *__restrict__ cnt) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        if (size[r] == 0) continue;
        const uint32_t v = (uint32_t)(start[r] & 0xffffffffull);
        pos[v] = off[r];
        fill[r] = off[r] + 1u;
        front[atomicAdd(&cnt[0], 1u)] = v;
    }
}

// One wave per frontier vertex: every unplaced neighbour keeps the smallest
// place among its frontier neighbours; the first to reach it lists it.
__global__ void k_rc_expand(unsigned int nf, const uint32_t *__restrict__ front, const int64_t *__restrict__ row_ptr,
                            const int32_t *__restrict__ col, const uint32_t *__restrict__ pos,
                            uint32_t *__restrict__ par, uint32_t *__restrict__ cand, unsigned int *__restrict__ ncand) {
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned int nw = gridDim.x * (IBLOCK / WAVE);
    for (unsigned int f = blockIdx.x * (IBLOCK / WAVE) + (threadIdx.x >> 6); f < nf; f += nw) {
        const uint32_t v = front[f];
        const uint32_t pv = pos[v];
        const int64_t b1 = row_ptr[v + 1];
        for (int64_t p = row_ptr[v] + lane; p < b1; p += WAVE) {
            const int32_t u = col[p];
            if (pos[u] != RC_UNSET) continue;
            if (atomicMin(&par[u], pv) == RC_UNSET) cand[atomicAdd(ncand, 1u)] = (uint32_t)u;
        }
    }
}

// Sort key of a candidate: (smallest neighbour place, degree); its id breaks
// ties through the stable sort of candidates already in id order.
__global__ void k_rc_keys(unsigned int nc, const uint32_t *__restrict__ cand, const uint32_t *__restrict__ par,
                          const int64_t *__restrict__ row_ptr, unsigned long long *__restrict__ key) {
    for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
        const uint32_t u = cand[i];
        key[i] = ((unsigned long long)par[u] << 32) | (unsigned long long)(row_ptr[u + 1] - row_ptr[u]);
    }
}

// A component's candidates are contiguous in the sorted level (their
// parents' places lie in the component's range): first index of each run,
// the places, then the component's next free place.
__global__ void k_rc_first(unsigned int nc, const uint32_t *__restrict__ vert, const int32_t *__restrict__ root,
                           uint32_t *__restrict__ first) {
    for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
        const int32_t r = root[vert[i]];
        if (i == 0 || root[vert[i - 1]] != r) first[r] = i;
    }
}

__global__ void k_rc_place(unsigned int nc, const uint32_t *__restrict__ vert, const int32_t *__restrict__ root,
                           const uint32_t *__restrict__ first, const uint32_t *__restrict__ fill,
                           uint32_t *__restrict__ pos) {
    for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
        const uint32_t u = vert[i];
        const int32_t r = root[u];
        pos[u] = fill[r] + (i - first[r]);
    }
}

__global__ void k_rc_advance(unsigned int nc, const uint32_t *__restrict__ vert, const int32_t *__restrict__ root,
                             const uint32_t *__restrict__ first, uint32_t *__restrict__ fill) {
    for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
        const int32_t r = root[vert[i]];
        if (i + 1 == nc || root[vert[i + 1]] != r) fill[r] += i - first[r] + 1u;
    }
}

// Reversed: the vertex at Cuthill-McKee place q is stored as n - 1 - q.
__global__ void k_rc_order(int64_t n, const uint32_t *__restrict__ pos, uint32_t *__restrict__ vid_sorted) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        vid_sorted[n - 1 - (int64_t)pos[v]] = (uint32_t)v;
}

struct IngestLayout {
    unsigned long long *key0, *key1;     // [m_in] pair keys (sort double buffer)
    uint32_t *idx0, *idx1;               // [m_in] list indices / edge ids
    uint32_t *head, *edge_of;            // [m_in]
    int32_t *ea, *eb;                    // [m_in] edges (a < b)
    float *ew, *ew2;                     // [m_in]
    uint32_t *deg, *lower_cnt, *upper_cnt, *new_of;   // [n]
    uint64_t *lower_start, *upper_start, *deg64;      // [n]
    unsigned long long *vkey0, *vkey1;   // [n]
    uint32_t *vid0, *vid1;               // [n]
    unsigned int *flags;                 // [4]: error bits, d_max, runs for a workgroup, runs for a wave
    // reverse Cuthill-McKee order ([n] each)
    int32_t *rc_root;                    // component of every vertex (its smallest id)
    uint32_t *rc_pos;                    // place in the Cuthill-McKee order (RC_UNSET before)
    uint32_t *rc_par;                    // smallest place among a candidate's placed neighbours
    uint32_t *rc_size, *rc_off, *rc_fill, *rc_first;  // per component root: size, first place, next place,
                                                      // first index in the sorted candidates
    unsigned long long *rc_start;        // per component root: (degree << 32 | id) of its start
    uint32_t *rc_front, *rc_cand, *rc_cand2, *rc_vert;
    unsigned long long *rc_key0, *rc_key1;
    unsigned int *rc_cnt;                // [2]: frontier size, candidates
    void *temp;                          // rocPRIM temporary storage
    size_t temp_bytes;
};

// Largest temporary storage any of the pipeline's rocPRIM calls asks for (0
// when a query fails; the launch then reports the error).
static size_t rocprim_temp_bytes(int64_t m_in, int64_t n) {
    size_t need = 0, t = 0;
    hipError_t e = hipSuccess;
    const size_t mm = (size_t)std::max<int64_t>(1, m_in), nn = (size_t)std::max<int64_t>(1, n);
    e = rocprim::radix_sort_pairs(nullptr, t, (unsigned long long *)nullptr, (unsigned long long *)nullptr,
                                  (uint32_t *)nullptr, (uint32_t *)nullptr, mm, 0, 64);
    need = std::max(need, e == hipSuccess ? t : 0);
    e = rocprim::radix_sort_pairs(nullptr, t, (unsigned long long *)nullptr, (unsigned long long *)nullptr,
                                  (uint32_t *)nullptr, (uint32_t *)nullptr, nn, 0, 64);
    need = std::max(need, e == hipSuccess ? t : 0);
    e = rocprim::radix_sort_pairs(nullptr, t, (uint32_t *)nullptr, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                  (uint32_t *)nullptr, mm, 0, 32);
    need = std::max(need, e == hipSuccess ? t : 0);
    e = rocprim::exclusive_scan(nullptr, t, (uint32_t *)nullptr, (uint32_t *)nullptr, 0u, mm,
                                rocprim::plus<uint32_t>());
    need = std::max(need, e == hipSuccess ? t : 0);
    e = rocprim::exclusive_scan(nullptr, t, (uint64_t *)nullptr, (uint64_t *)nullptr, (uint64_t)0, nn + 1,
                                rocprim::plus<uint64_t>());
    need = std::max(need, e == hipSuccess ? t : 0);
    e = rocprim::exclusive_scan(nullptr, t, (uint32_t *)nullptr, (uint32_t *)nullptr, 0u, nn,
                                rocprim::plus<uint32_t>());
    need = std::max(need, e == hipSuccess ? t : 0);
    e = rocprim::radix_sort_keys(nullptr, t, (uint32_t *)nullptr, (uint32_t *)nullptr, nn, 0, 32);
    need = std::max(need, e == hipSuccess ? t : 0);
    return need;
}

static size_t ingest_layout(int64_t n, int64_t m_in, void *ws, size_t ws_bytes, IngestLayout *L) {
    Carver c(ws, ws_bytes);
    const size_t mm = (size_t)std::max<int64_t>(1, m_in), nn = (size_t)std::max<int64_t>(1, n) + 1;
    IngestLayout l;
    l.key0 = c.take<unsigned long long>(mm);
    l.key1 = c.take<unsigned long long>(mm);
    l.idx0 = c.take<uint32_t>(mm);
    l.idx1 = c.take<uint32_t>(mm);
    l.head = c.take<uint32_t>(mm);
    l.edge_of = c.take<uint32_t>(mm);
    l.ea = c.take<int32_t>(mm);
    l.eb = c.take<int32_t>(mm);
    l.ew = c.take<float>(mm);
    l.ew2 = c.take<float>(mm);
    l.deg = c.take<uint32_t>(nn);
    l.lower_cnt = c.take<uint32_t>(nn);
    l.upper_cnt = c.take<uint32_t>(nn);
    l.new_of = c.take<uint32_t>(nn);
    l.lower_start = c.take<uint64_t>(nn);
    l.upper_start = c.take<uint64_t>(nn);
    l.deg64 = c.take<uint64_t>(nn);
    l.vkey0 = c.take<unsigned long long>(nn);
    l.vkey1 = c.take<unsigned long long>(nn);
    l.vid0 = c.take<uint32_t>(nn);
    l.vid1 = c.take<uint32_t>(nn);
    l.flags = c.take<unsigned int>(4);
    l.rc_root = c.take<int32_t>(nn);
    l.rc_pos = c.take<uint32_t>(nn);
    l.rc_par = c.take<uint32_t>(nn);
    l.rc_size = c.take<uint32_t>(nn);
    l.rc_off = c.take<uint32_t>(nn);
    l.rc_fill = c.take<uint32_t>(nn);
    l.rc_first = c.take<uint32_t>(nn);
    l.rc_start = c.take<unsigned long long>(nn);
    l.rc_front = c.take<uint32_t>(nn);
    l.rc_cand = c.take<uint32_t>(nn);
    l.rc_cand2 = c.take<uint32_t>(nn);
    l.rc_vert = c.take<uint32_t>(nn);
    l.rc_key0 = c.take<unsigned long long>(nn);
    l.rc_key1 = c.take<unsigned long long>(nn);
    l.rc_cnt = c.take<unsigned int>(2);
    l.temp_bytes = rocprim_temp_bytes(m_in, n);
    l.temp = c.take<char>(l.temp_bytes);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

static unsigned igrid(int64_t count) { return grid_for(std::max<int64_t>(1, count), IBLOCK); }

#define AD_RP(call)                                                         \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) return fail(AD_ERR_HIP, std::string("rocPRIM: ") + hipGetErrorString(e_)); \
    } while (0)

// Degrees of the m edges (ea < eb, sorted by (ea, eb)) without atomics:
// upper_cnt from the runs of ea, lower_cnt from the runs of eb after a
// stable sort of the edge ids by eb (left in idx1 / edge_of for the lower
// placement), deg = upper + lower.  deg, upper_cnt, lower_cnt: [n];
// vid0 / vid1 serve as scratch.
static ad_status edge_counts(int64_t n, int64_t m, const int32_t *ea, const int32_t *eb, const IngestLayout &L,
                             hipStream_t st) {
    ad_status s;
    for (uint32_t *p : {L.upper_cnt, L.lower_cnt, L.vid0, L.vid1}) {
        s = fill_i32((int32_t *)p, 0, n, st);
        if (s != AD_OK) return s;
    }
    hipLaunchKernelGGL(k_count_marks, dim3(igrid(m)), dim3(IBLOCK), 0, st, m, ea, L.vid0, L.upper_cnt);
    AD_LAUNCH_CHECK("k_count_marks");
    hipLaunchKernelGGL(k_edge_b, dim3(igrid(m)), dim3(IBLOCK), 0, st, m, eb, L.idx0, L.head);
    AD_LAUNCH_CHECK("k_edge_b");
    size_t tb = L.temp_bytes;
    AD_RP(rocprim::radix_sort_pairs(L.temp, tb, L.idx0, L.idx1, L.head, L.edge_of, (size_t)m, 0, bits_for(n), st));
    hipLaunchKernelGGL(k_count_marks, dim3(igrid(m)), dim3(IBLOCK), 0, st, m, (const int32_t *)L.idx1, L.vid1,
                       L.lower_cnt);
    AD_LAUNCH_CHECK("k_count_marks");
    hipLaunchKernelGGL(k_count_finish, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.vid0, L.upper_cnt,
                       (const uint32_t *)nullptr, (uint32_t *)nullptr);
    AD_LAUNCH_CHECK("k_count_finish");
    hipLaunchKernelGGL(k_count_finish, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.vid1, L.lower_cnt, L.upper_cnt,
                       L.deg);
    AD_LAUNCH_CHECK("k_count_finish");
    return AD_OK;
}

// The edges (ea < eb, sorted by (ea, eb); weights ew or NULL) as the
// symmetric CSR: per-row counts (upper_cnt: edges whose smaller endpoint is
// the row, lower_cnt: larger), the edges sorted by larger endpoint
// (idx1 / edge_of), the degrees and their maximum (flags[1]), row_ptr, then
// the upper entries in edge order and the lower ones.  w_out NULL: no weights.
static ad_status place_csr(int64_t n, int64_t m, const int32_t *ea, const int32_t *eb, const float *ew,
                           int64_t *row_ptr, int32_t *col, float *w_out, int32_t *eid, const IngestLayout &L,
                           hipStream_t st) {
    ad_status s;
    if (n > 0) {
        s = fill_i32((int32_t *)L.deg, 0, n, st);
        if (s != AD_OK) return s;
        if (m > 0) {
            s = edge_counts(n, m, ea, eb, L, st);
            if (s != AD_OK) return s;
        } else {
            s = fill_i32((int32_t *)L.lower_cnt, 0, n, st);
            if (s != AD_OK) return s;
            s = fill_i32((int32_t *)L.upper_cnt, 0, n, st);
            if (s != AD_OK) return s;
        }
        hipLaunchKernelGGL(k_degree_max, dim3(std::min<unsigned>(256, igrid(n))), dim3(IBLOCK), 0, st, n, L.deg,
                           L.flags + 1);
        AD_LAUNCH_CHECK("k_degree_max");
    }
    // row_ptr = exclusive scan of the degrees over n + 1 entries (the last one 0)
    s = fill_i32((int32_t *)(L.deg64 + n), 0, 2, st);
    if (s != AD_OK) return s;
    if (n > 0) {
        hipLaunchKernelGGL(k_u32_to_u64, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.deg, L.deg64);
        AD_LAUNCH_CHECK("k_u32_to_u64");
    }
    size_t tb = L.temp_bytes;
    AD_RP(rocprim::exclusive_scan(L.temp, tb, L.deg64, (uint64_t *)row_ptr, (uint64_t)0, (size_t)n + 1,
                                  rocprim::plus<uint64_t>(), st));
    if (m > 0) {
        hipLaunchKernelGGL(k_u32_to_u64, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.upper_cnt, L.deg64);
        AD_LAUNCH_CHECK("k_u32_to_u64");
        tb = L.temp_bytes;
        AD_RP(rocprim::exclusive_scan(L.temp, tb, L.deg64, L.upper_start, (uint64_t)0, (size_t)n,
                                      rocprim::plus<uint64_t>(), st));
        hipLaunchKernelGGL(k_u32_to_u64, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.lower_cnt, L.deg64);
        AD_LAUNCH_CHECK("k_u32_to_u64");
        tb = L.temp_bytes;
        AD_RP(rocprim::exclusive_scan(L.temp, tb, L.deg64, L.lower_start, (uint64_t)0, (size_t)n,
                                      rocprim::plus<uint64_t>(), st));
        hipLaunchKernelGGL(k_place_upper, dim3(igrid(m)), dim3(IBLOCK), 0, st, m, ea, eb, ew, row_ptr, L.lower_cnt,
                           L.upper_start, col, w_out, eid);
        AD_LAUNCH_CHECK("k_place_upper");
        // lower entries from the edges sorted (stably) by their larger endpoint
        hipLaunchKernelGGL(k_place_lower, dim3(igrid(m)), dim3(IBLOCK), 0, st, m, L.idx1, L.edge_of, ea, ew, row_ptr,
                           L.lower_start, col, w_out, eid);
        AD_LAUNCH_CHECK("k_place_lower");
    }
    return AD_OK;
}

// Relabel the edges by new_of and number them again in (smaller, larger)
// order: ea, eb rewritten, the weights (when given) permuted into ew2.
static ad_status relabel_edges(int64_t m, const int32_t *ea, const int32_t *eb, const float *ew,
                               const IngestLayout &L, hipStream_t st) {
    if (m <= 0) return AD_OK;
    hipLaunchKernelGGL(k_relabel_keys, dim3(igrid(m)), dim3(IBLOCK), 0, st, m, ea, eb, L.new_of, L.key0, L.idx0);
    AD_LAUNCH_CHECK("k_relabel_keys");
    size_t tb = L.temp_bytes;
    AD_RP(rocprim::radix_sort_pairs(L.temp, tb, L.key0, L.key1, L.idx0, L.idx1, (size_t)m, 0, 64, st));
    hipLaunchKernelGGL(k_unpack_edges, dim3(igrid(m)), dim3(IBLOCK), 0, st, m, L.key1, L.idx1, ew, L.ea, L.eb,
                       L.ew2);
    AD_LAUNCH_CHECK("k_unpack_edges");
    return AD_OK;
}

// Reverse Cuthill-McKee order of the CSR (n vertices, m edges): vid_sorted[r]
// is the vertex stored at r.  One host read-back per level of the search.
static ad_status rcm_order(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *eid,
                           const IngestLayout &L, uint32_t *vid_sorted, hipStream_t st) {
    ad_graph g{};
    g.n = n;
    g.m = m;
    g.row_ptr = row_ptr;
    g.col = m > 0 ? col : nullptr;
    g.eid = m > 0 ? eid : nullptr;
    ad_status s = label_components(&g, L.rc_root, nullptr, st);
    if (s != AD_OK) return s;
    s = fill_i32((int32_t *)L.rc_size, 0, n, st);
    if (s != AD_OK) return s;
    s = fill_u64(L.rc_start, ~0ull, n, st);
    if (s != AD_OK) return s;
    s = fill_i32((int32_t *)L.rc_cnt, 0, 2, st);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_rc_init, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, row_ptr, L.rc_root, L.rc_size, L.rc_start,
                       L.rc_pos, L.rc_par);
    AD_LAUNCH_CHECK("k_rc_init");
    size_t tb = L.temp_bytes;
    AD_RP(rocprim::exclusive_scan(L.temp, tb, L.rc_size, L.rc_off, 0u, (size_t)n, rocprim::plus<uint32_t>(), st));
    hipLaunchKernelGGL(k_rc_seed, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.rc_size, L.rc_off, L.rc_start, L.rc_pos,
                       L.rc_fill, L.rc_front, L.rc_cnt);
    AD_LAUNCH_CHECK("k_rc_seed");
    unsigned int nf = 0;
    AD_HIP(hipMemcpyAsync(&nf, L.rc_cnt, sizeof(nf), hipMemcpyDeviceToHost, st));
    AD_HIP(hipStreamSynchronize(st));
    uint32_t *front = L.rc_front, *next = L.rc_vert;
    const unsigned wgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(n, IBLOCK / WAVE)));
    int64_t placed = nf;
    while (nf > 0 && placed < n) {
        s = fill_i32((int32_t *)L.rc_cnt + 1, 0, 1, st);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_rc_expand, dim3(wgrid), dim3(IBLOCK), 0, st, nf, front, row_ptr, col, L.rc_pos, L.rc_par,
                           L.rc_cand, L.rc_cnt + 1);
        AD_LAUNCH_CHECK("k_rc_expand");
        unsigned int nc = 0;
        AD_HIP(hipMemcpyAsync(&nc, L.rc_cnt + 1, sizeof(nc), hipMemcpyDeviceToHost, st));
        AD_HIP(hipStreamSynchronize(st));
        if (nc == 0) break;
        if ((int64_t)nc > n - placed) return fail(AD_ERR_INTERNAL, "search listed a vertex twice");
        // candidates by id, then stably by (parent place, degree)
        tb = L.temp_bytes;
        AD_RP(rocprim::radix_sort_keys(L.temp, tb, L.rc_cand, L.rc_cand2, (size_t)nc, 0, bits_for(n), st));
        hipLaunchKernelGGL(k_rc_keys, dim3(igrid(nc)), dim3(IBLOCK), 0, st, nc, L.rc_cand2, L.rc_par, row_ptr,
                           L.rc_key0);
        AD_LAUNCH_CHECK("k_rc_keys");
        tb = L.temp_bytes;
        AD_RP(rocprim::radix_sort_pairs(L.temp, tb, L.rc_key0, L.rc_key1, L.rc_cand2, next, (size_t)nc, 0, 64, st));
        hipLaunchKernelGGL(k_rc_first, dim3(igrid(nc)), dim3(IBLOCK), 0, st, nc, next, L.rc_root, L.rc_first);
        AD_LAUNCH_CHECK("k_rc_first");
        hipLaunchKernelGGL(k_rc_place, dim3(igrid(nc)), dim3(IBLOCK), 0, st, nc, next, L.rc_root, L.rc_first,
                           L.rc_fill, L.rc_pos);
        AD_LAUNCH_CHECK("k_rc_place");
        hipLaunchKernelGGL(k_rc_advance, dim3(igrid(nc)), dim3(IBLOCK), 0, st, nc, next, L.rc_root, L.rc_first,
                           L.rc_fill);
        AD_LAUNCH_CHECK("k_rc_advance");
        std::swap(front, next);
        nf = nc;
        placed += nc;
    }
    if (placed != n) return fail(AD_ERR_INTERNAL, "search did not place every vertex");
    hipLaunchKernelGGL(k_rc_order, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.rc_pos, vid_sorted);
    AD_LAUNCH_CHECK("k_rc_order");
    return AD_OK;
}

static ad_status ingest_impl(int64_t n, int64_t m_in, const int32_t *u, const int32_t *v, const float *w,
                             const int32_t *orig_in, int32_t order, int64_t *row_ptr, int32_t *col, float *w_out,
                             int32_t *eid, int32_t *orig_out, int64_t *m_host, int32_t *d_max_host,
                             int64_t *n_dropped_host, const IngestLayout &L, hipStream_t st) {
    TraceScope trace("k_ingest", st);
    ad_status s = fill_i32((int32_t *)L.flags, 0, 4, st);
    if (s != AD_OK) return s;
    int64_t m = 0;
    if (m_in > 0) {
        hipLaunchKernelGGL(k_pair_keys, dim3(igrid(m_in)), dim3(IBLOCK), 0, st, m_in, n, u, v, w, L.key0, L.idx0,
                           L.flags);
        AD_LAUNCH_CHECK("k_pair_keys");
        size_t tb = L.temp_bytes;
        AD_RP(rocprim::radix_sort_pairs(L.temp, tb, L.key0, L.key1, L.idx0, L.idx1, (size_t)m_in, 0, 64, st));
        hipLaunchKernelGGL(k_run_heads, dim3(igrid(m_in)), dim3(IBLOCK), 0, st, m_in, L.key1, L.head);
        AD_LAUNCH_CHECK("k_run_heads");
        tb = L.temp_bytes;
        AD_RP(rocprim::exclusive_scan(L.temp, tb, L.head, L.edge_of, 0u, (size_t)m_in, rocprim::plus<uint32_t>(),
                                      st));
        unsigned int hflags[2];
        uint32_t last[2];
        AD_HIP(hipMemcpyAsync(hflags, L.flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
        AD_HIP(hipMemcpyAsync(&last[0], L.edge_of + (m_in - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        AD_HIP(hipMemcpyAsync(&last[1], L.head + (m_in - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        AD_HIP(hipStreamSynchronize(st));
        if (hflags[0] & 1u) return fail(AD_ERR_GRAPH, "edge list names a vertex outside [0, n)");
        if (hflags[0] & 2u) return fail(AD_ERR_GRAPH, "a listed weight is not finite and positive");
        m = (int64_t)last[0] + (int64_t)last[1];
        if (m > 0) {
            // run bounds in key0 (free after the sort), long runs listed in idx0
            uint2 *bounds = reinterpret_cast<uint2 *>(L.key0);
            hipLaunchKernelGGL(k_run_bounds, dim3(igrid(m_in)), dim3(IBLOCK), 0, st, m_in, L.key1, L.head, L.edge_of,
                               bounds);
            AD_LAUNCH_CHECK("k_run_bounds");
            // runs for a wave listed in idx0, runs for a workgroup in ew2 (both free here)
            uint32_t *big_list = reinterpret_cast<uint32_t *>(L.ew2);
            hipLaunchKernelGGL(k_merge_runs, dim3(igrid(m)), dim3(IBLOCK), 0, st, m, bounds, L.key1, L.idx1, w, L.ea,
                               L.eb, L.ew, L.idx0, L.flags + 3, big_list, L.flags + 2);
            AD_LAUNCH_CHECK("k_merge_runs");
            if (w) {
                hipLaunchKernelGGL(k_merge_long, dim3(1024), dim3(IBLOCK), 0, st, L.flags + 3, L.idx0, bounds, L.idx1,
                                   w, L.ew);
                AD_LAUNCH_CHECK("k_merge_long");
                hipLaunchKernelGGL(k_merge_big, dim3(1024), dim3(MERGE_TB), 0, st, L.flags + 2, big_list, bounds,
                                   L.idx1, w, L.ew);
                AD_LAUNCH_CHECK("k_merge_big");
            }
        }
    }
    const int32_t *ea = L.ea, *eb = L.eb;
    const float *ew = L.ew;
    if (order == 1 && n > 0) {
        s = fill_i32((int32_t *)L.deg, 0, n, st);
        if (s != AD_OK) return s;
        if (m > 0) {
            // degrees before relabelling: run lengths of the sorted smaller and larger endpoints
            s = edge_counts(n, m, ea, eb, L, st);
            if (s != AD_OK) return s;
        }
        hipLaunchKernelGGL(k_vertex_keys, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.deg, L.vkey0, L.vid0);
        AD_LAUNCH_CHECK("k_vertex_keys");
        size_t tb = L.temp_bytes;
        AD_RP(rocprim::radix_sort_pairs(L.temp, tb, L.vkey0, L.vkey1, L.vid0, L.vid1, (size_t)n, 0, 64, st));
        hipLaunchKernelGGL(k_new_ids, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.vid1, L.new_of, orig_in, orig_out);
        AD_LAUNCH_CHECK("k_new_ids");
        s = relabel_edges(m, ea, eb, w ? ew : nullptr, L, st);
        if (s != AD_OK) return s;
        if (m > 0) ew = L.ew2;
    } else if (order == 2 && n > 0) {
        // the graph under the listed ids (in the outputs, rewritten below) for the search
        s = place_csr(n, m, ea, eb, nullptr, row_ptr, col, nullptr, eid, L, st);
        if (s != AD_OK) return s;
        s = rcm_order(n, m, row_ptr, col, eid, L, L.vid1, st);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_new_ids, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, L.vid1, L.new_of, orig_in, orig_out);
        AD_LAUNCH_CHECK("k_new_ids");
        s = relabel_edges(m, ea, eb, w ? ew : nullptr, L, st);
        if (s != AD_OK) return s;
        if (m > 0) ew = L.ew2;
    } else if (n > 0) {
        hipLaunchKernelGGL(k_orig_identity, dim3(igrid(n)), dim3(IBLOCK), 0, st, n, orig_in, orig_out);
        AD_LAUNCH_CHECK("k_orig_identity");
    }
    s = place_csr(n, m, ea, eb, w ? ew : nullptr, row_ptr, col, w ? w_out : nullptr, eid, L, st);
    if (s != AD_OK) return s;
    unsigned int dmax = 0;
    if (n > 0) AD_HIP(hipMemcpyAsync(&dmax, L.flags + 1, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
    AD_HIP(hipStreamSynchronize(st));
    *m_host = m;
    if (d_max_host) *d_max_host = (int32_t)dmax;
    if (n_dropped_host) *n_dropped_host = m_in - m;
    return AD_OK;
}

}  // namespace ad

using namespace ad;

extern "C" size_t ad_ingest_workspace_size(int64_t n, int64_t m_in) {
    if (n < 0 || m_in < 0 || n >= ((int64_t)1 << 31) || m_in >= ((int64_t)1 << 31)) return 0;
    return ingest_layout(n, m_in, nullptr, 0, nullptr);
}

extern "C" ad_status ad_ingest(int64_t n, int64_t m_in, const int32_t *u, const int32_t *v, const float *w,
                               const int32_t *orig_id, int32_t order, int64_t *row_ptr, int32_t *col, float *w_out,
                               int32_t *eid, int32_t *orig_id_out, int64_t *m_host, int32_t *d_max_host,
                               int64_t *n_dropped_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || m_in < 0) return fail(AD_ERR_INVALID_ARG, "negative n or edge count");
    if (n >= ((int64_t)1 << 31) || m_in >= ((int64_t)1 << 31))
        return fail(AD_ERR_UNSUPPORTED, "n and the edge count must be below 2^31");
    if (order < 0 || order > 2)
        return fail(AD_ERR_INVALID_ARG, "order must be 0 (as listed), 1 (by degree) or 2 (reverse Cuthill-McKee)");
    if (m_in > 0 && (!u || !v)) return fail(AD_ERR_INVALID_ARG, "u or v is NULL");
    if (!row_ptr || !m_host) return fail(AD_ERR_INVALID_ARG, "row_ptr or m_host is NULL");
    if (m_in > 0 && (!col || !eid)) return fail(AD_ERR_INVALID_ARG, "col or eid is NULL");
    if (n > 0 && !orig_id_out) return fail(AD_ERR_INVALID_ARG, "orig_id_out is NULL");
    if (w && m_in > 0 && !w_out) return fail(AD_ERR_INVALID_ARG, "w_out is NULL for a weighted list");
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    IngestLayout L;
    if (ingest_layout(n, m_in, ws, ws_bytes, &L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    return ingest_impl(n, m_in, u, v, w, orig_id, order, row_ptr, col, w_out, eid, orig_id_out, m_host, d_max_host,
                       n_dropped_host, L, stream);
}
