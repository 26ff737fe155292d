// ad_internal.h -- shared device/host helpers of libad (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

#include "../../include/ad.h"

namespace ad {

// ------------------------------------------------------------------ errors --

void set_error(const std::string &msg);
ad_status fail(ad_status s, const std::string &msg);
ad_status hip_fail(hipError_t e, const char *what);

#define AD_HIP(call)                                             \
    do {                                                         \
        hipError_t _e = (call);                                  \
        if (_e != hipSuccess) return ::ad::hip_fail(_e, #call);  \
    } while (0)

#define AD_LAUNCH_CHECK(what)                                    \
    do {                                                         \
        hipError_t _e = hipGetLastError();                       \
        if (_e != hipSuccess) return ::ad::hip_fail(_e, what);   \
    } while (0)

// --------------------------------------------------------------- workspace --

// Bump allocator over the caller's workspace; every slice is 256-byte aligned.
struct Carver {
    char *base;
    size_t cap;
    size_t used = 0;
    bool measuring;   // base == nullptr: only count bytes
    Carver(void *b, size_t c) : base((char *)b), cap(c), measuring(b == nullptr) {}
    template <typename T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        T *p = measuring ? nullptr : reinterpret_cast<T *>(base + used);
        used += bytes;
        return p;
    }
    bool ok() const { return measuring || used <= cap; }
};

// ---------------------------------------------------------------- numerics --

struct bf16 { uint16_t bits; };

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

// Round to nearest even; NaN stays NaN (quietened).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename T> struct acc_of { typedef float type; };
template <> struct acc_of<double> { typedef double type; };

// Vector of VEC storage elements, naturally aligned.
template <typename T, int VEC> struct alignas(sizeof(T) * VEC) vstore { T v[VEC]; };

template <int VEC, typename T, typename A>
__device__ __forceinline__ void load_vec(const T *p, A (&out)[VEC]) {
    vstore<T, VEC> t = *reinterpret_cast<const vstore<T, VEC> *>(p);
#pragma unroll
    for (int q = 0; q < VEC; ++q) out[q] = (A)t.v[q];
}
template <int VEC, typename A>
__device__ __forceinline__ void load_vec(const bf16 *p, A (&out)[VEC]) {
    vstore<uint16_t, VEC> t = *reinterpret_cast<const vstore<uint16_t, VEC> *>(p);
#pragma unroll
    for (int q = 0; q < VEC; ++q) out[q] = (A)bf16_to_f32(t.v[q]);
}
template <int VEC, typename T, typename A>
__device__ __forceinline__ void store_vec(T *p, const A (&in)[VEC]) {
    vstore<T, VEC> t;
#pragma unroll
    for (int q = 0; q < VEC; ++q) t.v[q] = (T)in[q];
    *reinterpret_cast<vstore<T, VEC> *>(p) = t;
}
template <int VEC, typename A>
__device__ __forceinline__ void store_vec(bf16 *p, const A (&in)[VEC]) {
    vstore<uint16_t, VEC> t;
#pragma unroll
    for (int q = 0; q < VEC; ++q) t.v[q] = f32_to_bf16((float)in[q]);
    *reinterpret_cast<vstore<uint16_t, VEC> *>(p) = t;
}

// Order-preserving map of a double onto uint64 (for min/max atomics).
__device__ __forceinline__ unsigned long long ord_encode(double x) {
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double ord_decode(unsigned long long u) {
    unsigned long long b = (u & 0x8000000000000000ull) ? (u & 0x7fffffffffffffffull) : ~u;
    double d;
    __builtin_memcpy(&d, &b, 8);
    return d;
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128-bit products; round keys advance by the Weyl constants.
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Uniform start value on the 2^-24 grid in [-1/2, 1/2) from a 64-bit word.
__device__ __forceinline__ double start_from_word(uint64_t w) {
    return (double)(w >> 40) * (1.0 / 16777216.0) - 0.5;
}

// ------------------------------------------------------------ wave helpers --

constexpr int WAVE = 64;

template <typename T>
__device__ __forceinline__ T shfl_down(T v, int delta) { return __shfl_down(v, delta, WAVE); }
template <typename T>
__device__ __forceinline__ T shfl(T v, int src) { return __shfl(v, src, WAVE); }

// Lanes per neighbour row (C) for R elements loaded VEC at a time.
inline int lanes_per_row(int R, int vec) { return (R + vec - 1) / vec; }

// Largest power of two p with p * c <= lanes.
inline int pow2_slots(int lanes, int c) {
    int p = 1;
    while (p * 2 * c <= lanes) p *= 2;
    return p;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__device__ __forceinline__ int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Grid for a grid-stride loop over `count` items.
inline unsigned grid_for(int64_t count, int block) {
    int64_t b = ceil_div(count, block);
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (unsigned)b;
}

// Slot in a list shared by the wave: lanes with `take` get consecutive
// slots from one atomic add on *counter (per wave, not per lane).
__device__ __forceinline__ unsigned int wave_append(bool take, unsigned int *counter) {
    const unsigned long long mask = __ballot(take);
    if (mask == 0) return 0;
    const int lane = threadIdx.x & (WAVE - 1);
    const int leader = __ffsll((long long)mask) - 1;
    unsigned int base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned int)__popcll(mask));
    base = __shfl(base, leader, WAVE);
    const unsigned long long below = lane ? (mask & ((1ull << lane) - 1)) : 0ull;
    return base + (unsigned int)__popcll(below);
}

// Small device fills (no hipMemsetAsync: the calls may be graph-captured).
ad_status fill_u64(unsigned long long *p, unsigned long long v, int64_t count, hipStream_t s);
ad_status fill_u8(uint8_t *p, uint8_t v, int64_t count, hipStream_t s);
ad_status fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s);

// Device-wide exclusive scan of v[0 .. count) in place, *total = the sum
// (three launches: per-block sums, a scan of those, per-block apply).  With
// weights w (may be NULL) it also fills splits[0 .. XCDS]: splits[0] = 0,
// splits[XCDS] = *total and, for 0 < x < XCDS, the scanned offset of the
// element after the one holding the point x / XCDS of the total weight.
constexpr int SCAN_PER_BLOCK = 1024;     // elements per block (256 threads x 4)
struct ScanScratch {
    unsigned int *blk_v;                 // [ceil(count / SCAN_PER_BLOCK)]
    unsigned long long *blk_w;           // same
    unsigned long long *total_w;         // [1]
};
size_t scan_scratch_blocks(int64_t count);
ad_status scan_exclusive(int64_t count, unsigned int *v, const unsigned long long *w, unsigned int *total,
                         unsigned int *splits, const ScanScratch &sc, hipStream_t s);

// Rows with lo < degree <= hi appended to list (count must start at 0).
ad_status collect_rows(const ad_graph *g, int64_t lo, int64_t hi, int32_t *list,
                       unsigned int *count, hipStream_t s);

ad_status check_graph_args(const ad_graph *g);

// Kernel timing for ad_trace_*: while tracing is on, a TraceScope brackets
// the launches made during its lifetime with HIP events on the stream.
struct TraceScope {
    const char *name;
    hipStream_t stream;
    int launches;                 // kernel launches the scope brackets (counted in the summary)
    hipEvent_t a = nullptr, b = nullptr;
    int dev = 0;                  // device of the events
    TraceScope(const char *name, hipStream_t s, int launches = 1);
    ~TraceScope();
};
// While one exists on this thread, TraceScope records nothing (used around
// stream capture and internal timing).
struct TraceSuppress {
    TraceSuppress();
    ~TraceSuppress();
};

// Graph segments: several independent graphs packed as one block-diagonal
// CSR (rows of graph g are [row_off[g], row_off[g+1])).  Per-graph work is
// laid out in chunks of CENTRE_ROWS rows and tiles of PLAN_TILE rows that
// start at each graph's first row, so every graph is processed exactly as
// it would be alone.  G = 1 with null arrays is a single graph.
struct Segs {
    int32_t G = 1;
    const int64_t *row_off = nullptr;    // [G+1]
    const int64_t *chunk_off = nullptr;  // [G+1] cumulative CENTRE_ROWS chunks
    const int64_t *tile_off = nullptr;   // [G+1] cumulative PLAN_TILE tiles
    const int32_t *row_graph = nullptr;  // [n] graph of each row
    int64_t nchunks = 0;                 // host copies of chunk_off[G], tile_off[G]
    int64_t ntiles = 0;
};

constexpr int CENTRE_ROWS = 1024;   // rows per centring / min-max chunk
constexpr int64_t COMP_CHUNK = 256;  // component members per centring chunk (ad_components)
constexpr int PLAN_TILE = 64;       // rows per launch-plan tile

// Shift of row i: per component (comp_of given; isolated rows 0), else the
// graph's.
__device__ __forceinline__ const double *row_shift(const double *__restrict__ shift,
                                                   const int32_t *__restrict__ comp_of, int64_t i, int g, int R,
                                                   bool &zero) {
    if (comp_of) {
        const int32_t c = comp_of[i];
        zero = c < 0;
        return shift + (int64_t)(c < 0 ? 0 : c) * R;
    }
    zero = false;
    return shift + (int64_t)g * R;
}

// Largest g in [0, G) with off[g] <= x (empty segments are skipped over).
__device__ __forceinline__ int seg_find(const int64_t *__restrict__ off, int G, int64_t x) {
    int lo = 0, hi = G - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Rows [r0, r1) and graph of chunk / tile `b` of size `size`.
__device__ __forceinline__ void seg_span(const Segs &sg, const int64_t *__restrict__ off, int64_t n, int64_t b,
                                         int64_t size, int &g, int64_t &r0, int64_t &r1) {
    if (off) {
        g = seg_find(off, sg.G, b);
        r0 = sg.row_off[g] + (b - off[g]) * size;
        r1 = min(sg.row_off[g + 1], r0 + size);
    } else {
        g = 0;
        r0 = b * size;
        r1 = min(n, r0 + size);
    }
}

// XCD-aware walk of a persistent grid over the launch-plan entries.  The
// hardware hands workgroups to the 8 XCDs round robin (workgroup b on XCD
// b % 8), each XCD with its own L2.  Main workgroup mb of nmb (numbered
// after a leading group of workgroups whose count is a multiple of 8)
// belongs to group mb % 8, and group x walks plan entries
// [splits[x], splits[x + 1]) -- contiguous ranges holding equal shares of
// the entries' edges -- with all its waves, so an XCD's waves work on
// neighbouring rows (for packed batches: on the same few graphs) at any
// time.  Every entry is visited once whatever the placement.  With
// xcd_groups == 1 (or fewer than 8 main workgroups) one group walks [0, np)
// cyclically: on a single graph without row locality (a random power-law
// graph stored by degree) that keeps the XCDs' loads even and measures
// faster; packed batches of small graphs use the 8 groups.
constexpr unsigned int XCDS = 8;
constexpr int MAX_DEVICES = 64;
constexpr int QUEUE_PAD = 32;                          // words between counters (one 128-byte line)
constexpr int QUEUE_GROUPS = 64;                       // counters per queue (hub rows, plan chunks)
constexpr int QUEUE_SET = 2 * QUEUE_GROUPS * QUEUE_PAD;
constexpr int QUEUE_SLOTS = 3;
struct PlanWalk {
    unsigned long long first, end, stride;
};
__device__ __forceinline__ PlanWalk plan_walk(unsigned int np, const unsigned int *__restrict__ splits,
                                              int xcd_groups, unsigned int mb, unsigned int nmb, int wave,
                                              int waves_per_block) {
    const unsigned int groups = (xcd_groups > 1 && nmb >= XCDS) ? XCDS : 1u;
    const unsigned int x = mb % groups, lb = mb / groups;
    const unsigned int nb = (nmb - x + groups - 1) / groups;    // workgroups in group x
    PlanWalk w;
    const unsigned long long a = groups == 1 ? 0ull : splits[x];
    w.end = groups == 1 ? (unsigned long long)np : (unsigned long long)splits[x + 1];
    w.first = a + (unsigned long long)lb * waves_per_block + wave;
    w.stride = (unsigned long long)nb * waves_per_block;
    return w;
}
inline int64_t round_up_xcds(int64_t v) { return (v + XCDS - 1) / XCDS * XCDS; }

// Launch shape and plan of a JOR sweep (see ad_relax.hip).
struct SweepShape {
    int vec, C, SPRW;     // values per lane, lanes per neighbour row, slots per wave
    int rpw_fixed;        // 0: rows per wave chosen per tile
    int64_t hub_d;        // rows longer than this get a workgroup each
    int upper_only = 0;   // rows per wave from the upper entries (j > i) only
};

// First entry of row `row` in [beg, end) whose column exceeds the row: the
// upper entries (j > i) are that suffix, columns being ascending in a row.
__device__ __forceinline__ int64_t upper_start(const int32_t *__restrict__ col, int64_t beg, int64_t end,
                                               int64_t row) {
    int64_t lo = beg, hi = end;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)col[mid] > row) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}
SweepShape sweep_shape(int R, size_t in_bytes, int rpw_req, int64_t hub_req);

struct SweepPlan {
    SweepShape sh;
    int32_t *hub_list;
    unsigned int *hub_count;
    long long *plan;            // (first row << 16) | (rows << 8) | log2(rows per wave), per wave
    unsigned int *plan_count;
    unsigned int *splits;       // [XCDS + 1] plan offsets of the XCD groups' ranges
    // QUEUE_SLOTS sets of work-queue counters (QUEUE_SET words each); sweep
    // launch t on this plan uses set t mod QUEUE_SLOTS and clears the set launch
    // t + 2 uses (that of launch t - 1, finished by stream order)
    unsigned int *queue;
    mutable unsigned int turn = 0;
    int xcd_groups = 1;         // XCDS for packed batches of several graphs, else 1
    unsigned long long *tile_nnz;  // [ntiles] planned entries (non-hub; upper only if so planned)
    ScanScratch scan;
    int *tile_lg;
    unsigned int *tile_waves;
};
// ntiles_cap: tiles of the layout (ceil(n / PLAN_TILE) for one graph).
size_t sweep_plan_bytes(int64_t n, int64_t ntiles_cap);
void sweep_plan_carve(Carver &c, int64_t n, int64_t ntiles_cap, SweepPlan &p);
// Builds the hub list (if build_hubs) and the per-tile plan on the stream.
ad_status sweep_plan_build(const ad_graph *g, SweepPlan &p, bool build_hubs, const Segs &sg, hipStream_t st);

// The whole relaxation of ad_relax over packed graph segments: minmax_out
// [G][2R], shift_out [G][R]; graph g's start vectors use key word
// o->graph_id + g.
size_t relax_segs_workspace(const ad_graph *g, const ad_relax_opts *o, const Segs &sg);
ad_status relax_segs(const ad_graph *g, const ad_relax_opts *o, const void *x0, void *x_out, double *minmax_out,
                     double *shift_out, void *ckpt, void *ws, size_t ws_bytes, const Segs &sg, hipStream_t st);

// ad_edge_dist over packed graph segments (minmax [G][2R]).  With rho_ent
// (FP32 rho only) every CSR entry's distance is also written there, in
// entry order, from a pass over whole rows.
size_t edge_dist_segs_workspace(const ad_graph *g, const Segs &sg);
ad_status edge_dist_segs(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x, const double *minmax,
                         ad_dtype rho_dtype, void *rho, void *ws, size_t ws_bytes, const Segs &sg,
                         hipStream_t stream, float *rho_ent = nullptr);

// Connected components by union-find: parent[i] = the smallest vertex of
// i's component (flags unused, may be NULL).
ad_status label_components(const ad_graph *g, int32_t *parent, unsigned int *flags, hipStream_t stream);

// Algorithm 3 at fixed per-degree budgets, keep[] only (rows are independent,
// so packed graphs need no segment information).
size_t sparsify_workspace(const ad_graph *g);
ad_status sparsify_fixed(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                         const int32_t *budget, uint8_t *keep, void *ws, size_t ws_bytes, hipStream_t stream);

// xout = (1 - omega) xin + omega * diag(inv_s) W xin, FP32.
ad_status sweep_f32(const ad_graph *g, const float *inv_s, float omega, const float *xin, float *xout, int R,
                    const SweepPlan &plan, hipStream_t st);
// s_i and 1/s_i; rows longer than the plan's hub degree come from its hub list.
ad_status weighted_degree_f32(const ad_graph *g, float *inv_s, float *sdeg, const SweepPlan &pl, hipStream_t st);

}  // namespace ad
