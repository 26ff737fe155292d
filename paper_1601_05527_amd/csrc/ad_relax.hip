// ad_relax.hip -- start vectors, JOR sweeps and the rescale statistics of
// Algorithm 1 (ComputeAlgDist) on gfx950.
//
// Data layout: the R test vectors are stored as one row-major block X[n][R],
// so the R values of a vertex are contiguous (R * sizeof(T) bytes) and one
// gather of a neighbour row serves all R vectors.  A sweep is a sparse-times-
// dense product over the CSR: for row i, C lanes cover the R values of one
// neighbour (VEC values per lane, 16-byte loads), SPR such lane groups
// ("slots") walk the neighbour list in parallel, and a shuffle tree combines
// the slots.  Rows longer than `hub_d` go to a second kernel that gives each
// of them a 256-thread workgroup.  Arithmetic order is fixed, so results are
// bitwise repeatable.
//
// Numerics: the start block is shifted per vector -- and, given the graph's
// connected components, per component -- by the weighted mean
// sum_i s_i x_i / sum_i s_i over the component, rounded to the 2^-24 grid.
// The sweep matrix keeps every vector that is constant on each component
// fixed, so this changes x^(k) by exactly those constants (the start values
// lie on the same grid, so the subtraction itself is exact) and leaves the
// rescaled vectors unchanged, while the sweeps work on differences from each
// component's conserved mean.  Their rounding errors then scale with how far
// a component still is from its limit: a small component that has nearly
// converged keeps its own tiny differences, which a single graph-wide shift
// would drown in the rounding of its distance from the graph-wide mean.
// Storage rounding of the last sweeps is the other limit of FP32 vectors;
// the last fp64_tail sweeps are therefore stored and computed in FP64.
#include "ad_internal.h"

#include <math.h>

#include <algorithm>
#include <atomic>

namespace ad {

constexpr int BLOCK = 256;
constexpr int MM_SLOTS = 16;       // copies of each graph's min / max codes (k_minmax)
constexpr int MM_SPLIT = 4;        // k_minmax blocks per CENTRE_ROWS chunk
constexpr int SWEEP_UNROLL = 8;     // row gathers in flight per lane

// s_i = sum_j w_ij in FP64 (LPR lanes per row, strided partial sums combined
// by a fixed shuffle tree).  FP32 sweeps multiply by inv_s = 1/s_i (0 for
// isolated vertices); FP64 sweeps divide by s_i, which they read from inv_s
// (A == double) or from s64.
template <typename A>
__device__ __forceinline__ A sweep_scale(double s) {
    if constexpr (sizeof(A) == 8) return (A)s;
    else return s > 0.0 ? (A)(1.0 / s) : (A)0;
}
template <typename A>
__device__ __forceinline__ A neighbour_avg(A acc, A is) {
    if constexpr (sizeof(A) == 8) return acc / is;    // correctly rounded quotient
    else return acc * is;
}

template <typename A>
__global__ __launch_bounds__(BLOCK) void k_weighted_degree(int64_t n, const int64_t *__restrict__ row_ptr,
                                                          const float *__restrict__ w, A *__restrict__ inv_s,
                                                          float *__restrict__ sdeg, double *__restrict__ s64,
                                                          int LPR, int64_t hub_d) {
    const int64_t i = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    int64_t b = 0, e = 0;
    if (i < n) {
        b = row_ptr[i];
        e = row_ptr[i + 1];
    }
    if (e - b > hub_d) return;      // whole row group is one hub row: k_weighted_degree_hub
    double s = 0.0;
    if (w) {
        // four loads in flight per lane, added in entry order
        int64_t p = b + lane;
        for (; p + 3 * LPR < e; p += 4 * (int64_t)LPR) {
            const float w0 = w[p], w1 = w[p + LPR], w2 = w[p + 2 * LPR], w3 = w[p + 3 * LPR];
            s += (double)w0;
            s += (double)w1;
            s += (double)w2;
            s += (double)w3;
        }
        for (; p < e; p += LPR) s += (double)w[p];
    } else if (lane == 0) {
        s = (double)(e - b);
    }
    for (int d = LPR >> 1; d >= 1; d >>= 1) s += shfl_down(s, d);
    if (i < n && lane == 0) {
        inv_s[i] = sweep_scale<A>(e > b ? s : 0.0);
        sdeg[i] = (float)s;
        if (s64) s64[i] = s;
    }
}

// s_i for the listed long rows: a workgroup per row, strided FP64 partial
// sums combined by a fixed tree in LDS.
template <typename A>
__global__ __launch_bounds__(BLOCK) void k_weighted_degree_hub(const int32_t *__restrict__ list,
                                                              const unsigned int *__restrict__ count,
                                                              const int64_t *__restrict__ row_ptr,
                                                              const float *__restrict__ w, A *__restrict__ inv_s,
                                                              float *__restrict__ sdeg, double *__restrict__ s64) {
    __shared__ double part[BLOCK];
    const unsigned int nh = *count;
    for (unsigned int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int64_t i = list[h];
        const int64_t b = row_ptr[i], e = row_ptr[i + 1];
        double s = 0.0;
        if (w) {
            int64_t p = b + threadIdx.x;
            for (; p + 3 * BLOCK < e; p += 4 * BLOCK) {
                const float w0 = w[p], w1 = w[p + BLOCK], w2 = w[p + 2 * BLOCK], w3 = w[p + 3 * BLOCK];
                s += (double)w0;
                s += (double)w1;
                s += (double)w2;
                s += (double)w3;
            }
            for (; p < e; p += BLOCK) s += (double)w[p];
        } else if (threadIdx.x == 0) {
            s = (double)(e - b);
        }
        part[threadIdx.x] = s;
        __syncthreads();
        for (int d = BLOCK / 2; d >= 1; d >>= 1) {
            if ((int)threadIdx.x < d) part[threadIdx.x] += part[threadIdx.x + d];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            inv_s[i] = sweep_scale<A>(part[0]);
            sdeg[i] = (float)part[0];
            if (s64) s64[i] = part[0];
        }
        __syncthreads();
    }
}

static int degree_lanes(double avg) {
    int lpr = 1;
    while (lpr < 16 && lpr < avg) lpr <<= 1;
    return lpr;
}


// Partial sums of s_i * x_i^(0) (per vector) and of s_i over CENTRE_ROWS
// rows.  Thread (row offset, q) handles the Philox block q, i.e. vectors
// 4q .. 4q+3, of its rows; the block then adds per vector in thread order.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_centre_partials(int64_t n, int R, const float *__restrict__ sdeg,
                                                          const int32_t *__restrict__ orig_id, uint64_t seed,
                                                          uint64_t gid, const T *__restrict__ x0,
                                                          double *__restrict__ part, double *__restrict__ part_s,
                                                          Segs sg) {
    __shared__ double acc_l[4][BLOCK];
    __shared__ double s_l[BLOCK];
    const int t = threadIdx.x;
    const int nq = (R + 3) >> 2;
    const int stride = BLOCK / nq;           // rows visited per step
    const int q = t % nq;
    const int row_off = t / nq;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double sacc = 0.0;
    int g;
    int64_t r0, r1;
    seg_span(sg, sg.chunk_off, n, blockIdx.x, CENTRE_ROWS, g, r0, r1);
    const uint64_t gkey = gid + (uint64_t)g;
    if (row_off < stride) {
        for (int64_t i = r0 + row_off; i < r1; i += stride) {
            const double s = (double)sdeg[i];
            if (x0) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (4 * q + c < R) acc[c] += s * (double)x0[i * R + 4 * q + c];
            } else {
                uint64_t words[4];
                const int32_t key = orig_id ? orig_id[i] : (int32_t)i;
                philox4x64_10((uint64_t)(uint32_t)key, (uint64_t)q, 0, 0, seed, gkey, words);
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += s * start_from_word(words[c]);
            }
            sacc += s;
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) acc_l[c][t] = acc[c];
    s_l[t] = sacc;
    __syncthreads();
    if (t < R) {
        const int qq = t >> 2, c = t & 3;
        double a = 0.0;
        for (int u = qq; u < stride * nq; u += nq) a += acc_l[c][u];
        part[(int64_t)blockIdx.x * R + t] = a;
    }
    if (t == 0) {
        double a = 0.0;
        for (int u = 0; u < stride * nq; u += nq) a += s_l[u];
        part_s[blockIdx.x] = a;
    }
}

// shift_r = weighted mean rounded to the 2^-24 grid; resets the min/max codes.
// One block per graph: thread t sums the graph's partial blocks t, t+BLOCK,
// ... in order, then thread 0 adds the BLOCK subtotals in order (a fixed
// summation tree).
__global__ __launch_bounds__(BLOCK) void k_centre_finalize(int R, int64_t nblocks, const double *__restrict__ part,
                                                          const double *__restrict__ part_s, int centre,
                                                          double *__restrict__ shift,
                                                          unsigned long long *__restrict__ mm, Segs sg) {
    __shared__ double sub[BLOCK];
    __shared__ double S;
    const int t = threadIdx.x;
    const int g = blockIdx.x;
    const int64_t c0 = sg.chunk_off ? sg.chunk_off[g] : 0;
    const int64_t c1 = sg.chunk_off ? sg.chunk_off[g + 1] : nblocks;
    double a = 0.0;
    for (int64_t b = c0 + t; b < c1; b += BLOCK) a += part_s[b];
    sub[t] = a;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int q = 0; q < BLOCK; ++q) tot += sub[q];
        S = tot;
    }
    __syncthreads();
    for (int r = 0; r < R; ++r) {
        a = 0.0;
        for (int64_t b = c0 + t; b < c1; b += BLOCK) a += part[b * R + r];
        sub[t] = a;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int q = 0; q < BLOCK; ++q) tot += sub[q];
            double sh = 0.0;
            if (centre && S > 0.0) sh = rint((tot / S) * 16777216.0) * (1.0 / 16777216.0);
            shift[(int64_t)g * R + r] = sh;
            for (int sl = 0; sl < MM_SLOTS; ++sl) {
                unsigned long long *m_ = mm + ((int64_t)sl * sg.G + g) * 2 * R;
                m_[r] = ~0ull;                        // running min code
                m_[R + r] = 0ull;                     // running max code
            }
        }
        __syncthreads();
    }
}

// Per-component centring.  The members of every component (ad_components)
// are cut into chunks of COMP_CHUNK; one wave sums a chunk: lane l takes
// members l, l + 64, ... of the chunk in that order, and a fixed shuffle
// tree adds the lanes, so the sums depend only on the grouping.

__device__ __forceinline__ double wave_sum(double v) {
    for (int d = WAVE / 2; d >= 1; d >>= 1) v += shfl_down(v, d);
    return v;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_comp_partials(int R, int64_t n_comp, int64_t n_chunks,
                                                        const int32_t *__restrict__ members,
                                                        const int64_t *__restrict__ comp_start,
                                                        const int64_t *__restrict__ chunk_start,
                                                        const float *__restrict__ sdeg,
                                                        const int32_t *__restrict__ orig_id, uint64_t seed,
                                                        uint64_t gid, const T *__restrict__ x0,
                                                        const int32_t *__restrict__ row_graph,
                                                        double *__restrict__ part, double *__restrict__ part_s) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t ch = (int64_t)blockIdx.x * (BLOCK / WAVE) + (threadIdx.x >> 6);
    if (ch >= n_chunks) return;                      // uniform across the wave
    int64_t lo = 0, hi = n_comp - 1;                 // last component starting at or before ch
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (chunk_start[mid] <= ch) lo = mid;
        else hi = mid - 1;
    }
    const int64_t p0 = comp_start[lo] + (ch - chunk_start[lo]) * COMP_CHUNK;
    const int64_t p1 = min(comp_start[lo + 1], p0 + COMP_CHUNK);
    double sacc = 0.0;
    for (int64_t p = p0 + lane; p < p1; p += WAVE) sacc += (double)sdeg[members[p]];
    sacc = wave_sum(sacc);
    if (lane == 0) part_s[ch] = sacc;
    const int nq = (R + 3) >> 2;
    for (int q = 0; q < nq; ++q) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t p = p0 + lane; p < p1; p += WAVE) {
            const int32_t i = members[p];
            const double s = (double)sdeg[i];
            if (x0) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (4 * q + c < R) acc[c] += s * (double)x0[(int64_t)i * R + 4 * q + c];
            } else {
                uint64_t words[4];
                const int32_t key = orig_id ? orig_id[i] : i;
                const uint64_t g = row_graph ? (uint64_t)row_graph[i] : 0ull;
                philox4x64_10((uint64_t)(uint32_t)key, (uint64_t)q, 0, 0, seed, gid + g, words);
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += s * start_from_word(words[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double v = wave_sum(acc[c]);
            if (lane == 0 && 4 * q + c < R) part[ch * R + 4 * q + c] = v;
        }
    }
}

// Sums over the chunks of component c (chunk partials part[ch][r] and
// part_s[ch]) for one wave: lane l adds chunks c0 + l, c0 + l + 64, ... in
// that order (eight loads in flight per lane), then a fixed shuffle tree
// adds the lanes.  The order depends only on the component's chunk range.
__device__ __forceinline__ void comp_chunk_sums(int64_t c0, int64_t c1, int R, int r,
                                                const double *__restrict__ part,
                                                const double *__restrict__ part_s, double &S, double &X) {
    const int lane = threadIdx.x & (WAVE - 1);
    constexpr int B = 8;
    double s = 0.0, x = 0.0;
    int64_t ch = c0 + lane;
    for (; ch + (int64_t)(B - 1) * WAVE < c1; ch += (int64_t)B * WAVE) {
        double a[B], b[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            b[u] = part_s[ch + (int64_t)u * WAVE];
            a[u] = part[(ch + (int64_t)u * WAVE) * R + r];
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            s += b[u];
            x += a[u];
        }
    }
    for (; ch < c1; ch += WAVE) {
        s += part_s[ch];
        x += part[ch * R + r];
    }
    S = wave_sum(s);
    X = wave_sum(x);
}

// shift[c][r] = the weighted mean of component c rounded to the 2^-24 grid:
// one wave per (component, vector).
__global__ __launch_bounds__(BLOCK) void k_comp_finalize(int R, int64_t n_comp, const int64_t *__restrict__ chunk_start,
                                                        const double *__restrict__ part,
                                                        const double *__restrict__ part_s, int centre,
                                                        double *__restrict__ shift) {
    const int64_t pairs = n_comp * R;
    for (int64_t idx = (int64_t)blockIdx.x * (BLOCK / WAVE) + (threadIdx.x >> 6); idx < pairs;
         idx += (int64_t)gridDim.x * (BLOCK / WAVE)) {     // uniform across the wave
        const int64_t c = idx / R;
        const int r = (int)(idx - c * R);
        double S, X;
        comp_chunk_sums(chunk_start[c], chunk_start[c + 1], R, r, part, part_s, S, X);
        if ((threadIdx.x & (WAVE - 1)) == 0)
            shift[idx] = (centre && S > 0.0) ? rint((X / S) * 16777216.0) * (1.0 / 16777216.0) : 0.0;
    }
}

// Current weighted mean of every component (the BF16 re-centring): one wave
// per chunk sums s_i x_i per vector over the chunk's members as
// k_comp_partials does (G vectors per pass); k_comp_drift then adds the
// chunks of each component as comp_chunk_sums does, keeps c = mean rounded
// to FP32 for the next sweep to subtract, and adds c to the component's shift.
template <typename T, int G>
__global__ __launch_bounds__(BLOCK) void k_comp_drift_partials(int R, int64_t n_comp, int64_t n_chunks,
                                                              const int32_t *__restrict__ members,
                                                              const int64_t *__restrict__ comp_start,
                                                              const int64_t *__restrict__ chunk_start,
                                                              const float *__restrict__ sdeg,
                                                              const T *__restrict__ x, double *__restrict__ part) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t ch = (int64_t)blockIdx.x * (BLOCK / WAVE) + (threadIdx.x >> 6);
    if (ch >= n_chunks) return;                      // uniform across the wave
    int64_t lo = 0, hi = n_comp - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (chunk_start[mid] <= ch) lo = mid;
        else hi = mid - 1;
    }
    const int64_t p0 = comp_start[lo] + (ch - chunk_start[lo]) * COMP_CHUNK;
    const int64_t p1 = min(comp_start[lo + 1], p0 + COMP_CHUNK);
    // G vectors per pass (G divides R), read with one load per member
    for (int q0 = 0; q0 < R; q0 += G) {
        double acc[G];
#pragma unroll
        for (int c = 0; c < G; ++c) acc[c] = 0.0;
        for (int64_t p = p0 + lane; p < p1; p += WAVE) {
            const int32_t i = members[p];
            const double s = (double)sdeg[i];
            float v[G];
            load_vec<G>(x + (int64_t)i * R + q0, v);
#pragma unroll
            for (int c = 0; c < G; ++c) acc[c] += s * (double)v[c];
        }
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const double v = wave_sum(acc[c]);
            if (lane == 0) part[ch * R + q0 + c] = v;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_comp_drift(int R, int64_t n_comp, const int64_t *__restrict__ chunk_start,
                                                     const double *__restrict__ part,
                                                     const double *__restrict__ part_s, float *__restrict__ drift,
                                                     double *__restrict__ shift) {
    const int64_t pairs = n_comp * R;
    for (int64_t idx = (int64_t)blockIdx.x * (BLOCK / WAVE) + (threadIdx.x >> 6); idx < pairs;
         idx += (int64_t)gridDim.x * (BLOCK / WAVE)) {     // uniform across the wave
        const int64_t c = idx / R;
        const int r = (int)(idx - c * R);
        double S, X;
        comp_chunk_sums(chunk_start[c], chunk_start[c + 1], R, r, part, part_s, S, X);
        if ((threadIdx.x & (WAVE - 1)) == 0) {
            const float d = S > 0.0 ? (float)(X / S) : 0.0f;
            drift[idx] = d;
            shift[idx] += (double)d;
        }
    }
}

// The running min / max codes of every graph (MM_SLOTS copies) start empty.
__global__ void k_mm_reset(int64_t count, int R, unsigned long long *__restrict__ mm) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    mm[idx] = ((idx / R) % 2 == 0) ? ~0ull : 0ull;
}

// x^(0) - shift into the start buffer.  One Philox block feeds 4 vectors.
template <typename T, typename Tx>
__global__ void k_init(int64_t n, int R, const int32_t *__restrict__ orig_id, uint64_t seed,
                       uint64_t gid, const T *__restrict__ x0, const double *__restrict__ shift,
                       const int32_t *__restrict__ comp_of, Tx *__restrict__ x,
                       const int32_t *__restrict__ row_graph) {
    const int nq = (R + 3) >> 2;
    const int64_t total = n * nq;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / nq;
        int q = (int)(idx - i * nq);
        const int g = row_graph ? row_graph[i] : 0;
        uint64_t words[4];
        if (!x0) {
            int32_t key = orig_id ? orig_id[i] : (int32_t)i;
            philox4x64_10((uint64_t)(uint32_t)key, (uint64_t)q, 0, 0, seed, gid + (uint64_t)g, words);
        }
        bool zero;
        const double *sh = row_shift(shift, comp_of, i, g, R, zero);
        for (int c = 0; c < 4; ++c) {
            int r = 4 * q + c;
            if (r >= R) break;
            double v = x0 ? (double)x0[i * R + r] : start_from_word(words[c]);
            x[i * R + r] = (Tx)(zero ? v : v - sh[r]);
        }
    }
}

// Re-centring of BF16 sweeps: every component's current weighted mean c
// (FP32, per vector) is subtracted from the sweep's output rows.  The sweep
// matrix maps the component-constant vector c to itself, so the result is
// x^(t) - c exactly up to rounding, a change of frame that the relaxation
// adds to the component's shift; the stored values stay on the scale of
// the component's own differences instead of on that of the mean drift that
// BF16 rounding accumulates.
struct SweepDrift {
    const float *c = nullptr;         // [n_comp][R], or NULL: none
    const int32_t *comp_of = nullptr; // [n]
};
template <typename A, int VEC>
__device__ __forceinline__ void apply_drift(const SweepDrift &dr, int64_t row, int R, int off, A (&res)[VEC]) {
    if (!dr.c) return;
    const int32_t c = dr.comp_of[row];
    if (c < 0) return;
    const float *d = dr.c + (int64_t)c * R + off;
#pragma unroll
    for (int q = 0; q < VEC; ++q) res[q] -= (A)d[q];
}

// One lane's part of a launch-plan entry (first row << 16 | rows in the
// entry << 8 | log2 rows per wave): its row, slot of C lanes within the
// row's SPR slots, and chunk of the R values.
struct EntryLane {
    int64_t row;
    int SPR, slot, chunk;
    bool active;
};
__device__ __forceinline__ EntryLane entry_lane(long long e, int lane, int C, int SPRW) {
    EntryLane q;
    const int nrows = (int)((e >> 8) & 0xff);
    q.SPR = SPRW >> (int)(e & 0xff);
    const int group = C * q.SPR;
    const int rw = lane / group;
    const int sub = lane - rw * group;
    q.slot = sub / C;
    q.chunk = sub - q.slot * C;
    q.row = (e >> 16) + rw;
    q.active = rw < nrows;
    return q;
}

// Registers a gathered value is held in until it is used: its stored type,
// except BF16, which is widened on load.
template <typename T> struct held_of { typedef T type; };
template <> struct held_of<bf16> { typedef float type; };

// Accumulate sum_j w_ij x_j over the entries p0, p0 + stride, p0 + 2 stride,
// ... < end into acc (VEC values of one lane's chunk), in that order.  U
// column/weight pairs are loaded first, then U gathers are issued together,
// so each lane keeps U row reads in flight.  Gathered values stay in their
// stored width until the FMA, so an FP32 row summed in FP64 holds half the
// registers.
template <int U, int VEC, typename Tin, typename A>
__device__ __forceinline__ void gather_rows(const int32_t *__restrict__ col, const float *__restrict__ w,
                                            const Tin *__restrict__ xin, int64_t p0, int64_t end,
                                            int64_t stride, int R, int off, A (&acc)[VEC]) {
    for (int64_t p = p0; p < end; p += (int64_t)U * stride) {
        int32_t jj[U];
        A ww[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + u * stride;
            const bool ok = q < end;
            jj[u] = ok ? col[q] : -1;
            ww[u] = ok ? (w ? (A)w[q] : (A)1) : (A)0;
        }
        typedef typename held_of<Tin>::type H;
        H v[U][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (jj[u] >= 0) {
                load_vec<VEC>(xin + (int64_t)jj[u] * R + off, v[u]);
            } else {
#pragma unroll
                for (int q = 0; q < VEC; ++q) v[u][q] = (H)0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = fma(ww[u], (A)v[u][q], acc[q]);
        }
    }
}

// Work queues of a sweep launch (one set of counters per launch, see
// SweepPlan::queue): QUEUE_GROUPS counters hand out hub rows (group g owns
// list positions g, g + QUEUE_GROUPS, ...) and QUEUE_GROUPS more hand out
// chunks of SWEEP_CHUNK plan entries.  For packed batches the first XCDS
// plan groups are the XCD groups, group g's chunk k being entries splits[g]
// + k CH ... of its edge-balanced range; otherwise group g's chunk k is
// entries (g + QUEUE_GROUPS k) CH ... of the whole plan.  Spreading the
// tickets over many counters keeps each counter's atomics few: they are
// served one at a time per address.
constexpr int SWEEP_CHUNK = 4;
constexpr unsigned int NO_CHUNK = 0xffffffffu;

__device__ __forceinline__ bool chunk_range(bool contig, const unsigned int *__restrict__ splits, unsigned int np,
                                            int g, unsigned int k, unsigned int &lo, unsigned int &hi) {
    const unsigned long long a = contig ? splits[g] : 0ull;
    const unsigned long long b = contig ? splits[g + 1] : (unsigned long long)np;
    const unsigned long long c =
        contig ? (unsigned long long)k : (unsigned long long)g + (unsigned long long)QUEUE_GROUPS * k;
    const unsigned long long first = a + c * SWEEP_CHUNK;
    if (first >= b) return false;
    lo = (unsigned int)first;
    hi = (unsigned int)std::min<unsigned long long>(first + SWEEP_CHUNK, b);
    return true;
}

__device__ __forceinline__ bool hub_item(int g, unsigned int k, unsigned int nh, unsigned int &h) {
    const unsigned long long i = (unsigned long long)g + (unsigned long long)QUEUE_GROUPS * k;
    if (i >= nh) return false;
    h = (unsigned int)i;
    return true;
}

// One ticket from a queue counter for the whole wave (all lanes active).
__device__ __forceinline__ unsigned int wave_ticket(unsigned int *q, int lane) {
    unsigned int v = 0;
    if (lane == 0) v = atomicAdd(q, 1u);
    return (unsigned int)__builtin_amdgcn_readfirstlane((int)v);
}

// A wave (all lanes active) takes its next item: `pending` is a ticket
// already drawn from group grp (or NO_CHUNK), and item(g, k, out) says
// whether ticket k of group g names an item.  When group grp is exhausted,
// the wave's lanes read every group's counter at once and the wave moves to
// the first group from grp on that still has items.  Returns false once no
// group has any.  Ends: a failed draw only happens on a group that had
// items when probed, and the items are finite.
template <typename Item>
__device__ __forceinline__ bool take_item(unsigned int *ctr, int ngroups, int &grp, unsigned int pending,
                                          int lane, Item item, unsigned int &out0, unsigned int &out1) {
    unsigned int k = pending;
    for (;;) {
        if (k == NO_CHUNK) k = wave_ticket(ctr + grp * QUEUE_PAD, lane);
        if (item(grp, k, out0, out1)) return true;
        bool left = false;
        if (lane < ngroups) {
            int g2 = grp + lane;
            if (g2 >= ngroups) g2 -= ngroups;
            const unsigned int v =
                __hip_atomic_load(ctr + g2 * QUEUE_PAD, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned int d0, d1;
            left = item(g2, v, d0, d1);
        }
        const unsigned long long mask = __ballot(left);
        if (mask == 0) return false;
        grp += __ffsll((long long)mask) - 1;
        if (grp >= ngroups) grp -= ngroups;
        k = NO_CHUNK;
    }
}

__device__ __forceinline__ long long lane_word(long long v, int i) {
    const int lo = __builtin_amdgcn_readlane((int)(unsigned int)v, i);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), i);
    return (long long)(((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo);
}

// Waves per SIMD the sweep is compiled for: four with up to four values
// per lane (the FP32 and BF16 forms at R <= 16, the FP64 forms with their
// halved unroll), which fits the register budget of four waves without
// spilling; no request otherwise.
template <typename A, int VEC>
constexpr int sweep_waves_per_eu() {
    return VEC <= 4 ? 4 : 1;
}

// One JOR sweep over all rows, in one launch.  Long rows (degree > hub_d)
// get a 256-thread workgroup each: SPRW slots per wave, partial sums
// combined across the 4 waves in LDS.  The other rows follow the launch plan
// (see below): per wave 2^lg rows, per row SPRW / 2^lg slots of C lanes, VEC
// values per lane.  Each row is summed by one wave (or one workgroup) in a
// fixed order, so the result does not depend on which wave takes it.
//
// Static walk (!QUEUED, one graph): blocks [0, hub_blocks) take the listed
// long rows, strided, and come first so the longest work starts first;
// blocks [hub_blocks, ...) walk the plan as a persistent grid.
//
// Queued walk (QUEUED, packed batches): a grid no larger than the device
// holds at once; every workgroup first takes long rows from the hub queue,
// then its waves take chunks of the plan from the XCD groups' queues, so
// uneven graphs and rows even out over the whole device.  Block 0 also
// clears the counters the launch after next will use.
template <typename Tin, typename Tout, typename A, int VEC, int U, bool QUEUED>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sweep_waves_per_eu<A, VEC>()))) void k_sweep(
    int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const float *__restrict__ w, const A *__restrict__ inv_s, A omega,
    const Tin *__restrict__ xin, Tout *__restrict__ xout, int R, int C,
    int64_t hub_d, int SPRW, int hub_blocks, const int32_t *__restrict__ hub_list,
    const unsigned int *__restrict__ hub_count, const long long *__restrict__ plan,
    const unsigned int *__restrict__ plan_count, const unsigned int *__restrict__ splits, int xcd_groups,
    unsigned int *__restrict__ queue, unsigned int *__restrict__ queue_clear, SweepDrift dr) {
    __shared__ A part[BLOCK / WAVE][64];
    __shared__ unsigned int s_row;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    const A keep = (A)1 - omega;
    if constexpr (!QUEUED) {
    if ((int)blockIdx.x < hub_blocks) {
        const int slot_w = lane / C;
        const int chunk = lane - slot_w * C;
        const bool lane_on = slot_w < SPRW;
        const int slots = SPRW * (BLOCK / WAVE);
        const int slot = wave * SPRW + slot_w;
        const int off = chunk * VEC;
        const unsigned int nh = *hub_count;
        for (unsigned int h = blockIdx.x; h < nh; h += hub_blocks) {
            const int64_t row = hub_list[h];
            const int64_t beg = row_ptr[row], end = row_ptr[row + 1];
            A acc[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = (A)0;
            if (lane_on) gather_rows<U, VEC>(col, w, xin, beg + slot, end, slots, R, off, acc);
            for (int d = SPRW >> 1; d >= 1; d >>= 1) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) acc[q] += shfl_down(acc[q], d * C);
            }
            if (lane_on && slot_w == 0) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) part[wave][off + q] = acc[q];
            }
            __syncthreads();
            if (wave == 0 && lane_on && slot_w == 0) {
                A sum[VEC], own[VEC], res[VEC];
#pragma unroll
                for (int q = 0; q < VEC; ++q) sum[q] = part[0][off + q];
                for (int wv = 1; wv < BLOCK / WAVE; ++wv) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) sum[q] += part[wv][off + q];
                }
                load_vec<VEC>(xin + row * R + off, own);
                const A is = inv_s[row];
#pragma unroll
                for (int q = 0; q < VEC; ++q) res[q] = fma(omega, neighbour_avg(sum[q], is), keep * own[q]);
                apply_drift(dr, row, R, off, res);
                store_vec<VEC>(xout + row * R + off, res);
            }
            __syncthreads();
        }
        return;
    }
    // Other rows: waves walk plan entries (first row, rows in the tile, log2 rows per
    // wave) in XCD groups (plan_walk); SPRW / rpw slots of C lanes per row.  The
    // walk is software-pipelined: while an entry's columns and rows are read, the
    // row bounds of the next entry and the plan word of the one after are
    // already in flight, so each entry waits on two dependent reads, not four.
    const PlanWalk pw = plan_walk(*plan_count, splits, xcd_groups, blockIdx.x - hub_blocks, gridDim.x - hub_blocks,
                                  wave, BLOCK / WAVE);
    const unsigned long long stride = pw.stride;
    unsigned long long pi = pw.first;
    long long e_cur = pi < pw.end ? plan[pi] : 0;
    long long e_nxt = pi + stride < pw.end ? plan[pi + stride] : 0;
    EntryLane cur = entry_lane(e_cur, lane, C, SPRW);
    int64_t beg = 0, end = 0;
    if (pi < pw.end && cur.active) {
        beg = row_ptr[cur.row];
        end = row_ptr[cur.row + 1];
    }
    // settle the prologue's reads here, so the loop's first use of them does not
    // also wait for the prefetches issued ahead of it
    __builtin_amdgcn_s_waitcnt(0x0F70);    // vmcnt(0)
    for (; pi < pw.end; pi += stride) {
        // prefetch: plan word two entries ahead, row bounds of the next entry
        const long long e_nn = pi + 2 * stride < pw.end ? plan[pi + 2 * stride] : 0;
        const EntryLane nxt = entry_lane(e_nxt, lane, C, SPRW);
        int64_t beg_n = 0, end_n = 0;
        if (pi + stride < pw.end && nxt.active) {
            beg_n = row_ptr[nxt.row];
            end_n = row_ptr[nxt.row + 1];
        }
        const int64_t row = cur.row;
        const bool hub = (end - beg) > hub_d;
        const bool writer = cur.active && !hub && cur.slot == 0;
        const int off = cur.chunk * VEC;
        // the row's own values and 1/s do not depend on the gathers: load them first
        A own[VEC];
        A is = (A)0;
        if (writer) {
            load_vec<VEC>(xin + row * R + off, own);
            is = inv_s[row];
        }
        A acc[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] = (A)0;
        if (cur.active && !hub) gather_rows<U, VEC>(col, w, xin, beg + cur.slot, end, cur.SPR, R, off, acc);
        for (int d = cur.SPR >> 1; d >= 1; d >>= 1) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] += shfl_down(acc[q], d * C);
        }
        if (writer) {
            A res[VEC];
            if (end > beg) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) res[q] = fma(omega, neighbour_avg(acc[q], is), keep * own[q]);
                apply_drift(dr, row, R, off, res);
            } else {
#pragma unroll
                for (int q = 0; q < VEC; ++q) res[q] = own[q];
            }
            store_vec<VEC>(xout + row * R + off, res);
        }
        cur = nxt;
        beg = beg_n;
        end = end_n;
        e_nxt = e_nn;
    }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2 * QUEUE_GROUPS)
        __hip_atomic_store(queue_clear + threadIdx.x * QUEUE_PAD, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    // long rows, a workgroup each.  Wave 0 keeps the block's place in the hub
    // queue; thread 0 draws the next row's ticket while this row runs.
    {
        const int slot_w = lane / C;
        const int chunk = lane - slot_w * C;
        const bool lane_on = slot_w < SPRW;
        const int slots = SPRW * (BLOCK / WAVE);
        const int slot = wave * SPRW + slot_w;
        const int off = chunk * VEC;
        const unsigned int nh = *hub_count;
        int hgrp = (int)(blockIdx.x % QUEUE_GROUPS);
        auto hub_at = [nh](int g, unsigned int k, unsigned int &h, unsigned int &) { return hub_item(g, k, nh, h); };
        if (wave == 0) {
            unsigned int h0 = 0, unused = 0;
            const bool ok = take_item(queue, QUEUE_GROUPS, hgrp, NO_CHUNK, lane, hub_at, h0, unused);
            if (lane == 0) s_row = ok ? h0 : NO_CHUNK;
        }
        __syncthreads();
        unsigned int h = s_row;
        while (h != NO_CHUNK) {
            unsigned int ticket = 0;
            if (threadIdx.x == 0) ticket = atomicInc(queue + hgrp * QUEUE_PAD, 0xffffffffu);
            const int64_t row = hub_list[h];
            const int64_t beg = row_ptr[row], end = row_ptr[row + 1];
            A acc[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = (A)0;
            if (lane_on) gather_rows<U, VEC>(col, w, xin, beg + slot, end, slots, R, off, acc);
            for (int d = SPRW >> 1; d >= 1; d >>= 1) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) acc[q] += shfl_down(acc[q], d * C);
            }
            if (lane_on && slot_w == 0) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) part[wave][off + q] = acc[q];
            }
            __syncthreads();
            if (wave == 0 && lane_on && slot_w == 0) {
                A sum[VEC], own[VEC], res[VEC];
#pragma unroll
                for (int q = 0; q < VEC; ++q) sum[q] = part[0][off + q];
                for (int wv = 1; wv < BLOCK / WAVE; ++wv) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) sum[q] += part[wv][off + q];
                }
                load_vec<VEC>(xin + row * R + off, own);
                const A is = inv_s[row];
#pragma unroll
                for (int q = 0; q < VEC; ++q) res[q] = fma(omega, neighbour_avg(sum[q], is), keep * own[q]);
                apply_drift(dr, row, R, off, res);
                store_vec<VEC>(xout + row * R + off, res);
            }
            if (wave == 0) {
                unsigned int hn = 0, unused = 0;
                const unsigned int k = (unsigned int)__builtin_amdgcn_readfirstlane((int)ticket);
                const bool ok = take_item(queue, QUEUE_GROUPS, hgrp, k, lane, hub_at, hn, unused);
                if (lane == 0) s_row = ok ? hn : NO_CHUNK;
            }
            __syncthreads();
            h = s_row;
        }
    }

    // other rows: chunks of plan entries (first row, rows in the tile, log2 rows
    // per wave), each wave starting in a group of its own.  The chunk after next
    // is drawn while a chunk runs, its plan words are read one chunk ahead, and
    // the row bounds of the next entry are read while an entry's rows are
    // gathered.
    const unsigned int np = *plan_count;
    unsigned int *qg = queue + QUEUE_GROUPS * QUEUE_PAD;
    const bool contig = xcd_groups > 1;
    const int ngroups = contig ? (int)XCDS : QUEUE_GROUPS;
    int grp = (int)((blockIdx.x * (BLOCK / WAVE) + wave) % (unsigned int)ngroups);
    if (contig) grp = (int)(blockIdx.x % XCDS);
    auto plan_at = [contig, splits, np](int g, unsigned int k, unsigned int &lo, unsigned int &hi) {
        return chunk_range(contig, splits, np, g, k, lo, hi);
    };
    unsigned int lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
    bool more = take_item(qg, ngroups, grp, NO_CHUNK, lane, plan_at, lo0, hi0);
    if (more) more = take_item(qg, ngroups, grp, NO_CHUNK, lane, plan_at, lo1, hi1);
    if (!more) lo1 = hi1 = 0;
    lo0 = (unsigned int)__builtin_amdgcn_readfirstlane((int)lo0);
    hi0 = (unsigned int)__builtin_amdgcn_readfirstlane((int)hi0);
    lo1 = (unsigned int)__builtin_amdgcn_readfirstlane((int)lo1);
    hi1 = (unsigned int)__builtin_amdgcn_readfirstlane((int)hi1);
    long long w0 = lane < (int)(hi0 - lo0) ? plan[lo0 + lane] : 0;
    long long w1 = lane < (int)(hi1 - lo1) ? plan[lo1 + lane] : 0;
    EntryLane cur = entry_lane(hi0 > lo0 ? lane_word(w0, 0) : 0, lane, C, SPRW);
    int64_t beg = 0, end = 0;
    if (cur.active) {
        beg = row_ptr[cur.row];
        end = row_ptr[cur.row + 1];
    }
    // settle the prologue's reads here: the loop's first uses of them then wait
    // for nothing that is issued inside the loop
    __builtin_amdgcn_s_waitcnt(0x0F70);    // vmcnt(0)
    while (hi0 > lo0) {
        // lane 0 draws the ticket of the chunk after next; the wave reads it after this chunk
        const bool drawing = more;
        unsigned int pend_raw = 0;
        if (drawing && lane == 0) pend_raw = atomicInc(qg + grp * QUEUE_PAD, 0xffffffffu);
        const int len0 = (int)(hi0 - lo0);
        for (int i = 0; i < len0; ++i) {
            const long long e_n = i + 1 < len0 ? lane_word(w0, i + 1) : (hi1 > lo1 ? lane_word(w1, 0) : 0);
            const EntryLane nxt = entry_lane(e_n, lane, C, SPRW);
            int64_t beg_n = 0, end_n = 0;
            if (nxt.active) {
                beg_n = row_ptr[nxt.row];
                end_n = row_ptr[nxt.row + 1];
            }
            const int64_t row = cur.row;
            const bool hub = (end - beg) > hub_d;
            const bool writer = cur.active && !hub && cur.slot == 0;
            const int off = cur.chunk * VEC;
            // the row's own values and 1/s do not depend on the gathers: load them first
            A own[VEC];
            A is = (A)0;
            if (writer) {
                load_vec<VEC>(xin + row * R + off, own);
                is = inv_s[row];
            }
            A acc[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = (A)0;
            if (cur.active && !hub) gather_rows<U, VEC>(col, w, xin, beg + cur.slot, end, cur.SPR, R, off, acc);
            for (int d = cur.SPR >> 1; d >= 1; d >>= 1) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) acc[q] += shfl_down(acc[q], d * C);
            }
            // every read of this entry (and the next entry's bounds) has landed by
            // now; saying so keeps the next entry from waiting on this row's store
            __builtin_amdgcn_s_waitcnt(0x0F70);    // vmcnt(0)
            if (writer) {
                A res[VEC];
                if (end > beg) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) res[q] = fma(omega, neighbour_avg(acc[q], is), keep * own[q]);
                    apply_drift(dr, row, R, off, res);
                } else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) res[q] = own[q];
                }
                store_vec<VEC>(xout + row * R + off, res);
            }
            cur = nxt;
            beg = beg_n;
            end = end_n;
        }
        lo0 = lo1;
        hi0 = hi1;
        w0 = w1;
        lo1 = hi1 = 0;
        if (drawing) {
            const unsigned int pend = (unsigned int)__builtin_amdgcn_readfirstlane((int)pend_raw);
            more = take_item(qg, ngroups, grp, pend, lane, plan_at, lo1, hi1);
            if (!more) lo1 = hi1 = 0;
            lo1 = (unsigned int)__builtin_amdgcn_readfirstlane((int)lo1);
            hi1 = (unsigned int)__builtin_amdgcn_readfirstlane((int)hi1);
        }
        w1 = lane < (int)(hi1 - lo1) ? plan[lo1 + lane] : 0;
    }
}

// Launch plan of the sweep: rows are taken in tiles of PLAN_TILE; a tile's
// rows per wave follow its longest non-hub row (or, with upper_only, its
// longest upper suffix), so that one round of
// SWEEP_UNROLL gathers per slot covers it (short rows share a wave, long
// rows get more slots).  A fixed rows-per-wave request overrides this.
__global__ __launch_bounds__(BLOCK) void k_plan_tiles(int64_t n, const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, int upper_only,
                                                      int64_t hub_d, int spr_max, int rpw_fixed,
                                                      int *__restrict__ tile_lg,
                                                      unsigned int *__restrict__ tile_waves,
                                                      unsigned long long *__restrict__ tile_nnz, Segs sg,
                                                      int64_t ntiles) {
    // one wave per tile (PLAN_TILE == WAVE rows), one lane per row
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    for (int64_t t = (int64_t)blockIdx.x * (BLOCK / WAVE) + (threadIdx.x >> 6); t < ntiles; t += nw) {
        int g;
        int64_t r0, r1;
        seg_span(sg, sg.tile_off, n, t, PLAN_TILE, g, r0, r1);
        int64_t d = 0;
        const int64_t i = r0 + lane;
        if (i < r1) {
            const int64_t beg = row_ptr[i], end = row_ptr[i + 1];
            if (end - beg <= hub_d) d = upper_only ? end - upper_start(col, beg, end, i) : end - beg;
        }
        int64_t dm = d, ds = d;
        for (int o = WAVE / 2; o >= 1; o >>= 1) {
            dm = max(dm, (int64_t)__shfl_xor(dm, o, WAVE));
            ds += (int64_t)__shfl_xor(ds, o, WAVE);
        }
        int lg;
        if (rpw_fixed > 0) {
            lg = 31 - __clz(rpw_fixed);
        } else {
            int spr = 1;
            while (spr < spr_max && (int64_t)spr * SWEEP_UNROLL < dm) spr <<= 1;
            const int rpw = spr_max / spr;
            lg = 31 - __clz(rpw);
        }
        if (lane == 0) {
            tile_lg[t] = lg;
            tile_waves[t] = (unsigned int)ceil_div_dev(r1 - r0, (int64_t)1 << lg);
            tile_nnz[t] = (unsigned long long)ds;
        }
    }
}

__global__ void k_plan_fill(int64_t n, const int *__restrict__ tile_lg, const unsigned int *__restrict__ tile_off,
                            long long *__restrict__ plan, Segs sg, int64_t ntiles) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        int g;
        int64_t r0, r1;
        seg_span(sg, sg.tile_off, n, t, PLAN_TILE, g, r0, r1);
        const int lg = tile_lg[t];
        unsigned int o = tile_off[t];
        for (int64_t r = r0; r < r1; r += (int64_t)1 << lg) {
            const int64_t nr = min((int64_t)1 << lg, r1 - r);
            plan[o++] = ((long long)r << 16) | ((long long)nr << 8) | lg;
        }
    }
}

// Per-vector min and max of x^(k) = x + shift over non-isolated rows
// (ordered-integer atomics); MM_SPLIT blocks per chunk of CENTRE_ROWS rows of
// one graph, each taking 1 / MM_SPLIT of the chunk's rows.  Block b updates copy
// b % MM_SLOTS of the codes: atomics on one address from many blocks
// serialise at the memory side.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_minmax(int64_t n, int R, const int64_t *__restrict__ row_ptr,
                                                 const T *__restrict__ x, const double *__restrict__ shift,
                                                 const int32_t *__restrict__ comp_of,
                                                 unsigned long long *__restrict__ mm, Segs sg) {
    __shared__ double lo_l[BLOCK];
    __shared__ double hi_l[BLOCK];
    const int t = threadIdx.x;
    const int stride = BLOCK / R;
    const int r = t % R;
    const int row_off = t / R;
    int g;
    int64_t r0, r1;
    seg_span(sg, sg.chunk_off, n, blockIdx.x / MM_SPLIT, CENTRE_ROWS, g, r0, r1);
    {
        const int64_t q = (r1 - r0 + MM_SPLIT - 1) / MM_SPLIT;
        r0 += (int64_t)(blockIdx.x % MM_SPLIT) * q;
        r1 = min(r1, r0 + q);
    }
    double lo = INFINITY, hi = -INFINITY;
    if (row_off < stride) {
        // four rows per step, their loads issued together (min and max do not
        // depend on the order)
        constexpr int RU = 4;
        for (int64_t i0 = r0 + row_off; i0 < r1; i0 += (int64_t)RU * stride) {
            double v[RU];
            bool live[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t i = i0 + (int64_t)u * stride;
                live[u] = i < r1 && row_ptr[i + 1] != row_ptr[i];
                v[u] = 0.0;
                if (live[u]) {
                    bool zero;
                    const double *sh = row_shift(shift, comp_of, i, g, R, zero);
                    v[u] = (double)x[i * R + r] + (zero ? 0.0 : sh[r]);
                }
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!live[u]) continue;
                lo = fmin(lo, v[u]);
                hi = fmax(hi, v[u]);
            }
        }
    }
    lo_l[t] = lo;
    hi_l[t] = hi;
    __syncthreads();
    if (t < R) {
        double a = INFINITY, b = -INFINITY;
        for (int q = t; q < stride * R; q += R) {
            a = fmin(a, lo_l[q]);
            b = fmax(b, hi_l[q]);
        }
        if (a <= b) {
            unsigned long long *m_ = mm + ((int64_t)(blockIdx.x % MM_SLOTS) * sg.G + g) * 2 * R;
            atomicMin(&m_[t], ord_encode(a));
            atomicMax(&m_[R + t], ord_encode(b));
        }
    }
}

__global__ void k_minmax_out(int G, int R, const unsigned long long *__restrict__ mm, double *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)G * R) return;
    const int64_t g = idx / R;
    const int r = (int)(idx - g * R);
    unsigned long long a = ~0ull, b = 0ull;
    for (int sl = 0; sl < MM_SLOTS; ++sl) {
        const unsigned long long *m_ = mm + ((int64_t)sl * G + g) * 2 * R;
        a = min(a, m_[r]);
        b = max(b, m_[R + r]);
    }
    bool none = (a == ~0ull);
    out[g * 2 * R + r] = none ? INFINITY : ord_decode(a);
    out[g * 2 * R + R + r] = none ? -INFINITY : ord_decode(b);
}

// ------------------------------------------------------------------- host --

struct Buf {
    void *p;
    ad_dtype t;
    bool f32 = false;     // FP64 storage holding the results of FP32 arithmetic
};

static int pick_vec(int R, size_t elem_bytes) {
    int maxv = (int)(16 / elem_bytes);
    for (int v = maxv; v > 1; v >>= 1)
        if (R % v == 0) return v;
    return 1;
}

SweepShape sweep_shape(int R, size_t in_bytes, int rpw_req, int64_t hub_req) {
    SweepShape s;
    s.vec = pick_vec(R, in_bytes);
    s.C = lanes_per_row(R, s.vec);
    s.SPRW = pow2_slots(WAVE, s.C);
    int rpw = std::min(std::max(rpw_req, 0), s.SPRW);
    int p = 1;
    while (p * 2 <= rpw) p *= 2;        // a power of two dividing SPRW
    s.rpw_fixed = rpw > 0 ? p : 0;
    s.hub_d = hub_req > 0 ? hub_req : std::max<int64_t>(256, 2 * (int64_t)s.SPRW * SWEEP_UNROLL);
    return s;
}

size_t sweep_plan_bytes(int64_t n, int64_t ntiles_cap) {
    Carver c(nullptr, 0);
    SweepPlan p;
    sweep_plan_carve(c, n, ntiles_cap, p);
    return c.used;
}

void sweep_plan_carve(Carver &c, int64_t n, int64_t ntiles_cap, SweepPlan &p) {
    const int64_t nn = std::max<int64_t>(1, n);
    const int64_t ntiles = std::max<int64_t>(1, ntiles_cap);
    p.hub_list = c.take<int32_t>(nn);
    p.hub_count = c.take<unsigned int>(1);
    p.plan = c.take<long long>(nn + ntiles);
    p.plan_count = c.take<unsigned int>(1);
    p.tile_lg = c.take<int>(ntiles);
    p.tile_waves = c.take<unsigned int>(ntiles);
    p.tile_nnz = c.take<unsigned long long>(ntiles);
    p.splits = c.take<unsigned int>(XCDS + 1);
    p.queue = c.take<unsigned int>((size_t)QUEUE_SLOTS * QUEUE_SET);
    const size_t nblk = scan_scratch_blocks(ntiles);
    p.scan.blk_v = c.take<unsigned int>(nblk);
    p.scan.blk_w = c.take<unsigned long long>(nblk);
    p.scan.total_w = c.take<unsigned long long>(1);
}

ad_status sweep_plan_build(const ad_graph *g, SweepPlan &p, bool build_hubs, const Segs &sg, hipStream_t st) {
    ad_status s;
    p.xcd_groups = (sg.tile_off && sg.G > 1) ? (int)XCDS : 1;
    // every queue set starts at zero; each launch then clears the set the launch after next uses
    p.turn = 0;
    s = fill_i32((int32_t *)p.queue, 0, (int64_t)QUEUE_SLOTS * QUEUE_SET, st);
    if (s != AD_OK) return s;
    if (build_hubs) {
        s = fill_i32((int32_t *)p.hub_count, 0, 1, st);
        if (s != AD_OK) return s;
        s = collect_rows(g, p.sh.hub_d, (int64_t)1 << 62, p.hub_list, p.hub_count, st);
        if (s != AD_OK) return s;
    }
    const int64_t ntiles = sg.tile_off ? sg.ntiles : ceil_div(g->n, PLAN_TILE);
    if (ntiles <= 0) {
        ad_status s0 = fill_i32((int32_t *)p.splits, 0, XCDS + 1, st);
        if (s0 != AD_OK) return s0;
        return fill_i32((int32_t *)p.plan_count, 0, 1, st);
    }
    static_assert(PLAN_TILE == WAVE, "k_plan_tiles gives each tile one wave");
    hipLaunchKernelGGL(k_plan_tiles, dim3(grid_for(ntiles, BLOCK / WAVE)), dim3(BLOCK), 0, st, g->n, g->row_ptr, g->col,
                       p.sh.upper_only, p.sh.hub_d, p.sh.SPRW, p.sh.rpw_fixed, p.tile_lg, p.tile_waves, p.tile_nnz,
                       sg, ntiles);
    AD_LAUNCH_CHECK("k_plan_tiles");
    // tile offsets into the plan; for XCD groups also their edge-balanced ranges
    s = scan_exclusive(ntiles, p.tile_waves, p.xcd_groups > 1 ? p.tile_nnz : nullptr, p.plan_count, p.splits, p.scan,
                       st);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_plan_fill, dim3(grid_for(ntiles, BLOCK)), dim3(BLOCK), 0, st, g->n, p.tile_lg,
                       p.tile_waves, p.plan, sg, ntiles);
    AD_LAUNCH_CHECK("k_plan_fill");
    return AD_OK;
}

constexpr int64_t MAX_MAIN_BLOCKS = 4096;   // static walk: persistent, waves loop over plan entries

// Gathers in flight per lane: SWEEP_UNROLL, or half of it for FP64
// arithmetic, whose accumulators and wider rows would not fit the register
// budget of four waves per SIMD with eight.
template <typename A, int VEC>
constexpr int sweep_unroll() {
    return (sizeof(A) == 8 && VEC >= 2) ? SWEEP_UNROLL / 2 : SWEEP_UNROLL;
}

template <typename Tin, typename Tout, typename A, int VEC>
static ad_status launch_sweep_v(const ad_graph *g, const A *inv_s, A omega, const Tin *xin, Tout *xout,
                                int R, const SweepPlan &pl, hipStream_t st, SweepDrift dr) {
    const SweepShape &sh = pl.sh;
    if (pl.xcd_groups <= 1) {
        const int64_t main_blocks = std::min<int64_t>(MAX_MAIN_BLOCKS, ceil_div(g->n, BLOCK / WAVE));
        // at most 2m / hub_d rows exceed hub_d; unknown d_max (0) keeps the bound
        int64_t hub_blocks = 0;
        if (g->d_max == 0 || g->d_max > sh.hub_d)
            hub_blocks =
                round_up_xcds(std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(2 * g->m, sh.hub_d + 1))));
        const int64_t grid = main_blocks + hub_blocks;
        if (grid <= 0) return AD_OK;
        TraceScope trace("k_sweep", st);
        hipLaunchKernelGGL((k_sweep<Tin, Tout, A, VEC, sweep_unroll<A, VEC>(), false>), dim3((unsigned)grid), dim3(BLOCK), 0,
                           st, g->n, g->row_ptr, g->col, g->w, inv_s, omega, xin, xout, R, sh.C, sh.hub_d, sh.SPRW,
                           (int)hub_blocks, pl.hub_list, pl.hub_count, pl.plan, pl.plan_count, pl.splits,
                           pl.xcd_groups, (unsigned int *)nullptr, (unsigned int *)nullptr, dr);
        AD_LAUNCH_CHECK("k_sweep");
        return AD_OK;
    }
    auto kern = k_sweep<Tin, Tout, A, VEC, sweep_unroll<A, VEC>(), true>;
    // workgroups the device holds at once (per device, found once): the queues
    // hand out all work, so a larger grid would only add idle workgroups
    static std::atomic<int> resident[MAX_DEVICES];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) dev = 0;
    int cap = resident[dev].load(std::memory_order_relaxed);
    if (cap <= 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BLOCK, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 1;
        (void)hipGetLastError();
        cap = per_cu * cus;
        resident[dev].store(cap, std::memory_order_relaxed);
    }
    const int64_t grid = std::min<int64_t>(cap, std::max<int64_t>(XCDS, ceil_div(g->n, BLOCK / WAVE)));
    unsigned int *use = pl.queue + (size_t)(pl.turn % QUEUE_SLOTS) * QUEUE_SET;
    unsigned int *clear = pl.queue + (size_t)((pl.turn + QUEUE_SLOTS - 1) % QUEUE_SLOTS) * QUEUE_SET;
    ++pl.turn;
    TraceScope trace("k_sweep", st);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(BLOCK), 0, st, g->n, g->row_ptr, g->col, g->w, inv_s, omega,
                       xin, xout, R, sh.C, sh.hub_d, sh.SPRW, 0, pl.hub_list, pl.hub_count, pl.plan, pl.plan_count,
                       pl.splits, pl.xcd_groups, use, clear, dr);
    AD_LAUNCH_CHECK("k_sweep");
    return AD_OK;
}

// Vector widths a plan can ask for: at most 16 bytes of the plan's element
// type per lane, which is the input type except for FP64 sweeps run on the
// FP32 plan (the FP64 tail of FP32 storage: 4 doubles per lane).
template <typename Tin, typename Tout, typename A, int VEC>
static ad_status launch_sweep_w(const ad_graph *g, const A *inv_s, A omega, const Tin *xin, Tout *xout, int R,
                                const SweepPlan &pl, hipStream_t st, SweepDrift dr) {
    if constexpr (VEC * (sizeof(Tin) < 4 ? sizeof(Tin) : 4) <= 16)
        return launch_sweep_v<Tin, Tout, A, VEC>(g, inv_s, omega, xin, xout, R, pl, st, dr);
    return fail(AD_ERR_INTERNAL, "vector width beyond the plan's");
}

template <typename Tin, typename Tout, typename A>
static ad_status launch_sweep(const ad_graph *g, const A *inv_s, A omega, const Tin *xin, Tout *xout, int R,
                              const SweepPlan &pl, hipStream_t st, SweepDrift dr = SweepDrift()) {
    switch (pl.sh.vec) {
    case 1: return launch_sweep_w<Tin, Tout, A, 1>(g, inv_s, omega, xin, xout, R, pl, st, dr);
    case 2: return launch_sweep_w<Tin, Tout, A, 2>(g, inv_s, omega, xin, xout, R, pl, st, dr);
    case 4: return launch_sweep_w<Tin, Tout, A, 4>(g, inv_s, omega, xin, xout, R, pl, st, dr);
    case 8: return launch_sweep_w<Tin, Tout, A, 8>(g, inv_s, omega, xin, xout, R, pl, st, dr);
    }
    return fail(AD_ERR_INTERNAL, "bad vector width");
}

static size_t dtype_bytes(ad_dtype t) { return t == AD_F64 ? 8 : (t == AD_F32 ? 4 : 2); }

struct RelaxLayout {
    void *inv_s;
    float *sdeg;
    double *s64;              // s_i for the FP64 tail of FP32 / BF16 storage
    double *part, *part_s, *shift;
    float *drift;             // BF16 re-centring, [n_comp][R]
    unsigned long long *mm;
    SweepPlan p32, p16;
    void *bufA, *bufB;
    void *b16A, *b16B;
    void *b64A, *b64B;
};

static int64_t seg_chunks(const ad_graph *g, const Segs &sg) {
    return sg.chunk_off ? sg.nchunks : ceil_div(g->n, CENTRE_ROWS);
}
static int64_t seg_tiles(const ad_graph *g, const Segs &sg) {
    return sg.tile_off ? sg.ntiles : ceil_div(g->n, PLAN_TILE);
}

// Sweeps stored in FP64 at the end (the whole run for AD_F64).
static int fp64_sweeps(const ad_relax_opts *o) {
    if (o->store == AD_F64) return o->k;
    return std::min(std::max(o->fp64_tail, 0), std::max(o->k, 0));
}
static bool x_out_f64(const ad_relax_opts *o) { return o->store == AD_F64 || o->fp64_tail > 0; }

static size_t relax_layout(const ad_graph *g, const ad_relax_opts *o, void *ws, size_t ws_bytes,
                           RelaxLayout *L, const Segs &sg) {
    Carver c(ws, ws_bytes);
    const int64_t n = g->n > 0 ? g->n : 1;
    const int R = o->R;
    const bool comp = o->comp != nullptr;
    const int64_t nb = std::max<int64_t>(1, comp ? o->comp->n_chunks : seg_chunks(g, sg));
    const int64_t nshift = comp ? std::max<int64_t>(1, o->comp->n_comp) : (int64_t)sg.G;
    const int64_t nt = seg_tiles(g, sg);
    const bool f64 = o->store == AD_F64;
    const bool tail64 = !f64 && o->fp64_tail > 0 && o->k > 0;
    RelaxLayout l;
    l.inv_s = f64 ? (void *)c.take<double>(n) : (void *)c.take<float>(n);
    l.sdeg = c.take<float>(n);
    l.s64 = tail64 ? c.take<double>(n) : nullptr;
    l.part = c.take<double>(nb * R);
    l.part_s = c.take<double>(nb);
    l.shift = c.take<double>((size_t)nshift * R);
    l.drift = (comp && o->store == AD_BF16) ? c.take<float>((size_t)nshift * R) : nullptr;
    l.mm = c.take<unsigned long long>((size_t)MM_SLOTS * sg.G * 2 * R);
    sweep_plan_carve(c, n, nt, l.p32);
    if (o->store == AD_BF16) sweep_plan_carve(c, n, nt, l.p16);
    const size_t xb = f64 ? 8 : 4;
    l.bufA = c.take<char>((size_t)n * R * xb);
    l.bufB = c.take<char>((size_t)n * R * xb);
    if (o->store == AD_BF16) {
        l.b16A = c.take<uint16_t>((size_t)n * R);
        l.b16B = c.take<uint16_t>((size_t)n * R);
    } else {
        l.b16A = l.b16B = nullptr;
    }
    if (tail64) {
        l.b64A = c.take<double>((size_t)n * R);
        l.b64B = o->fp64_tail >= 2 ? c.take<double>((size_t)n * R) : nullptr;
    } else {
        l.b64A = l.b64B = nullptr;
    }
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

static ad_status check_relax_opts(const ad_relax_opts *o) {
    if (!o) return fail(AD_ERR_INVALID_ARG, "opts is NULL");
    if (o->R < 1 || o->R > 64) return fail(AD_ERR_INVALID_ARG, "R must be in [1, 64]");
    if (o->k < 0) return fail(AD_ERR_INVALID_ARG, "k must be >= 0");
    if (!(o->omega > 0.0 && o->omega <= 1.0)) return fail(AD_ERR_INVALID_ARG, "omega must be in (0, 1]");
    if (o->store != AD_F64 && o->store != AD_F32 && o->store != AD_BF16)
        return fail(AD_ERR_INVALID_ARG, "unknown storage type");
    if (o->store == AD_BF16 && o->fp32_tail < 1) return fail(AD_ERR_INVALID_ARG, "fp32_tail must be >= 1");
    if (o->fp64_tail < 0) return fail(AD_ERR_INVALID_ARG, "fp64_tail must be >= 0");
    if (o->store == AD_BF16 && o->fp64_tail > 0 && o->fp64_tail >= o->fp32_tail)
        return fail(AD_ERR_INVALID_ARG, "with BF16 storage fp64_tail must be below fp32_tail");
    if (o->ckpt_every < 0) return fail(AD_ERR_INVALID_ARG, "ckpt_every must be >= 0");
    if (o->ckpt_every > 0 && o->store == AD_BF16)
        return fail(AD_ERR_UNSUPPORTED, "checkpoints need FP32 or FP64 storage");
    if (o->ckpt_every > 0 && o->store != AD_F64 && o->fp64_tail > 0)
        return fail(AD_ERR_UNSUPPORTED, "checkpoints need fp64_tail == 0");
    if (o->rows_per_wave < 0 || o->hub_degree < 0) return fail(AD_ERR_INVALID_ARG, "negative tuning value");
    if (o->comp) {
        const ad_components *c = o->comp;
        if (c->n_comp < 0 || c->n_chunks < c->n_comp) return fail(AD_ERR_INVALID_ARG, "bad component counts");
        if (c->n_comp > 0 && (!c->comp_of || !c->members || !c->comp_start || !c->chunk_start))
            return fail(AD_ERR_INVALID_ARG, "component arrays are NULL");
    }
    return AD_OK;
}

// s_i and the sweep scale (1/s_i for FP32, s_i for FP64 arithmetic): rows up
// to the plan's hub degree by lane groups, longer rows (the plan's hub list)
// by a workgroup each; s64 (optional) receives s_i in FP64.
template <typename A>
static ad_status weighted_degree_impl(const ad_graph *g, A *inv_s, float *sdeg, double *s64, const SweepPlan &pl,
                                      hipStream_t st) {
    const int64_t n = g->n;
    if (n <= 0) return AD_OK;
    const int lpr = degree_lanes((double)(2 * g->m) / (double)n);
    hipLaunchKernelGGL((k_weighted_degree<A>), dim3((unsigned)ceil_div(n * lpr, BLOCK)), dim3(BLOCK), 0, st, n,
                       g->row_ptr, g->w, inv_s, sdeg, s64, lpr, pl.sh.hub_d);
    AD_LAUNCH_CHECK("k_weighted_degree");
    if (g->d_max == 0 || g->d_max > pl.sh.hub_d) {
        const unsigned grid = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(2 * g->m, pl.sh.hub_d + 1)));
        hipLaunchKernelGGL((k_weighted_degree_hub<A>), dim3(grid), dim3(BLOCK), 0, st, pl.hub_list, pl.hub_count,
                           g->row_ptr, g->w, inv_s, sdeg, s64);
        AD_LAUNCH_CHECK("k_weighted_degree_hub");
    }
    return AD_OK;
}

// One sweep from cur to dst in the types they are stored in.
static ad_status sweep_step(const ad_graph *g, const RelaxLayout &L, const RelaxLayout &P, double omega,
                            const Buf &cur, const Buf &dst, int R, hipStream_t st, SweepDrift dr) {
    if (dst.t == AD_F64 && dst.f32) {
        // the last sweep before the FP64 tail: FP32 arithmetic as the sweeps
        // before it, its results stored widened, so that the tail reads FP64 rows
        const float om = (float)omega;
        const float *is = (const float *)L.inv_s;
        if (cur.t == AD_F32)
            return launch_sweep<float, double, float>(g, is, om, (const float *)cur.p, (double *)dst.p, R, P.p32, st);
        if (cur.t == AD_BF16)
            return launch_sweep<bf16, double, float>(g, is, om, (const bf16 *)cur.p, (double *)dst.p, R, P.p16, st);
        return fail(AD_ERR_INTERNAL, "widened sweep from FP64");
    }
    if (dst.t == AD_F64) {
        // FP64 arithmetic, dividing by s_i: the FP64 storage form reads its
        // divisor from inv_s, the FP64 tail of FP32 storage from s64 and runs
        // on the FP32 plan
        if (cur.t == AD_F64) {
            if (L.s64)
                return launch_sweep<double, double, double>(g, L.s64, omega, (const double *)cur.p,
                                                            (double *)dst.p, R, P.p32, st);
            return launch_sweep<double, double, double>(g, (const double *)L.inv_s, omega, (const double *)cur.p,
                                                        (double *)dst.p, R, P.p32, st);
        }
        if (cur.t == AD_F32)
            return launch_sweep<float, double, double>(g, L.s64, omega, (const float *)cur.p, (double *)dst.p, R,
                                                       P.p32, st);
        return fail(AD_ERR_INTERNAL, "BF16 to FP64 sweep");
    }
    const float om = (float)omega;
    const float *is = (const float *)L.inv_s;
    if (cur.t == AD_F32 && dst.t == AD_F32)
        return launch_sweep<float, float, float>(g, is, om, (const float *)cur.p, (float *)dst.p, R, P.p32, st);
    if (cur.t == AD_F32 && dst.t == AD_BF16)
        return launch_sweep<float, bf16, float>(g, is, om, (const float *)cur.p, (bf16 *)dst.p, R, P.p32, st, dr);
    if (cur.t == AD_BF16 && dst.t == AD_BF16)
        return launch_sweep<bf16, bf16, float>(g, is, om, (const bf16 *)cur.p, (bf16 *)dst.p, R, P.p16, st, dr);
    if (cur.t == AD_BF16 && dst.t == AD_F32)
        return launch_sweep<bf16, float, float>(g, is, om, (const bf16 *)cur.p, (float *)dst.p, R, P.p16, st);
    return fail(AD_ERR_INTERNAL, "unsupported sweep types");
}

// Enqueue the whole relaxation.  `shift_out` may be NULL.
template <typename T>
static ad_status relax_impl(const ad_graph *g, const ad_relax_opts *o, const void *x0, void *x_out,
                            double *minmax_out, double *shift_out, void *ckpt, const RelaxLayout &L,
                            const Segs &sg, hipStream_t st) {
    typedef typename acc_of<T>::type A;
    const int R = o->R;
    const int64_t n = g->n;
    const ad_components *comp = o->comp;
    const int64_t nb = seg_chunks(g, sg);
    ad_status s;

    // launch plans first: the hub list also serves the weighted degrees
    RelaxLayout P = L;
    P.p32.sh = sweep_shape(R, sizeof(T), o->rows_per_wave, o->hub_degree);
    if (n > 0) {
        s = sweep_plan_build(g, P.p32, true, sg, st);
        if (s != AD_OK) return s;
        if (o->store == AD_BF16 && o->k > 0) {
            P.p16.sh = sweep_shape(R, 2, o->rows_per_wave, o->hub_degree);
            P.p16.sh.hub_d = P.p32.sh.hub_d;            // one hub list serves both
            P.p16.hub_list = P.p32.hub_list;
            P.p16.hub_count = P.p32.hub_count;
            s = sweep_plan_build(g, P.p16, false, sg, st);
            if (s != AD_OK) return s;
        }
    }

    // the shifts: written straight into shift_out when the caller wants them
    double *shift = shift_out ? shift_out : L.shift;
    if (n > 0) {
        s = weighted_degree_impl<A>(g, (A *)L.inv_s, L.sdeg, L.s64, P.p32, st);
        if (s != AD_OK) return s;
    }
    if (comp) {
        if (n > 0 && comp->n_chunks > 0) {
            hipLaunchKernelGGL((k_comp_partials<T>), dim3((unsigned)ceil_div(comp->n_chunks, BLOCK / WAVE)),
                               dim3(BLOCK), 0, st, R, comp->n_comp, comp->n_chunks, comp->members, comp->comp_start,
                               comp->chunk_start, L.sdeg, g->orig_id, o->seed, o->graph_id, (const T *)x0,
                               sg.row_graph, L.part, L.part_s);
            AD_LAUNCH_CHECK("k_comp_partials");
        }
        const int64_t cr = comp->n_comp * R;
        if (cr > 0) {
            hipLaunchKernelGGL(k_comp_finalize, dim3((unsigned)std::min<int64_t>(ceil_div(cr, BLOCK / WAVE), 1 << 16)), dim3(BLOCK), 0, st, R,
                               comp->n_comp, comp->chunk_start, L.part, L.part_s, 1, shift);
            AD_LAUNCH_CHECK("k_comp_finalize");
        }
        const int64_t mmc = (int64_t)MM_SLOTS * sg.G * 2 * R;
        hipLaunchKernelGGL(k_mm_reset, dim3((unsigned)ceil_div(mmc, BLOCK)), dim3(BLOCK), 0, st, mmc, R, L.mm);
        AD_LAUNCH_CHECK("k_mm_reset");
    } else {
        if (n > 0 && nb > 0) {
            hipLaunchKernelGGL((k_centre_partials<T>), dim3((unsigned)nb), dim3(BLOCK), 0, st, n, R, L.sdeg,
                               g->orig_id, o->seed, o->graph_id, (const T *)x0, L.part, L.part_s, sg);
            AD_LAUNCH_CHECK("k_centre_partials");
        }
        hipLaunchKernelGGL(k_centre_finalize, dim3((unsigned)sg.G), dim3(BLOCK), 0, st, R, n > 0 ? nb : (int64_t)0,
                           L.part, L.part_s, 1, shift, L.mm, sg);
        AD_LAUNCH_CHECK("k_centre_finalize");
    }
    const int32_t *comp_of = comp ? comp->comp_of : nullptr;

    const int nck = ad_relax_num_checkpoints(o);
    const size_t slot_elems = (size_t)n * R;
    const bool out64 = x_out_f64(o);
    const ad_dtype tstore = o->store == AD_F64 ? AD_F64 : AD_F32;
    Buf cur;
    if (o->k == 0) cur = {x_out, out64 ? AD_F64 : AD_F32};
    else cur = {ckpt && nck > 0 ? ckpt : L.bufA, tstore};
    if (n > 0) {
        int64_t total = n * ((R + 3) / 4);
        if (cur.t == AD_F64)
            hipLaunchKernelGGL((k_init<T, double>), dim3(grid_for(total, BLOCK)), dim3(BLOCK), 0, st, n, R,
                               g->orig_id, o->seed, o->graph_id, (const T *)x0, shift, comp_of, (double *)cur.p,
                               sg.row_graph);
        else
            hipLaunchKernelGGL((k_init<T, float>), dim3(grid_for(total, BLOCK)), dim3(BLOCK), 0, st, n, R,
                               g->orig_id, o->seed, o->graph_id, (const T *)x0, shift, comp_of, (float *)cur.p,
                               sg.row_graph);
        AD_LAUNCH_CHECK("k_init");
    }

    if (o->k > 0 && n > 0) {
        // one pair of trace events around the k back-to-back sweeps (an event
        // between two sweeps would cost the stream more than it measures)
        TraceScope trace("k_sweep", st, o->k);
        TraceSuppress per_launch;
        const int tail32 = o->store == AD_BF16 ? o->fp32_tail : o->k;
        const int tail64 = fp64_sweeps(o);
        for (int t = 1; t <= o->k; ++t) {
            const bool wide = t > o->k - tail64;
            Buf dst;
            if (t == o->k) {
                dst = {x_out, out64 ? AD_F64 : AD_F32};
            } else if (wide && o->store != AD_F64) {
                dst = {cur.p == L.b64A ? L.b64B : L.b64A, AD_F64};
            } else if (tail64 > 0 && t == o->k - tail64 && o->store != AD_F64) {
                dst = {L.b64A, AD_F64, true};
            } else if (ckpt && o->ckpt_every > 0 && t % o->ckpt_every == 0) {
                dst = {(char *)ckpt + (size_t)(t / o->ckpt_every) * slot_elems * sizeof(T), tstore};
            } else if (o->store == AD_BF16 && t <= o->k - tail32) {
                dst = {cur.p == L.b16A ? L.b16B : L.b16A, AD_BF16};
            } else {
                dst = {cur.p == L.bufA ? L.bufB : L.bufA, tstore};
            }
            SweepDrift dr;
            if (L.drift && dst.t == AD_BF16 && t >= 2 && comp->n_comp > 0) {
                const dim3 dgrid((unsigned)ceil_div(comp->n_chunks, BLOCK / WAVE));
#define AD_DRIFT_ARGS R, comp->n_comp, comp->n_chunks, comp->members, comp->comp_start, comp->chunk_start, L.sdeg, \
                      (const bf16 *)cur.p, L.part
                if (R % 8 == 0)
                    hipLaunchKernelGGL((k_comp_drift_partials<bf16, 8>), dgrid, dim3(BLOCK), 0, st, AD_DRIFT_ARGS);
                else if (R % 4 == 0)
                    hipLaunchKernelGGL((k_comp_drift_partials<bf16, 4>), dgrid, dim3(BLOCK), 0, st, AD_DRIFT_ARGS);
                else
                    hipLaunchKernelGGL((k_comp_drift_partials<bf16, 1>), dgrid, dim3(BLOCK), 0, st, AD_DRIFT_ARGS);
#undef AD_DRIFT_ARGS
                AD_LAUNCH_CHECK("k_comp_drift_partials");
                const int64_t cr = comp->n_comp * R;
                hipLaunchKernelGGL(k_comp_drift, dim3((unsigned)std::min<int64_t>(ceil_div(cr, BLOCK / WAVE), 1 << 16)), dim3(BLOCK), 0, st, R,
                                   comp->n_comp, comp->chunk_start, L.part, L.part_s, L.drift, shift);
                AD_LAUNCH_CHECK("k_comp_drift");
                dr.c = L.drift;
                dr.comp_of = comp->comp_of;
            }
            s = sweep_step(g, L, P, o->omega, cur, dst, R, st, dr);
            if (s != AD_OK) return s;
            cur = dst;
        }
    }

    if (n > 0 && nb > 0) {
        if (out64)
            hipLaunchKernelGGL((k_minmax<double>), dim3((unsigned)(nb * MM_SPLIT)), dim3(BLOCK), 0, st, n, R, g->row_ptr,
                               (const double *)x_out, shift, comp_of, L.mm, sg);
        else
            hipLaunchKernelGGL((k_minmax<float>), dim3((unsigned)(nb * MM_SPLIT)), dim3(BLOCK), 0, st, n, R, g->row_ptr,
                               (const float *)x_out, shift, comp_of, L.mm, sg);
        AD_LAUNCH_CHECK("k_minmax");
    }
    const int64_t gr = (int64_t)sg.G * R;
    hipLaunchKernelGGL(k_minmax_out, dim3((unsigned)ceil_div(gr, BLOCK)), dim3(BLOCK), 0, st, sg.G, R, L.mm,
                       minmax_out);
    AD_LAUNCH_CHECK("k_minmax_out");
    return AD_OK;
}

size_t relax_segs_workspace(const ad_graph *g, const ad_relax_opts *o, const Segs &sg) {
    return relax_layout(g, o, nullptr, 0, nullptr, sg);
}

ad_status relax_segs(const ad_graph *g, const ad_relax_opts *o, const void *x0, void *x_out, double *minmax_out,
                     double *shift_out, void *ckpt, void *ws, size_t ws_bytes, const Segs &sg, hipStream_t st) {
    RelaxLayout L;
    if (relax_layout(g, o, ws, ws_bytes, &L, sg) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    if (o->store == AD_F64) return relax_impl<double>(g, o, x0, x_out, minmax_out, shift_out, ckpt, L, sg, st);
    return relax_impl<float>(g, o, x0, x_out, minmax_out, shift_out, ckpt, L, sg, st);
}

ad_status sweep_f32(const ad_graph *g, const float *inv_s, float omega, const float *xin, float *xout, int R,
                    const SweepPlan &plan, hipStream_t st) {
    return launch_sweep<float, float, float>(g, inv_s, omega, xin, xout, R, plan, st);
}

ad_status weighted_degree_f32(const ad_graph *g, float *inv_s, float *sdeg, const SweepPlan &pl, hipStream_t st) {
    return weighted_degree_impl<float>(g, inv_s, sdeg, nullptr, pl, st);
}

}  // namespace ad

using namespace ad;

extern "C" int32_t ad_relax_num_checkpoints(const ad_relax_opts *o) {
    if (!o || o->ckpt_every <= 0 || o->k <= 0) return 0;
    return (o->k + o->ckpt_every - 1) / o->ckpt_every;
}

extern "C" size_t ad_relax_workspace_size(const ad_graph *g, const ad_relax_opts *o) {
    if (check_graph_args(g) != AD_OK || check_relax_opts(o) != AD_OK) return 0;
    return relax_layout(g, o, nullptr, 0, nullptr, Segs());
}

extern "C" ad_status ad_relax(const ad_graph *g, const ad_relax_opts *o, const void *x0, void *x_out,
                              double *minmax_out, double *shift_out, void *ckpt, void *ws,
                              size_t ws_bytes, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    s = check_relax_opts(o);
    if (s != AD_OK) return s;
    if (!minmax_out) return fail(AD_ERR_INVALID_ARG, "minmax_out is NULL");
    if (g->n > 0 && !x_out) return fail(AD_ERR_INVALID_ARG, "x_out is NULL");
    if (x0 && x0 == x_out) return fail(AD_ERR_INVALID_ARG, "x_out aliases x0");
    if (ckpt && ckpt == x_out) return fail(AD_ERR_INVALID_ARG, "x_out aliases ckpt");
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    return relax_segs(g, o, x0, x_out, minmax_out, shift_out, ckpt, ws, ws_bytes, Segs(), stream);
}
