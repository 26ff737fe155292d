// ad_select.hip -- edge distances (Algorithm 1, last steps), per-vertex
// ranking and selection (Algorithm 3) and the retention fit (Section 6.2).
//
// Distances: one lane per stored entry (i, j) with j > i walks the R values
// of both rows in order r = 0..R-1, so the sum for an edge has one fixed
// order and rho_ij == rho_ji bit for bit whichever endpoint computes it.
//
// Ranking: every stored entry (i, j) gets its position in row i's order
// (rho ascending for LOCAL, descending for GLOBAL; ties by orig_id[j]).
// Keys are unique inside a row, so ranks are well defined.  Rows of degree
// <= 64 rank by counting inside a wave (each lane compares its key with all
// others of its row through shuffles); rows of degree <= 8192 sort their
// keys with a bitonic network in LDS; longer rows count against keys read
// from memory.
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

#include <algorithm>
#include <vector>

namespace ad {

constexpr int SBLOCK = 256;
constexpr int SORT_CAP = 8192;       // longest row ranked in LDS
constexpr int WAVE_CAP = 512;        // longest row ranked inside one wave

// ---------------------------------------------------------------- distance --

template <typename Tx, typename Tr, int VEC>
__global__ __launch_bounds__(SBLOCK) void k_edge_dist(
    int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const Tx *__restrict__ x, const double *__restrict__ minmax,
    Tr *__restrict__ rho, int R, int LPR) {
    typedef typename acc_of<Tx>::type A;
    __shared__ A inv_l[64];
    if (threadIdx.x < R) {
        double lo = minmax[threadIdx.x], hi = minmax[R + threadIdx.x];
        inv_l[threadIdx.x] = (hi > lo) ? (A)(1.0 / (hi - lo)) : (A)0;
    }
    __syncthreads();
    // LPR lanes per row, SBLOCK / LPR rows per block
    const int rows_per_block = SBLOCK / LPR;
    const int64_t row = (int64_t)blockIdx.x * rows_per_block + threadIdx.x / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= n) return;
    const int64_t beg = row_ptr[row], end = row_ptr[row + 1];
    const Tx *xi = x + row * R;
    for (int64_t p = beg + lane; p < end; p += LPR) {
        const int32_t j = col[p];
        if (j <= row) continue;
        const Tx *xj = x + (int64_t)j * R;
        A acc = (A)0;
        for (int r0 = 0; r0 < R; r0 += VEC) {
            A a[VEC], b[VEC];
            load_vec<VEC>(xi + r0, a);
            load_vec<VEC>(xj + r0, b);
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                A d = (a[q] - b[q]) * inv_l[r0 + q];
                acc = fma(d, d, acc);
            }
        }
        rho[eid[p]] = (Tr)sqrt(acc);
    }
}

// ------------------------------------------------------------------ ranking --

enum { MODE_FIXED = 0, MODE_SIDES = 1 };

// (rho_a, id_a) comes before (rho_b, id_b) in the row's order.
template <typename Tr>
__device__ __forceinline__ bool before(Tr ra, int32_t ia, Tr rb, int32_t ib, int orient) {
    if (ra != rb) return orient == AD_LOCAL ? (ra < rb) : (ra > rb);
    return ia < ib;
}

__device__ __forceinline__ void emit(int mode, int64_t row, int32_t j, int32_t e, int64_t d, int64_t rank,
                                     const int32_t *__restrict__ budget, uint8_t *__restrict__ keep,
                                     unsigned long long *__restrict__ sides) {
    if (mode == MODE_FIXED) {
        if (rank < budget[d]) keep[e] = 1;
    } else {
        sides[2 * (int64_t)e + (row > j ? 1 : 0)] =
            ((unsigned long long)d << 32) | (unsigned long long)rank;
    }
}

// Rows with SW/2 < d <= SW (1 <= d <= SW for the smallest class): SW lanes
// per row, 64/SW rows per wave, ranks by counting through shuffles.
template <typename Tr, int SW>
__global__ __launch_bounds__(SBLOCK) void k_rank_small(
    int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id, const Tr *__restrict__ rho,
    int orient, int mode, int64_t dlo, const int32_t *__restrict__ budget, uint8_t *__restrict__ keep,
    unsigned long long *__restrict__ sides) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int seg = lane / SW;
    const int q = lane - seg * SW;
    const int64_t row = ((int64_t)blockIdx.x * (SBLOCK / WAVE) + (threadIdx.x >> 6)) * (WAVE / SW) + seg;
    int64_t beg = 0, d = 0;
    if (row < n) {
        beg = row_ptr[row];
        d = row_ptr[row + 1] - beg;
    }
    const bool mine = (d > dlo && d <= SW);
    if (!__any(mine)) return;          // wave-uniform: no row of this class here
    Tr my_rho = (Tr)0;
    int32_t my_id = 0, my_j = 0, my_e = 0;
    if (mine && q < d) {
        my_j = col[beg + q];
        my_e = eid[beg + q];
        my_rho = rho[my_e];
        my_id = orig_id ? orig_id[my_j] : my_j;
    }
    int64_t rank = 0;
    const int base = seg * SW;
#pragma unroll 8
    for (int t = 0; t < SW; ++t) {
        Tr r = shfl(my_rho, base + t);
        int32_t id = shfl(my_id, base + t);
        if (t < d && before(r, id, my_rho, my_id, orient)) ++rank;
    }
    if (mine && q < d) emit(mode, row, my_j, my_e, d, rank, budget, keep, sides);
}

// Order-preserving 64-bit key of (rho, orig_id) for the row's order.
__device__ __forceinline__ unsigned long long sort_key(float r, int32_t id, int orient) {
    uint32_t b = __float_as_uint(r);                 // rho >= 0: bits are monotone
    if (orient == AD_GLOBAL) b = ~b;
    return ((unsigned long long)b << 32) | (unsigned long long)(uint32_t)id;
}

// Listed rows with 64 < d <= 64 * KPL (FP32 distances): one wave per row,
// KPL keys per lane; each key's rank counts the smaller keys of the row,
// broadcast one lane at a time.
template <int KPL>
__global__ __launch_bounds__(SBLOCK) void k_rank_wave(
    const int32_t *__restrict__ list, const unsigned int *__restrict__ count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id, const float *__restrict__ rho,
    int orient, int mode, const int32_t *__restrict__ budget, uint8_t *__restrict__ keep,
    unsigned long long *__restrict__ sides) {
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned int nr = *count;
    const unsigned int waves = gridDim.x * (SBLOCK / WAVE);
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
                key[t] = sort_key(rho[ee[t]], orig_id ? orig_id[jj[t]] : jj[t], orient);
            } else {
                jj[t] = 0;
                ee[t] = 0;
                key[t] = ~0ull;
            }
        }
        int rank[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) rank[t] = 0;
#pragma unroll
        for (int ts = 0; ts < KPL; ++ts) {
            if (ts * WAVE >= d) break;                 // uniform across the wave
            for (int src = 0; src < WAVE; ++src) {
                const unsigned long long k = shfl(key[ts], src);
#pragma unroll
                for (int t = 0; t < KPL; ++t) rank[t] += (k < key[t]) ? 1 : 0;
            }
        }
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
            const int q = t * WAVE + lane;
            if (q < d) emit(mode, row, jj[t], ee[t], d, rank[t], budget, keep, sides);
        }
    }
}

// Listed rows with 64 < d <= SORT_CAP (FP32 distances): bitonic sort in LDS.
__global__ __launch_bounds__(SBLOCK) void k_rank_bitonic(
    const int32_t *__restrict__ list, const unsigned int *__restrict__ count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id, const float *__restrict__ rho,
    int orient, int mode, const int32_t *__restrict__ budget, uint8_t *__restrict__ keep,
    unsigned long long *__restrict__ sides) {
    __shared__ unsigned long long key[SORT_CAP];
    __shared__ uint16_t idx[SORT_CAP];
    const unsigned int nr = *count;
    for (unsigned int h = blockIdx.x; h < nr; h += gridDim.x) {
        const int64_t row = list[h];
        const int64_t beg = row_ptr[row];
        const int d = (int)(row_ptr[row + 1] - beg);
        int P = 1;
        while (P < d) P <<= 1;
        for (int t = threadIdx.x; t < P; t += SBLOCK) {
            if (t < d) {
                int32_t j = col[beg + t];
                key[t] = sort_key(rho[eid[beg + t]], orig_id ? orig_id[j] : j, orient);
            } else {
                key[t] = ~0ull;
            }
            idx[t] = (uint16_t)t;
        }
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = threadIdx.x; t < (P >> 1); t += SBLOCK) {
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
        for (int t = threadIdx.x; t < d; t += SBLOCK) {
            int at = idx[t];
            int64_t p = beg + at;
            emit(mode, row, col[p], eid[p], d, t, budget, keep, sides);
        }
        __syncthreads();
    }
}

// Listed rows ranked by counting against keys read from memory (FP64
// distances with d > 64, or any row longer than SORT_CAP).
template <typename Tr>
__global__ __launch_bounds__(SBLOCK) void k_rank_count(
    const int32_t *__restrict__ list, const unsigned int *__restrict__ count,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ eid, const int32_t *__restrict__ orig_id, const Tr *__restrict__ rho,
    int orient, int mode, const int32_t *__restrict__ budget, uint8_t *__restrict__ keep,
    unsigned long long *__restrict__ sides) {
    const unsigned int nr = *count;
    for (unsigned int h = blockIdx.x; h < nr; h += gridDim.x) {
        const int64_t row = list[h];
        const int64_t beg = row_ptr[row];
        const int64_t d = row_ptr[row + 1] - beg;
        for (int64_t t = threadIdx.x; t < d; t += SBLOCK) {
            const int32_t j = col[beg + t];
            const int32_t e = eid[beg + t];
            const Tr r = rho[e];
            const int32_t id = orig_id ? orig_id[j] : j;
            int64_t rank = 0;
            for (int64_t u = 0; u < d; ++u) {
                const int32_t ju = col[beg + u];
                const Tr ru = rho[eid[beg + u]];
                const int32_t iu = orig_id ? orig_id[ju] : ju;
                if (before(ru, iu, r, id, orient)) ++rank;
            }
            emit(mode, row, j, e, d, rank, budget, keep, sides);
        }
    }
}

// Block-wide sum of per-thread counts; thread 0 adds it to *out (one atomic
// per block; integer addition, so the total does not depend on order).
__device__ __forceinline__ void block_add(unsigned long long c, unsigned long long *out) {
    __shared__ unsigned long long part[SBLOCK / WAVE];
    for (int d = WAVE / 2; d >= 1; d >>= 1) c += shfl_down(c, d);
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < SBLOCK / WAVE; ++w) t += part[w];
        if (t) atomicAdd(out, t);
    }
}

constexpr int COUNT_BLOCKS = 512;

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

// Estimated grid index of each edge's threshold (0: kept at every e).
__global__ void k_fit_grid(int64_t m, const unsigned long long *__restrict__ sides,
                           unsigned long long *__restrict__ G) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long best = ~0ull;
        for (int s = 0; s < 2; ++s) {
            unsigned long long v = sides[2 * e + s];
            unsigned long long d = v >> 32, r = v & 0xffffffffull;
            unsigned long long gidx;
            if (r == 0 || d < 2) {
                gidx = 0;
            } else {
                double t = log((double)(r + 1)) / log((double)d);
                double gi = ceil(t * GRID);
                gidx = gi <= 0.0 ? 0ull : (unsigned long long)gi;
            }
            best = gidx < best ? gidx : best;
        }
        G[e] = best;
    }
}

// state[0] = prefix of selected digits, state[1] = rank still to skip (K-1 based).
__global__ void k_select_init(unsigned long long *state, unsigned long long K) {
    state[0] = 0;
    state[1] = K;
}

__global__ __launch_bounds__(SBLOCK) void k_radix_hist(int64_t m, const unsigned long long *__restrict__ G,
                                                      int shift, int pass,
                                                      const unsigned long long *__restrict__ state,
                                                      unsigned int *__restrict__ hist) {
    __shared__ unsigned int h[NBINS];
    for (int b = threadIdx.x; b < NBINS; b += SBLOCK) h[b] = 0;
    __syncthreads();
    const unsigned long long prefix = state[0];
    // runs of equal bins in one thread's sequence are added at once
    int last = -1;
    unsigned int run = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long g = G[e];
        if (pass > 0 && (g >> (shift + DIGIT)) != prefix) continue;
        const int b = (int)((g >> shift) & (NBINS - 1));
        if (b == last) {
            ++run;
        } else {
            if (run) atomicAdd(&h[last], run);
            last = b;
            run = 1;
        }
    }
    if (run) atomicAdd(&h[last], run);
    __syncthreads();
    for (int b = threadIdx.x; b < NBINS; b += SBLOCK)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

__global__ __launch_bounds__(SBLOCK) void k_radix_pick(const unsigned int *__restrict__ hist,
                                                      unsigned long long *state) {
    __shared__ unsigned long long part[SBLOCK];
    constexpr int PER = NBINS / SBLOCK;
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
        state[0] = (state[0] << DIGIT) | (unsigned long long)bin;
        state[1] = need - run;
    }
}

// Exact counts at two grid points from host budget tables; keep[] for the first.
__global__ __launch_bounds__(SBLOCK) void k_fit_count(int64_t m, const unsigned long long *__restrict__ sides,
                            const int32_t *__restrict__ tab_hi, const int32_t *__restrict__ tab_lo,
                            int use_lo, uint8_t *__restrict__ keep,
                            unsigned long long *__restrict__ counts) {
    unsigned long long c_hi = 0, c_lo = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long a = sides[2 * e], b = sides[2 * e + 1];
        unsigned long long da = a >> 32, ra = a & 0xffffffffull;
        unsigned long long db = b >> 32, rb = b & 0xffffffffull;
        bool k_hi = ra < (unsigned long long)tab_hi[da] || rb < (unsigned long long)tab_hi[db];
        keep[e] = k_hi ? 1 : 0;
        c_hi += k_hi;
        if (use_lo) c_lo += (ra < (unsigned long long)tab_lo[da] || rb < (unsigned long long)tab_lo[db]);
    }
    block_add(c_hi, &counts[0]);
    __syncthreads();
    block_add(c_lo, &counts[1]);
}

__global__ void k_store_count(const unsigned long long *__restrict__ c, int64_t *__restrict__ out) {
    *out = (int64_t)c[0];
}

// ------------------------------------------------------------------- host --

struct SelLayout {
    int32_t *list_big, *list_mid, *list_huge;
    unsigned int *cnt;            // [3]: wave-ranked, huge, LDS-sorted
    unsigned long long *sides;    // [2m]
    unsigned long long *G;        // [m]
    unsigned int *hist;           // [NBINS]
    unsigned long long *state;    // [2]
    unsigned long long *counts;   // [2]
    int32_t *tab_hi, *tab_lo;     // [d_max + 1]
};

static size_t sel_layout(const ad_graph *g, void *ws, size_t ws_bytes, SelLayout *L) {
    Carver c(ws, ws_bytes);
    const int64_t n = std::max<int64_t>(1, g->n), m = std::max<int64_t>(1, g->m);
    SelLayout l;
    l.list_big = c.take<int32_t>(n);
    l.list_mid = c.take<int32_t>(n);
    l.list_huge = c.take<int32_t>(n);
    l.cnt = c.take<unsigned int>(3);
    l.sides = c.take<unsigned long long>(2 * m);
    l.G = c.take<unsigned long long>(m);
    l.hist = c.take<unsigned int>(NBINS);
    l.state = c.take<unsigned long long>(2);
    l.counts = c.take<unsigned long long>(2);
    l.tab_hi = c.take<int32_t>((size_t)g->d_max + 1);
    l.tab_lo = c.take<int32_t>((size_t)g->d_max + 1);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

static void budget_table(int32_t d_max, double e, std::vector<int32_t> &t) {
    t.assign((size_t)d_max + 1, 0);
    for (int32_t d = 1; d <= d_max; ++d) {
        double p = floor(pow((double)d, e));
        int64_t c = (int64_t)p;
        if (c < 1) c = 1;
        if (c > d) c = d;
        t[d] = (int32_t)c;
    }
}

// Rank every entry of every row and emit per `mode`.
template <typename Tr>
static ad_status rank_all(const ad_graph *g, const Tr *rho, int orient, int mode, const int32_t *budget,
                          uint8_t *keep, const SelLayout &L, hipStream_t st) {
    const int64_t n = g->n;
    if (n <= 0 || g->m <= 0) return AD_OK;
    TraceScope trace("k_rank", st);
    const int rows_per_block_8 = (SBLOCK / WAVE) * (WAVE / 8);
    hipLaunchKernelGGL((k_rank_small<Tr, 8>), dim3((unsigned)ceil_div(n, rows_per_block_8)), dim3(SBLOCK), 0,
                       st, n, g->row_ptr, g->col, g->eid, g->orig_id, rho, orient, mode, (int64_t)0, budget,
                       keep, L.sides);
    AD_LAUNCH_CHECK("k_rank_small<8>");
    if (g->d_max > 8) {
        const int rpb = (SBLOCK / WAVE) * (WAVE / 16);
        hipLaunchKernelGGL((k_rank_small<Tr, 16>), dim3((unsigned)ceil_div(n, rpb)), dim3(SBLOCK), 0, st, n,
                           g->row_ptr, g->col, g->eid, g->orig_id, rho, orient, mode, (int64_t)8, budget, keep,
                           L.sides);
        AD_LAUNCH_CHECK("k_rank_small<16>");
    }
    if (g->d_max > 16) {
        const int rpb = (SBLOCK / WAVE) * (WAVE / 32);
        hipLaunchKernelGGL((k_rank_small<Tr, 32>), dim3((unsigned)ceil_div(n, rpb)), dim3(SBLOCK), 0, st, n,
                           g->row_ptr, g->col, g->eid, g->orig_id, rho, orient, mode, (int64_t)16, budget, keep,
                           L.sides);
        AD_LAUNCH_CHECK("k_rank_small<32>");
    }
    if (g->d_max > 32) {
        const int rpb = (SBLOCK / WAVE);
        hipLaunchKernelGGL((k_rank_small<Tr, 64>), dim3((unsigned)ceil_div(n, rpb)), dim3(SBLOCK), 0, st, n,
                           g->row_ptr, g->col, g->eid, g->orig_id, rho, orient, mode, (int64_t)32, budget, keep,
                           L.sides);
        AD_LAUNCH_CHECK("k_rank_small<64>");
    }
    if (g->d_max > 64) {
        ad_status s = fill_i32((int32_t *)L.cnt, 0, 3, st);
        if (s != AD_OK) return s;
        const bool f32 = sizeof(Tr) == 4;
        const int64_t cap = f32 ? SORT_CAP : 64;
        unsigned grid = (unsigned)std::min<int64_t>(2048, n);
        if (f32) {
            s = collect_rows(g, 64, WAVE_CAP, L.list_big, &L.cnt[0], st);
            if (s != AD_OK) return s;
            hipLaunchKernelGGL((k_rank_wave<WAVE_CAP / WAVE>), dim3(grid), dim3(SBLOCK), 0, st, L.list_big,
                               &L.cnt[0], g->row_ptr, g->col, g->eid, g->orig_id, (const float *)rho, orient, mode,
                               budget, keep, L.sides);
            AD_LAUNCH_CHECK("k_rank_wave");
            if (g->d_max > WAVE_CAP) {
                s = collect_rows(g, WAVE_CAP, cap, L.list_mid, &L.cnt[2], st);
                if (s != AD_OK) return s;
                hipLaunchKernelGGL(k_rank_bitonic, dim3(grid), dim3(SBLOCK), 0, st, L.list_mid, &L.cnt[2],
                                   g->row_ptr, g->col, g->eid, g->orig_id, (const float *)rho, orient, mode,
                                   budget, keep, L.sides);
                AD_LAUNCH_CHECK("k_rank_bitonic");
            }
        }
        if (g->d_max > cap) {
            s = collect_rows(g, cap, (int64_t)1 << 62, L.list_huge, &L.cnt[1], st);
            if (s != AD_OK) return s;
            hipLaunchKernelGGL((k_rank_count<Tr>), dim3(grid), dim3(SBLOCK), 0, st, L.list_huge, &L.cnt[1],
                               g->row_ptr, g->col, g->eid, g->orig_id, rho, orient, mode, budget, keep,
                               L.sides);
            AD_LAUNCH_CHECK("k_rank_count");
        }
    }
    return AD_OK;
}

static ad_status check_sel_args(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                                uint8_t *keep, int64_t *n_kept, void *ws, size_t ws_bytes, SelLayout *L) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (rho_dtype != AD_F32 && rho_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "rho must be F32 or F64");
    if (orient != AD_LOCAL && orient != AD_GLOBAL) return fail(AD_ERR_INVALID_ARG, "unknown orientation");
    if (g->m > 0 && (!rho || !keep)) return fail(AD_ERR_INVALID_ARG, "rho or keep is NULL");
    if (!n_kept) return fail(AD_ERR_INVALID_ARG, "n_kept is NULL");
    if (g->m > 0 && g->d_max <= 0) return fail(AD_ERR_INVALID_ARG, "d_max must be set for selection");
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (sel_layout(g, ws, ws_bytes, L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    return AD_OK;
}

}  // namespace ad

using namespace ad;

extern "C" ad_status ad_edge_dist(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                                  const double *minmax, void *rho, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (R < 1 || R > 64) return fail(AD_ERR_INVALID_ARG, "R must be in [1, 64]");
    if (x_dtype != AD_F32 && x_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "x must be F32 or F64");
    if (g->m > 0 && (!x || !minmax || !rho)) return fail(AD_ERR_INVALID_ARG, "x, minmax or rho is NULL");
    if (g->n <= 0 || g->m <= 0) return AD_OK;
    const double avg = (double)(2 * g->m) / (double)g->n;
    int lpr = 1;
    while (lpr < 64 && lpr < avg) lpr <<= 1;   // lanes per row ~ average degree
    const unsigned nb = (unsigned)ceil_div(g->n, SBLOCK / lpr);
    TraceScope trace("k_edge_dist", stream);
    if (x_dtype == AD_F64) {
        if (R % 2 == 0)
            hipLaunchKernelGGL((k_edge_dist<double, double, 2>), dim3(nb), dim3(SBLOCK), 0, stream, g->n, g->row_ptr,
                               g->col, g->eid, (const double *)x, minmax, (double *)rho, R, lpr);
        else
            hipLaunchKernelGGL((k_edge_dist<double, double, 1>), dim3(nb), dim3(SBLOCK), 0, stream, g->n, g->row_ptr,
                               g->col, g->eid, (const double *)x, minmax, (double *)rho, R, lpr);
    } else {
        if (R % 4 == 0)
            hipLaunchKernelGGL((k_edge_dist<float, float, 4>), dim3(nb), dim3(SBLOCK), 0, stream, g->n, g->row_ptr,
                               g->col, g->eid, (const float *)x, minmax, (float *)rho, R, lpr);
        else if (R % 2 == 0)
            hipLaunchKernelGGL((k_edge_dist<float, float, 2>), dim3(nb), dim3(SBLOCK), 0, stream, g->n, g->row_ptr,
                               g->col, g->eid, (const float *)x, minmax, (float *)rho, R, lpr);
        else
            hipLaunchKernelGGL((k_edge_dist<float, float, 1>), dim3(nb), dim3(SBLOCK), 0, stream, g->n, g->row_ptr,
                               g->col, g->eid, (const float *)x, minmax, (float *)rho, R, lpr);
    }
    AD_LAUNCH_CHECK("k_edge_dist");
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

extern "C" ad_status ad_sparsify(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                                 const int32_t *budget, uint8_t *keep, int64_t *n_kept, void *ws,
                                 size_t ws_bytes, hipStream_t stream) {
    SelLayout L;
    ad_status s = check_sel_args(g, rho_dtype, rho, orient, keep, n_kept, ws, ws_bytes, &L);
    if (s != AD_OK) return s;
    if (g->m > 0 && !budget) return fail(AD_ERR_INVALID_ARG, "budget is NULL");
    s = fill_u64(L.counts, 0, 1, stream);
    if (s != AD_OK) return s;
    if (g->m > 0) {
        s = fill_u8(keep, 0, g->m, stream);
        if (s != AD_OK) return s;
        if (rho_dtype == AD_F32)
            s = rank_all<float>(g, (const float *)rho, orient, MODE_FIXED, budget, keep, L, stream);
        else
            s = rank_all<double>(g, (const double *)rho, orient, MODE_FIXED, budget, keep, L, stream);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_count_bytes, dim3((unsigned)std::min<int64_t>(COUNT_BLOCKS, ceil_div(g->m, SBLOCK))),
                           dim3(SBLOCK), 0, stream, g->m, keep,
                           L.counts);
        AD_LAUNCH_CHECK("k_count_bytes");
    }
    hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, stream, L.counts, n_kept);
    AD_LAUNCH_CHECK("k_store_count");
    return AD_OK;
}

extern "C" ad_status ad_sparsify_fit(const ad_graph *g, ad_dtype rho_dtype, const void *rho, ad_orient orient,
                                     double target, uint8_t *keep, int64_t *n_kept, double *e_used_host,
                                     void *ws, size_t ws_bytes, hipStream_t stream) {
    SelLayout L;
    ad_status s = check_sel_args(g, rho_dtype, rho, orient, keep, n_kept, ws, ws_bytes, &L);
    if (s != AD_OK) return s;
    if (!(target > 0.0 && target <= 1.0)) return fail(AD_ERR_INVALID_ARG, "target must be in (0, 1]");
    if (!e_used_host) return fail(AD_ERR_INVALID_ARG, "e_used_host is NULL");
    const int64_t m = g->m;
    s = fill_u64(L.counts, 0, 2, stream);
    if (s != AD_OK) return s;
    if (m == 0) {
        hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, stream, L.counts, n_kept);
        AD_LAUNCH_CHECK("k_store_count");
        AD_HIP(hipStreamSynchronize(stream));
        *e_used_host = 0.0;
        return AD_OK;
    }
    // Fewest kept edges meeting the target, in the bisection's own test.
    int64_t K = (int64_t)ceil(target * (double)m);
    if (K < 1) K = 1;
    if (K > m) K = m;
    while (K > 1 && (double)(K - 1) / (double)m >= target) --K;
    while (K < m && (double)K / (double)m < target) ++K;

    if (rho_dtype == AD_F32)
        s = rank_all<float>(g, (const float *)rho, orient, MODE_SIDES, nullptr, keep, L, stream);
    else
        s = rank_all<double>(g, (const double *)rho, orient, MODE_SIDES, nullptr, keep, L, stream);
    if (s != AD_OK) return s;
    TraceScope trace_fit("k_fit_select", stream);
    hipLaunchKernelGGL(k_fit_grid, dim3(grid_for(m, SBLOCK)), dim3(SBLOCK), 0, stream, m, L.sides, L.G);
    AD_LAUNCH_CHECK("k_fit_grid");
    hipLaunchKernelGGL(k_select_init, dim3(1), dim3(1), 0, stream, L.state, (unsigned long long)K);
    AD_LAUNCH_CHECK("k_select_init");
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = (3 - pass) * DIGIT;
        s = fill_i32((int32_t *)L.hist, 0, NBINS, stream);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)std::min<int64_t>(COUNT_BLOCKS, ceil_div(m, SBLOCK))),
                           dim3(SBLOCK), 0, stream, m, L.G, shift, pass,
                           L.state, L.hist);
        AD_LAUNCH_CHECK("k_radix_hist");
        hipLaunchKernelGGL(k_radix_pick, dim3(1), dim3(SBLOCK), 0, stream, L.hist, L.state);
        AD_LAUNCH_CHECK("k_radix_pick");
    }
    unsigned long long gstar = 0;
    AD_HIP(hipMemcpyAsync(&gstar, L.state, sizeof(gstar), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipStreamSynchronize(stream));
    const unsigned long long GMAX = 1ull << 40;
    if (gstar > GMAX) gstar = GMAX;

    // Confirm with exact budget tables: count(g) >= K and count(g - 1) < K.
    std::vector<int32_t> th, tl;
    unsigned long long hc[2];
    long long g_try = (long long)gstar;
    for (int attempt = 0; attempt < 64; ++attempt) {
        const double e_hi = (double)g_try / GRID;
        const bool use_lo = g_try > 0;
        budget_table(g->d_max, e_hi, th);
        if (use_lo) budget_table(g->d_max, (double)(g_try - 1) / GRID, tl);
        else tl = th;
        AD_HIP(hipMemcpyAsync(L.tab_hi, th.data(), th.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
        AD_HIP(hipMemcpyAsync(L.tab_lo, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
        s = fill_u64(L.counts, 0, 2, stream);
        if (s != AD_OK) return s;
        hipLaunchKernelGGL(k_fit_count, dim3((unsigned)std::min<int64_t>(COUNT_BLOCKS, ceil_div(m, SBLOCK))),
                           dim3(SBLOCK), 0, stream, m, L.sides, L.tab_hi,
                           L.tab_lo, use_lo ? 1 : 0, keep, L.counts);
        AD_LAUNCH_CHECK("k_fit_count");
        AD_HIP(hipMemcpyAsync(hc, L.counts, sizeof(hc), hipMemcpyDeviceToHost, stream));
        AD_HIP(hipStreamSynchronize(stream));
        const bool hi_ok = (int64_t)hc[0] >= K;
        const bool lo_ok = !use_lo || (int64_t)hc[1] < K;
        if (hi_ok && lo_ok) {
            hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, stream, L.counts, n_kept);
            AD_LAUNCH_CHECK("k_store_count");
            AD_HIP(hipStreamSynchronize(stream));
            *e_used_host = e_hi;
            return AD_OK;
        }
        if (!hi_ok) {
            if (g_try >= (long long)GMAX) break;
            ++g_try;
        } else {
            --g_try;
        }
    }
    return fail(AD_ERR_INTERNAL, "retention fit did not settle on a grid point");
}
