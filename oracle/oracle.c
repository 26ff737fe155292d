/*
 * oracle.c -- plain FP64 CPU oracle for algebraic-distance sparsification
 * (John & Safro, "Single- and Multi-level Network Sparsification by
 * Algebraic Distance", arXiv 1601.05527).
 *
 * TEST INFRASTRUCTURE.  This file exists to check the HIP library: only the
 * tests, the smoke check and the benchmark's CPU-baseline leg call it.  It
 * shares no code, header or table with the library; it follows the paper's
 * algorithms step by step, in double precision, with plain loops (one
 * sequential sum per row, in CSR order).  OpenMP only splits independent
 * vertices across threads, as the paper's own implementation does
 * (Section 6.4, "Parallelization").
 *
 * Graph input: symmetric CSR of an undirected simple graph (Preliminaries):
 *   row_ptr[n+1] (int64), col[2m] (int32), w[2m] (float, NULL = unit),
 *   eid[2m] (int32 undirected edge id shared by both mirror entries),
 *   orig_id[n] (int32, NULL = identity).
 *
 * Readings of points the paper leaves open (the library follows the same
 * readings with its own code):
 *   - relaxation weight: the parameter omega multiplies the neighbour
 *     average, the paper's alpha = 1 - omega multiplies the old value
 *     (Algorithm 1; every experiment uses 1/2, where both coincide);
 *   - R vectors r = 0..R-1, k sweeps t = 1..k, each reading only t-1 values
 *     (Jacobi, Algorithm 1);
 *   - random start: uniform values from Philox4x64-10 (Salmon et al.,
 *     SC'11), key (seed, graph_id), counter (orig_id[i], r/4, 0, 0), word
 *     r%4, top 24 bits scaled by 2^-24, minus 1/2;
 *   - isolated vertices keep their value, are left out of the rescale's
 *     min/max and have no edges;
 *   - "rescale x back to (-0.5, 0.5)": once per vector after the sweeps, the
 *     min-max affine map onto [-1/2, 1/2] over non-isolated vertices; a
 *     degenerate range maps to 0;
 *   - distance: rho_e = sqrt(sum_r (xhat_i - xhat_j)^2) (Algorithm 1), the
 *     strength delta_e = 1/sqrt(rho_e^2 + eps) is monotone in rho_e;
 *   - budget of vertex i: c_i = min(d_i, max(1, floor(pow(d_i, e)))) with
 *     the C library's double pow (Section 4, "top d_i^e");
 *   - LOCAL keeps the delta-strong edges (rho ascending), GLOBAL the
 *     delta-weak ones (rho descending); ties in rho go to the smaller
 *     orig_id of the neighbour in both orientations; an edge is kept when
 *     either endpoint selects it (Algorithm 3);
 *   - retention fit: bisection on e in [0, 1], 40 halvings, returning the
 *     smallest e found whose retained fraction reaches the target (the
 *     binary-search fitting of Section 6.2).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops below (a timing knob of the test harness; the
 * results do not depend on it).  Without OpenMP both calls are no-ops and
 * one thread runs. */
void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10, written from the published definition (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11):
 * ten rounds of two 64x64->128 multiplications with the round key bumped by
 * the Weyl constants between rounds.                                        */

static void orc_mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t mul0 = 0xD2E7470EE14C6C93ULL, mul1 = 0xCA5A826395121157ULL;
    const uint64_t weyl0 = 0x9E3779B97F4A7C15ULL, weyl1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += weyl0; k1 += weyl1; }
        uint64_t hi0, lo0, hi1, lo1;
        orc_mulhilo64(mul0, x0, &hi0, &lo0);
        orc_mulhilo64(mul1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* x_i^(0) <- rand(-0.5, 0.5) for test vector r (Algorithm 1). */
double orc_start_value(uint64_t seed, uint64_t graph_id, int32_t vertex_key, int32_t r)
{
    uint64_t key[2] = {seed, graph_id};
    uint64_t ctr[4] = {(uint64_t)(uint32_t)vertex_key, (uint64_t)(r / 4), 0, 0};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    uint64_t top24 = out[r % 4] >> 40;
    return (double)top24 * (1.0 / 16777216.0) - 0.5;
}

/* All R start vectors, stored [n][R]. */
void orc_start_vectors(int64_t n, int32_t R, uint64_t seed, uint64_t graph_id,
                       const int32_t *orig_id, double *x0)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t r = 0; r < R; ++r)
            x0[i * R + r] = orc_start_value(seed, graph_id,
                                            orig_id ? orig_id[i] : (int32_t)i, r);
}

/* ------------------------------------------------------------------------ */
/* One JOR sweep of one test vector (Algorithm 1):
 *   x_i^(t) = (1 - omega) x_i^(t-1) + omega * sum_j w_ij x_j^(t-1) / sum_j w_ij
 * Isolated vertices keep their value.                                       */
static void orc_jor_sweep(int64_t n, const int64_t *row_ptr, const int32_t *col,
                          const float *w, double omega, const double *x_old,
                          double *x_new)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        int64_t beg = row_ptr[i], end = row_ptr[i + 1];
        if (beg == end) { x_new[i] = x_old[i]; continue; }
        double num = 0.0, den = 0.0;
        for (int64_t p = beg; p < end; ++p) {
            double wij = w ? (double)w[p] : 1.0;
            num += wij * x_old[col[p]];
            den += wij;
        }
        x_new[i] = (1.0 - omega) * x_old[i] + omega * (num / den);
    }
}

/* k sweeps of one vector; x holds x^(0) on entry and x^(k) on exit.
 * If trace != NULL it receives x^(0..k) as trace[t*n + i].                   */
void orc_relax_vector(int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const float *w, int32_t k, double omega, double *x,
                      double *trace)
{
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (trace) memcpy(trace, x, sizeof(double) * (size_t)n);
    for (int32_t t = 1; t <= k; ++t) {
        orc_jor_sweep(n, row_ptr, col, w, omega, x, tmp);
        memcpy(x, tmp, sizeof(double) * (size_t)n);
        if (trace) memcpy(trace + (size_t)t * (size_t)n, x, sizeof(double) * (size_t)n);
    }
    free(tmp);
}

/* "Rescale x back to (-0.5, 0.5)" (Algorithm 1): min-max map over the
 * non-isolated vertices.  Returns min and max through lo/hi.                 */
void orc_rescale_vector(int64_t n, const int64_t *row_ptr, const double *x,
                        double *xhat, double *lo, double *hi)
{
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] == row_ptr[i]) continue;
        if (x[i] < mn) mn = x[i];
        if (x[i] > mx) mx = x[i];
    }
    for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] == row_ptr[i] || !(mx > mn)) xhat[i] = 0.0;
        else xhat[i] = (x[i] - mn) / (mx - mn) - 0.5;
    }
    if (lo) *lo = mn;
    if (hi) *hi = mx;
}

/* ComputeAlgDist (Algorithm 1) for R test vectors, returning the L2
 * algebraic distance rho_e = sqrt(R_e) per undirected edge.
 *   x0     : NULL -> Philox start vectors; else [n][R] start values.
 *   xk     : optional [n][R] output of x^(k) (before the rescale).
 *   xhat   : optional [n][R] output of the rescaled vectors.
 *   minmax : optional [2R] output, min then max of each x^(k).
 */
void orc_algebraic_distance(int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const float *w, const int32_t *eid,
                            const int32_t *orig_id, int64_t m, int32_t R,
                            int32_t k, double omega, uint64_t seed,
                            uint64_t graph_id, const double *x0, double *rho,
                            double *xk, double *xhat, double *minmax)
{
    double *acc = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    double *x = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *xh = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t r = 0; r < R; ++r) {
        for (int64_t i = 0; i < n; ++i)
            x[i] = x0 ? x0[i * R + r]
                      : orc_start_value(seed, graph_id,
                                        orig_id ? orig_id[i] : (int32_t)i, r);
        orc_relax_vector(n, row_ptr, col, w, k, omega, x, NULL);
        double lo, hi;
        orc_rescale_vector(n, row_ptr, x, xh, &lo, &hi);
        if (minmax) { minmax[r] = lo; minmax[R + r] = hi; }
        if (xk) for (int64_t i = 0; i < n; ++i) xk[i * R + r] = x[i];
        if (xhat) for (int64_t i = 0; i < n; ++i) xhat[i * R + r] = xh[i];
        /* R_ij += (x_i - x_j)^2 over every edge, visited from its upper entry */
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                int32_t j = col[p];
                if (j <= i) continue;
                double d = xh[i] - xh[j];
                acc[eid[p]] += d * d;
            }
    }
    for (int64_t e = 0; e < m; ++e) rho[e] = sqrt(acc[e]);
    free(acc); free(x); free(xh);
}

/* delta_e = 1 / sqrt(rho_e^2 + eps) (Algorithm 1, return step). */
void orc_strength(int64_t m, const double *rho, double eps, double *delta)
{
    for (int64_t e = 0; e < m; ++e) delta[e] = 1.0 / sqrt(rho[e] * rho[e] + eps);
}

/* Optional normalization (Algorithm 1, last step): delta_e is divided by
 * sqrt(f_i f_j), where f is the degree d_i (as Algorithm 1 writes it) or,
 * with by_strength, the weighted degree s_i = sum_j w_ij (as the text
 * around it says).  Written as the distance whose reciprocal is the
 * normalized delta: out_e = sqrt(rho_e^2 + eps) * sqrt(f_i * f_j), so that
 * the normalized delta-strong edges are the ones with small out_e.
 * Every edge is visited from its upper entry (j > i).                      */
void orc_normalize_dist(int64_t n, const int64_t *row_ptr, const int32_t *col,
                        const float *w, const int32_t *eid, const double *rho,
                        int32_t by_strength, double eps, double *out)
{
    double *f = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            acc += (by_strength && w) ? (double)w[p] : 1.0;
        f[i] = acc;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t j = col[p];
            if (j <= i) continue;
            double r = rho[eid[p]];
            out[eid[p]] = sqrt(r * r + eps) * sqrt(f[i] * f[j]);
        }
    free(f);
}

/* ------------------------------------------------------------------------ */
/* Sparsify (Algorithm 3).                                                   */

/* Budget of a vertex of degree d: the top d^e neighbours, at least one. */
int64_t orc_budget(int64_t d, double e)
{
    if (d <= 0) return 0;
    double p = floor(pow((double)d, e));
    int64_t c = (int64_t)p;
    if (c < 1) c = 1;
    if (c > d) c = d;
    return c;
}

typedef struct { double rho; int32_t other; int32_t edge; } orc_item;

static int orc_cmp_local(const void *a, const void *b)
{
    const orc_item *x = (const orc_item *)a, *y = (const orc_item *)b;
    if (x->rho < y->rho) return -1;
    if (x->rho > y->rho) return 1;
    return (x->other > y->other) - (x->other < y->other);
}

static int orc_cmp_global(const void *a, const void *b)
{
    const orc_item *x = (const orc_item *)a, *y = (const orc_item *)b;
    if (x->rho > y->rho) return -1;
    if (x->rho < y->rho) return 1;
    return (x->other > y->other) - (x->other < y->other);
}

/* For every vertex: sort N_i by rho (ascending for LOCAL = 0, descending
 * for GLOBAL = 1), add the top c_i edges.  keep[m] receives 0/1; returns the
 * number of kept edges.                                                      */
int64_t orc_sparsify(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const int32_t *eid, const int32_t *orig_id, int64_t m,
                     const double *rho, int32_t orient, double e, uint8_t *keep)
{
    memset(keep, 0, (size_t)m);
#pragma omp parallel
    {
        orc_item *buf = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            int64_t beg = row_ptr[i], d = row_ptr[i + 1] - beg;
            if (d == 0) continue;
            if (d > cap) { free(buf); cap = d; buf = (orc_item *)malloc(sizeof(orc_item) * (size_t)cap); }
            for (int64_t q = 0; q < d; ++q) {
                int32_t j = col[beg + q];
                buf[q].rho = rho[eid[beg + q]];
                buf[q].other = orig_id ? orig_id[j] : j;
                buf[q].edge = eid[beg + q];
            }
            qsort(buf, (size_t)d, sizeof(orc_item), orient == 0 ? orc_cmp_local : orc_cmp_global);
            int64_t c = orc_budget(d, e);
            for (int64_t q = 0; q < c; ++q) keep[buf[q].edge] = 1;   /* same value from any writer */
        }
        free(buf);
    }
    int64_t kept = 0;
    for (int64_t q = 0; q < m; ++q) kept += keep[q];
    return kept;
}

/* Binary-search fitting of e to a target retention ratio |E_s|/|E|. */
double orc_fit_exponent(int64_t n, const int64_t *row_ptr, const int32_t *col,
                        const int32_t *eid, const int32_t *orig_id, int64_t m,
                        const double *rho, int32_t orient, double target,
                        uint8_t *keep, int64_t *n_kept)
{
    if (m == 0) { if (n_kept) *n_kept = 0; return 0.0; }
    int64_t kept = orc_sparsify(n, row_ptr, col, eid, orig_id, m, rho, orient, 0.0, keep);
    if ((double)kept / (double)m >= target) { if (n_kept) *n_kept = kept; return 0.0; }
    double lo = 0.0, hi = 1.0;
    for (int step = 0; step < 40; ++step) {
        double mid = 0.5 * (lo + hi);
        kept = orc_sparsify(n, row_ptr, col, eid, orig_id, m, rho, orient, mid, keep);
        if ((double)kept / (double)m >= target) hi = mid; else lo = mid;
    }
    kept = orc_sparsify(n, row_ptr, col, eid, orig_id, m, rho, orient, hi, keep);
    if (n_kept) *n_kept = kept;
    return hi;
}

/* ------------------------------------------------------------------------ */
/* Sparsify with binning (Algorithm 4, SparsifyB; bin rule of Section 4).
 *
 * The paper spreads N_i's distances over bins of width h = 3.5 sigma /
 * d_i^(1/3) (Scott's rule for a sample of d_i values), (max - min) / h of
 * them, and takes edges from all bins at random, up to d_i^e.  Readings:
 *   - the values binned are the per-edge distances handed in (rho, or its
 *     normalised form), sigma their population standard deviation over N_i
 *     (two passes in double, then rounded to single precision so that the
 *     bins do not depend on summation order), min and max exact;
 *   - h = (3.5 sigma) / cbrt(d_i) in double; number of bins
 *     B_i = max(1, ceil((max - min) / h)), or 1 when h == 0; entry q of
 *     N_i falls in bin min(B_i - 1, floor((rho_q - min) / h));
 *   - random order: vertex i draws a 32-bit key K_i, the low half of word 0
 *     of Philox4x64-10 with key (seed, graph_id) and counter (orig_id[i], 0,
 *     1, 0); its neighbour j gets priority u = fmix32(orig_id[j] ^ K_i),
 *     fmix32 being the 32-bit finalizer of MurmurHash3 (Appleby), a
 *     bijection, so priorities within N_i are distinct;
 *   - "randomly select bins and edges": rounds r = 0, 1, ...; in each round
 *     the non-empty bins are visited in increasing order of their smallest
 *     priority, and each bin still holding an unselected edge gives up the
 *     one of smallest priority; selection stops at c_i = budget(d_i, e)
 *     edges.  Bins are sampled evenly and every bin gets an edge before any
 *     bin gets a second; the selected sets grow with e, so the retention
 *     fit of Algorithm 3 applies unchanged;
 *   - an edge is kept when either endpoint selects it.                      */

static uint32_t orc_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

uint32_t orc_bin_vertex_key(uint64_t seed, uint64_t graph_id, int32_t vertex_key)
{
    uint64_t ctr[4] = {(uint64_t)(uint32_t)vertex_key, 0, 1, 0};
    uint64_t key[2] = {seed, graph_id};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return (uint32_t)out[0];
}

uint32_t orc_bin_priority(uint32_t vertex_key_bits, int32_t neighbour_key)
{
    return orc_fmix32((uint32_t)neighbour_key ^ vertex_key_bits);
}

/* Bins of N_i: nbins (returned) and bin[q] for q < d (values v[q]). */
static int64_t orc_bins_of(int64_t d, const double *v, int32_t *bin)
{
    double mn = v[0], mx = v[0], sum = 0.0;
    for (int64_t q = 0; q < d; ++q) {
        if (v[q] < mn) mn = v[q];
        if (v[q] > mx) mx = v[q];
        sum += v[q];
    }
    double mean = sum / (double)d, ss = 0.0;
    for (int64_t q = 0; q < d; ++q) ss += (v[q] - mean) * (v[q] - mean);
    double sigma = (double)(float)sqrt(ss / (double)d);
    double h = (3.5 * sigma) / cbrt((double)d);
    int64_t nb = 1;
    if (h > 0.0) {
        double k = ceil((mx - mn) / h);
        nb = k < 1.0 ? 1 : (int64_t)k;
    }
    for (int64_t q = 0; q < d; ++q) {
        int64_t b = 0;
        if (h > 0.0) {
            b = (int64_t)floor((v[q] - mn) / h);
            if (b > nb - 1) b = nb - 1;
        }
        bin[q] = (int32_t)b;
    }
    return nb;
}

/* The binning step alone, per CSR entry: bin[2m] and nbins[n]. */
void orc_bin_layout(int64_t n, const int64_t *row_ptr, const int32_t *eid, const double *rho,
                    int32_t *bin, int64_t *nbins)
{
#pragma omp parallel
    {
        double *v = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            int64_t beg = row_ptr[i], d = row_ptr[i + 1] - beg;
            nbins[i] = 0;
            if (d == 0) continue;
            if (d > cap) { free(v); cap = d; v = (double *)malloc(sizeof(double) * (size_t)cap); }
            for (int64_t q = 0; q < d; ++q) v[q] = rho[eid[beg + q]];
            nbins[i] = orc_bins_of(d, v, bin + beg);
        }
        free(v);
    }
}

typedef struct { int32_t bin; uint32_t u; int64_t pos; } orc_bitem;
typedef struct { uint32_t first_u; int64_t start, size; } orc_bin;

static int orc_cmp_bin_u(const void *a, const void *b)
{
    const orc_bitem *x = (const orc_bitem *)a, *y = (const orc_bitem *)b;
    if (x->bin != y->bin) return x->bin < y->bin ? -1 : 1;
    return (x->u > y->u) - (x->u < y->u);
}

static int orc_cmp_first_u(const void *a, const void *b)
{
    const orc_bin *x = (const orc_bin *)a, *y = (const orc_bin *)b;
    return (x->first_u > y->first_u) - (x->first_u < y->first_u);
}

/* Each vertex's own choices at exponent e: chosen[p] = 1 for the CSR
 * entries p that vertex row(p) selects.                                    */
void orc_binned_choices(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *eid,
                        const int32_t *orig_id, const double *rho, uint64_t seed, uint64_t graph_id,
                        double e, uint8_t *chosen)
{
#pragma omp parallel
    {
        orc_bitem *it = NULL;
        orc_bin *bins = NULL;
        double *v = NULL;
        int32_t *bin = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            int64_t beg = row_ptr[i], d = row_ptr[i + 1] - beg;
            if (d == 0) continue;
            if (d > cap) {
                free(it); free(bins); free(v); free(bin);
                cap = d;
                it = (orc_bitem *)malloc(sizeof(orc_bitem) * (size_t)cap);
                bins = (orc_bin *)malloc(sizeof(orc_bin) * (size_t)cap);
                v = (double *)malloc(sizeof(double) * (size_t)cap);
                bin = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            }
            for (int64_t q = 0; q < d; ++q) {
                v[q] = rho[eid[beg + q]];
                chosen[beg + q] = 0;
            }
            orc_bins_of(d, v, bin);
            uint32_t K = orc_bin_vertex_key(seed, graph_id, orig_id ? orig_id[i] : (int32_t)i);
            for (int64_t q = 0; q < d; ++q) {
                int32_t j = col[beg + q];
                it[q].bin = bin[q];
                it[q].u = orc_bin_priority(K, orig_id ? orig_id[j] : j);
                it[q].pos = beg + q;
            }
            /* each bin's edges in priority order, then the bins by their first priority */
            qsort(it, (size_t)d, sizeof(orc_bitem), orc_cmp_bin_u);
            int64_t nb = 0;
            for (int64_t q = 0; q < d; ++q) {
                if (q == 0 || it[q].bin != it[q - 1].bin) {
                    bins[nb].first_u = it[q].u;
                    bins[nb].start = q;
                    bins[nb].size = 0;
                    ++nb;
                }
                bins[nb - 1].size++;
            }
            qsort(bins, (size_t)nb, sizeof(orc_bin), orc_cmp_first_u);
            /* rounds over the bins until c_i edges are taken */
            int64_t c = orc_budget(d, e), taken = 0;
            for (int64_t r = 0; taken < c; ++r)
                for (int64_t b = 0; b < nb && taken < c; ++b)
                    if (r < bins[b].size) {
                        chosen[it[bins[b].start + r].pos] = 1;
                        ++taken;
                    }
        }
        free(it); free(bins); free(v); free(bin);
    }
}

/* SparsifyB at exponent e: keep[m] = 1 when either endpoint chooses the
 * edge; returns the kept count.                                            */
int64_t orc_sparsify_binned(int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const int32_t *eid, const int32_t *orig_id, int64_t m,
                            const double *rho, uint64_t seed, uint64_t graph_id, double e,
                            uint8_t *keep)
{
    memset(keep, 0, (size_t)m);
    int64_t nnz = row_ptr[n];
    uint8_t *chosen = (uint8_t *)malloc(nnz > 0 ? (size_t)nnz : 1);
    orc_binned_choices(n, row_ptr, col, eid, orig_id, rho, seed, graph_id, e, chosen);
    for (int64_t p = 0; p < nnz; ++p)
        if (chosen[p]) keep[eid[p]] = 1;
    free(chosen);
    int64_t kept = 0;
    for (int64_t q = 0; q < m; ++q) kept += keep[q];
    return kept;
}

/* The binary-search fitting of e (as orc_fit_exponent) for SparsifyB. */
double orc_fit_exponent_binned(int64_t n, const int64_t *row_ptr, const int32_t *col,
                               const int32_t *eid, const int32_t *orig_id, int64_t m,
                               const double *rho, uint64_t seed, uint64_t graph_id, double target,
                               uint8_t *keep, int64_t *n_kept)
{
    if (m == 0) { if (n_kept) *n_kept = 0; return 0.0; }
    int64_t kept = orc_sparsify_binned(n, row_ptr, col, eid, orig_id, m, rho, seed, graph_id, 0.0, keep);
    if ((double)kept / (double)m >= target) { if (n_kept) *n_kept = kept; return 0.0; }
    double lo = 0.0, hi = 1.0;
    for (int step = 0; step < 40; ++step) {
        double mid = 0.5 * (lo + hi);
        kept = orc_sparsify_binned(n, row_ptr, col, eid, orig_id, m, rho, seed, graph_id, mid, keep);
        if ((double)kept / (double)m >= target) hi = mid; else lo = mid;
    }
    kept = orc_sparsify_binned(n, row_ptr, col, eid, orig_id, m, rho, seed, graph_id, hi, keep);
    if (n_kept) *n_kept = kept;
    return hi;
}

/* ------------------------------------------------------------------------ */
/* Ingest: an edge list into the graph model of Section 2 (undirected, no
 * self-loops, no repeated pairs), as the symmetric CSR the other functions
 * read.  Readings: a listed pair (u, v) and (v, u) name the same edge;
 * self-loops are dropped; repeated pairs are merged into one edge whose
 * weight is the exact sum of the listed weights rounded once to single
 * precision (orc_exact_sum_f32); listed weights must be finite and
 * positive (the graph model's w > 0); edge ids enumerate the edges in order
 * of (smaller endpoint, larger endpoint), which is the CSR order of their
 * upper entries; each row lists its neighbours in ascending order.  With
 * order == 1 the vertices are stored by decreasing degree, ties by their id
 * in the list; with order == 2 in reverse Cuthill-McKee order (orc_rcm);
 * orig_out[new id] names the listed vertex (through orig_in when given).  Returns the number of edges m, -1 when an endpoint
 * lies outside [0, n), -2 for a weight that is not finite and positive;
 * n_dropped receives m_in - m.                                             */

typedef struct { int64_t a, b, idx; } orc_pair;

static int orc_cmp_pair(const void *x, const void *y)
{
    const orc_pair *p = (const orc_pair *)x, *q = (const orc_pair *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

typedef struct { int64_t row, col, e; } orc_entry;

static int orc_cmp_entry(const void *x, const void *y)
{
    const orc_entry *p = (const orc_entry *)x, *q = (const orc_entry *)y;
    if (p->row != q->row) return p->row < q->row ? -1 : 1;
    return (p->col > q->col) - (p->col < q->col);
}

typedef struct { int64_t deg, id; } orc_vdeg;

static int orc_cmp_vdeg(const void *x, const void *y)
{
    const orc_vdeg *p = (const orc_vdeg *)x, *q = (const orc_vdeg *)y;
    if (p->deg != q->deg) return p->deg > q->deg ? -1 : 1;     /* decreasing degree */
    return (p->id > q->id) - (p->id < q->id);
}

/* The exact sum of cnt positive finite floats, rounded once to single
 * precision (to nearest, ties to even).  Every float is an integer multiple
 * of 2^-149, so the sum is kept exactly as an integer count of 2^-149 in 11
 * base-2^32 digits (the largest float is below 2^277 such units; 2^31 of
 * them stay below 2^308).                                                  */
float orc_exact_sum_f32(const float *x, int64_t cnt)
{
    uint32_t dg[11];
    memset(dg, 0, sizeof(dg));
    for (int64_t q = 0; q < cnt; ++q) {
        uint32_t bits;
        memcpy(&bits, &x[q], sizeof(bits));
        uint32_t ex = (bits >> 23) & 0xffu, fr = bits & 0x7fffffu;
        uint64_t mant = ex ? (uint64_t)(fr | 0x800000u) : (uint64_t)fr;
        int shift = ex ? (int)ex - 1 : 0;          /* x = mant * 2^(shift - 149) */
        int k = shift / 32;
        uint64_t add = mant << (shift % 32);       /* below 2^56 */
        uint64_t carry = 0;
        for (int j = k; j < 11; ++j) {
            uint64_t part = j == k ? (add & 0xffffffffu) : (j == k + 1 ? add >> 32 : 0);
            uint64_t t = (uint64_t)dg[j] + part + carry;
            dg[j] = (uint32_t)t;
            carry = t >> 32;
            if (j > k && carry == 0) break;
        }
    }
    int top = -1;                                  /* highest set bit of the count */
    for (int j = 10; j >= 0 && top < 0; --j)
        for (int b = 31; b >= 0; --b)
            if ((dg[j] >> b) & 1u) { top = 32 * j + b; break; }
    if (top < 0) return 0.0f;
    if (top <= 23) return ldexpf((float)dg[0], -149);   /* below 2^24 units: exact */
    uint32_t mant = 0;
    for (int b = top; b > top - 24; --b) mant = (mant << 1) | ((dg[b / 32] >> (b % 32)) & 1u);
    int rnd = (int)((dg[(top - 24) / 32] >> ((top - 24) % 32)) & 1u);
    int sticky = 0;
    for (int b = top - 25; b >= 0 && !sticky; --b) sticky = (int)((dg[b / 32] >> (b % 32)) & 1u);
    if (rnd && (sticky || (mant & 1u))) {
        ++mant;
        if (mant == (1u << 24)) { mant >>= 1; ++top; }
    }
    if (top - 149 > 127) return INFINITY;
    return ldexpf((float)mant, top - 23 - 149);
}

/* Reverse Cuthill-McKee order of the merged graph (ea[e] < eb[e], m
 * edges): a storage layout offered beside the degree order (the paper takes
 * its graphs as given and discusses no layout; this is the classic
 * bandwidth-reducing one).  Readings: the connected components are taken
 * in increasing order of their smallest id (an isolated vertex is a
 * component of its own); each is searched breadth first from its vertex of
 * least degree (ties: the smallest id); when a vertex leaves the queue, its
 * not yet queued neighbours join it in increasing (degree, id) order; the
 * order of all components, concatenated, is reversed: the vertex at place q
 * gets the id n - 1 - q.                                                   */
typedef struct { int64_t deg, id; } orc_dv;

static int orc_cmp_dv(const void *x, const void *y)
{
    const orc_dv *p = (const orc_dv *)x, *q = (const orc_dv *)y;
    if (p->deg != q->deg) return p->deg < q->deg ? -1 : 1;     /* increasing degree */
    return (p->id > q->id) - (p->id < q->id);
}

static void orc_rcm(int64_t n, int64_t m, const int64_t *ea, const int64_t *eb, int64_t *new_of)
{
    size_t nn = (size_t)(n > 0 ? n : 1), mm = (size_t)(m > 0 ? 2 * m : 1);
    int64_t *deg = (int64_t *)calloc(nn, sizeof(int64_t));
    int64_t *ptr = (int64_t *)calloc(nn + 1, sizeof(int64_t));
    int64_t *adj = (int64_t *)malloc(sizeof(int64_t) * mm);
    int64_t *at = (int64_t *)malloc(sizeof(int64_t) * nn);
    for (int64_t e = 0; e < m; ++e) { deg[ea[e]]++; deg[eb[e]]++; }
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + deg[i];
    for (int64_t i = 0; i < n; ++i) at[i] = ptr[i];
    for (int64_t e = 0; e < m; ++e) { adj[at[ea[e]]++] = eb[e]; adj[at[eb[e]]++] = ea[e]; }
    /* components in order of their smallest id, each with its start vertex */
    int64_t *comp = (int64_t *)malloc(sizeof(int64_t) * nn);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * nn);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * nn);
    for (int64_t i = 0; i < n; ++i) comp[i] = -1;
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (comp[i] >= 0) continue;
        int64_t head = 0, tail = 0, best = i;
        comp[i] = nc;
        queue[tail++] = i;
        while (head < tail) {
            int64_t x = queue[head++];
            if (deg[x] < deg[best] || (deg[x] == deg[best] && x < best)) best = x;
            for (int64_t p = ptr[x]; p < ptr[x + 1]; ++p)
                if (comp[adj[p]] < 0) { comp[adj[p]] = nc; queue[tail++] = adj[p]; }
        }
        start[nc++] = best;
    }
    /* Cuthill-McKee: breadth first from each start, neighbours by (degree, id) */
    char *queued = (char *)calloc(nn, 1);
    orc_dv *nb = (orc_dv *)malloc(sizeof(orc_dv) * nn);
    int64_t place = 0;
    for (int64_t c = 0; c < nc; ++c) {
        int64_t head = place, tail = place;
        queue[tail++] = start[c];
        queued[start[c]] = 1;
        while (head < tail) {
            int64_t x = queue[head++];
            int64_t k = 0;
            for (int64_t p = ptr[x]; p < ptr[x + 1]; ++p) {
                int64_t y = adj[p];
                if (!queued[y]) { queued[y] = 1; nb[k].deg = deg[y]; nb[k].id = y; ++k; }
            }
            qsort(nb, (size_t)k, sizeof(orc_dv), orc_cmp_dv);
            for (int64_t j = 0; j < k; ++j) queue[tail++] = nb[j].id;
        }
        place = tail;
    }
    for (int64_t q = 0; q < n; ++q) new_of[queue[q]] = n - 1 - q;
    free(deg); free(ptr); free(adj); free(at); free(comp); free(start); free(queue); free(queued); free(nb);
}

int64_t orc_ingest(int64_t n, int64_t m_in, const int32_t *u, const int32_t *v, const float *w,
                   const int32_t *orig_in, int32_t order, int64_t *row_ptr, int32_t *col, float *w_out,
                   int32_t *eid, int32_t *orig_out, int64_t *n_dropped)
{
    for (int64_t q = 0; q < m_in; ++q)
        if (u[q] < 0 || u[q] >= n || v[q] < 0 || v[q] >= n) return -1;
    if (w)
        for (int64_t q = 0; q < m_in; ++q)
            if (!(w[q] > 0.0f && w[q] <= FLT_MAX)) return -2;      /* the graph model: finite w > 0 */
    orc_pair *pr = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(m_in > 0 ? m_in : 1));
    int64_t k = 0;
    for (int64_t q = 0; q < m_in; ++q) {
        if (u[q] == v[q]) continue;                         /* self-loop */
        pr[k].a = u[q] < v[q] ? u[q] : v[q];
        pr[k].b = u[q] < v[q] ? v[q] : u[q];
        pr[k].idx = q;
        ++k;
    }
    qsort(pr, (size_t)k, sizeof(orc_pair), orc_cmp_pair);
    /* merge repeated pairs: one edge, weight the exact sum of the listed
     * weights rounded once to single precision */
    int64_t *ea = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
    int64_t *eb = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
    float *ew = (float *)malloc(sizeof(float) * (size_t)(k > 0 ? k : 1));
    float *run = (float *)malloc(sizeof(float) * (size_t)(k > 0 ? k : 1));
    int64_t m = 0;
    for (int64_t q = 0; q < k;) {
        int64_t r = q;
        while (r < k && pr[r].a == pr[q].a && pr[r].b == pr[q].b) {
            if (w) run[r - q] = w[pr[r].idx];
            ++r;
        }
        ea[m] = pr[q].a;
        eb[m] = pr[q].b;
        ew[m] = w ? orc_exact_sum_f32(run, r - q) : 0.0f;
        ++m;
        q = r;
    }
    free(run);
    free(pr);
    /* vertex storage order */
    int64_t *new_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) new_of[i] = i;
    if ((order == 1 || order == 2) && n > 0) {
        if (order == 1) {
            orc_vdeg *vd = (orc_vdeg *)malloc(sizeof(orc_vdeg) * (size_t)n);
            for (int64_t i = 0; i < n; ++i) { vd[i].deg = 0; vd[i].id = i; }
            for (int64_t e = 0; e < m; ++e) { vd[ea[e]].deg++; vd[eb[e]].deg++; }
            qsort(vd, (size_t)n, sizeof(orc_vdeg), orc_cmp_vdeg);
            for (int64_t r = 0; r < n; ++r) new_of[vd[r].id] = r;
            free(vd);
        } else {
            orc_rcm(n, m, ea, eb, new_of);
        }
        /* relabel, then number the edges again in (smaller, larger) order */
        orc_pair *rp = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(m > 0 ? m : 1));
        for (int64_t e = 0; e < m; ++e) {
            int64_t x = new_of[ea[e]], y = new_of[eb[e]];
            rp[e].a = x < y ? x : y;
            rp[e].b = x < y ? y : x;
            rp[e].idx = e;
        }
        qsort(rp, (size_t)m, sizeof(orc_pair), orc_cmp_pair);
        float *ew2 = (float *)malloc(sizeof(float) * (size_t)(m > 0 ? m : 1));
        for (int64_t e = 0; e < m; ++e) {
            ew2[e] = ew[rp[e].idx];
            ea[e] = rp[e].a;
            eb[e] = rp[e].b;
        }
        free(ew);
        ew = ew2;
        free(rp);
    }
    for (int64_t i = 0; i < n; ++i) {
        int32_t id = orig_in ? orig_in[i] : (int32_t)i;
        orig_out[new_of[i]] = id;
    }
    free(new_of);
    /* both entries of every edge, sorted by (row, col) */
    orc_entry *en = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)(2 * m > 0 ? 2 * m : 1));
    for (int64_t e = 0; e < m; ++e) {
        en[2 * e].row = ea[e]; en[2 * e].col = eb[e]; en[2 * e].e = e;
        en[2 * e + 1].row = eb[e]; en[2 * e + 1].col = ea[e]; en[2 * e + 1].e = e;
    }
    qsort(en, (size_t)(2 * m), sizeof(orc_entry), orc_cmp_entry);
    for (int64_t i = 0; i <= n; ++i) row_ptr[i] = 0;
    for (int64_t p = 0; p < 2 * m; ++p) row_ptr[en[p].row + 1]++;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    for (int64_t p = 0; p < 2 * m; ++p) {
        col[p] = (int32_t)en[p].col;
        eid[p] = (int32_t)en[p].e;
        if (w && w_out) w_out[p] = ew[en[p].e];
    }
    free(en); free(ea); free(eb); free(ew);
    if (n_dropped) *n_dropped = m_in - m;
    return m;
}

/* ------------------------------------------------------------------------ */
/* Properties of a graph and of its sparsified subgraph (Preliminaries).     */

/* G_s = (V, {e : keep[e]}): the kept entries of every row, in order; the
 * subgraph's edge ids renumber the kept edges in increasing original id;
 * orig_edge[p] is the original id of entry p.  Returns m_s.               */
int64_t orc_subgraph(int64_t n, const int64_t *row_ptr, const int32_t *col, const float *w,
                     const int32_t *eid, int64_t m, const uint8_t *keep, int64_t *sub_row_ptr,
                     int32_t *sub_col, float *sub_w, int32_t *sub_eid, int32_t *orig_edge)
{
    int64_t *new_id = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t ms = 0;
    for (int64_t e = 0; e < m; ++e) new_id[e] = keep[e] ? ms++ : -1;
    int64_t q = 0;
    sub_row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (!keep[eid[p]]) continue;
            sub_col[q] = col[p];
            if (w && sub_w) sub_w[q] = w[p];
            sub_eid[q] = (int32_t)new_id[eid[p]];
            if (orig_edge) orig_edge[q] = eid[p];
            ++q;
        }
        sub_row_ptr[i + 1] = q;
    }
    free(new_id);
    return ms;
}

/* lambda_i: triangles vertex i belongs to, by testing every pair of its
 * neighbours for adjacency (rows are sorted: bsearch).                      */
static int orc_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

void orc_triangles(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t *lambda)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t t = 0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            for (int64_t q = p + 1; q < row_ptr[i + 1]; ++q) {
                int32_t a = col[p], b = col[q];
                int64_t lo = row_ptr[a], len = row_ptr[a + 1] - lo;
                if (len > 0 && bsearch(&b, col + lo, (size_t)len, sizeof(int32_t), orc_cmp_i32)) ++t;
            }
        lambda[i] = t;
    }
}

/* c_i = lambda_i / tau_i, tau_i = d_i (d_i - 1) / 2 (0 where d_i <= 1), and
 * C_G = the mean of c_i over V' = {i : d_i > 1} (Eq. cc; 0 when V' is
 * empty).  Returns C_G.                                                     */
double orc_clustering(int64_t n, const int64_t *row_ptr, const int64_t *lambda, double *c)
{
    double sum = 0.0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t d = row_ptr[i + 1] - row_ptr[i];
        c[i] = 0.0;
        if (d > 1) {
            c[i] = (double)lambda[i] / ((double)d * (double)(d - 1) / 2.0);
            sum += c[i];
            ++cnt;
        }
    }
    return cnt ? sum / (double)cnt : 0.0;
}

/* Connected components by breadth-first search; comp[i] = the smallest
 * vertex id of i's component.  Returns the number of components.            */
int64_t orc_components(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *comp)
{
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) comp[i] = -1;
    int64_t ncomp = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (comp[s] >= 0) continue;
        ++ncomp;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        comp[s] = (int32_t)s;      /* s is the smallest id not yet reached */
        while (head < tail) {
            int64_t i = queue[head++];
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                if (comp[col[p]] < 0) {
                    comp[col[p]] = (int32_t)s;
                    queue[tail++] = col[p];
                }
        }
    }
    free(queue);
    return ncomp;
}

/* Spearman rank correlation (Preliminaries): rho = 1 - 6 sum p_i^2 /
 * (n (n^2 - 1)), p_i = x_i - y_i the difference of the ranks of X_i and
 * Y_i; tied scores share the mean of their ranks.                          */
typedef struct { double v; int64_t i; } orc_score;

static int orc_cmp_score(const void *a, const void *b)
{
    const orc_score *x = (const orc_score *)a, *y = (const orc_score *)b;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return (x->i > y->i) - (x->i < y->i);
}

static void orc_ranks(int64_t n, const double *v, double *rank)
{
    orc_score *s = (orc_score *)malloc(sizeof(orc_score) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { s[i].v = v[i]; s[i].i = i; }
    qsort(s, (size_t)n, sizeof(orc_score), orc_cmp_score);
    for (int64_t a = 0; a < n;) {
        int64_t b = a;
        while (b < n && s[b].v == s[a].v) ++b;
        double r = 0.5 * (double)(a + 1 + b);          /* mean of ranks a+1 .. b */
        for (int64_t q = a; q < b; ++q) rank[s[q].i] = r;
        a = b;
    }
    free(s);
}

double orc_spearman(int64_t n, const double *x, const double *y)
{
    if (n < 2) return 0.0;
    double *rx = (double *)malloc(sizeof(double) * (size_t)n);
    double *ry = (double *)malloc(sizeof(double) * (size_t)n);
    orc_ranks(n, x, rx);
    orc_ranks(n, y, ry);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (rx[i] - ry[i]) * (rx[i] - ry[i]);
    free(rx); free(ry);
    return 1.0 - 6.0 * s / ((double)n * ((double)n * (double)n - 1.0));
}

/* ------------------------------------------------------------------------ */
/* Multilevel sparsification (Algorithm 6, MLSparsify; coarsening of
 * Section 5).  Readings:
 *   - strength of connection delta_ij = 1 / sqrt(rho_ij^2 + eps) (Algorithm
 *     1's return value), from the distances computed at that level;
 *   - i and j are strongly coupled when delta_ij >= theta * smax_i or
 *     delta_ij >= theta * smax_j, smax_i the largest strength at i;
 *   - seeds ("traversal of F, moving to C the nodes not strongly coupled to
 *     those already in C"): vertices in decreasing degree, ties in the
 *     pseudo-random order of fmix32(orig_id) (MurmurHash3's finalizer, a
 *     bijection), then smaller orig_id; a vertex becomes a seed when none of
 *     its strong neighbours is a seed yet;
 *   - restriction P (Eq. P): a seed is its own aggregate; any other vertex
 *     joins the seed neighbour of largest delta_ij (the normalising sum is
 *     the same for every j), ties by smaller orig_id; aggregates are
 *     numbered by their seeds' ids;
 *   - Galerkin coarse graph P^T L P: one coarse edge per pair of aggregates
 *     joined by fine edges, weight the sum of theirs (unit weights count
 *     edges); coarse vertices are named by their seeds' orig_id;
 *   - coarsening stops at n <= n_min, at level levels - 1, or when it would
 *     keep more than 90% of the vertices; that level is the coarsest;
 *   - level l uses graph id graph_id + l for its test vectors and its bin
 *     order;
 *   - the vector of per-level ratios (Section 6, implementation paragraph)
 *     lists the levels from the coarsest one reached: with D the index of
 *     the coarsest level, level l takes entry D - l.  A negative entry means
 *     no SparsifyB at that level (it keeps what it inherits; the coarsest
 *     level then keeps all its edges).  Otherwise the entry is SparsifyB's
 *     exponent e, or, with `fit`, the fraction of the level's edges that
 *     SparsifyB keeps, e fitted by the bisection of Section 6.2;
 *   - level-span (same paragraph): the D + 1 levels split into three
 *     segments (coarsest, middle, finest), segment s holding entries
 *     floor(s (D+1) / 3) .. floor((s+1) (D+1) / 3) - 1; the first `span`
 *     entries of the chosen segment take the value, all others -1;
 *   - uncoarsening: a fine edge between two aggregates keeps the state of
 *     their coarse edge, an edge inside an aggregate is kept; distances are
 *     recomputed on the fine graph less the dropped edges and SparsifyB
 *     chooses among its edges.                                               */

static double orc_strength_of(double rho, double eps)
{
    double t = rho * rho;
    t = t + eps;
    return 1.0 / sqrt(t);
}

typedef struct { int64_t deg; uint32_t hash; int32_t key; int64_t i; } orc_vprio;

static int orc_cmp_vprio(const void *a, const void *b)
{
    const orc_vprio *x = (const orc_vprio *)a, *y = (const orc_vprio *)b;
    if (x->deg != y->deg) return x->deg > y->deg ? -1 : 1;     /* larger degree first */
    if (x->hash != y->hash) return x->hash < y->hash ? -1 : 1; /* then the hashed name */
    return (x->key > y->key) - (x->key < y->key);
}

void orc_ml_seeds(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *eid,
                  const int32_t *orig_id, const double *rho, double eps, double theta, uint8_t *is_seed)
{
    double *smax = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        double mx = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            double d = orc_strength_of(rho[eid[p]], eps);
            if (d > mx) mx = d;
        }
        smax[i] = mx;
        is_seed[i] = 0;
    }
    orc_vprio *order = (orc_vprio *)malloc(sizeof(orc_vprio) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        order[i].deg = row_ptr[i + 1] - row_ptr[i];
        order[i].key = orig_id ? orig_id[i] : (int32_t)i;
        order[i].hash = orc_fmix32((uint32_t)order[i].key);
        order[i].i = i;
    }
    qsort(order, (size_t)n, sizeof(orc_vprio), orc_cmp_vprio);
    for (int64_t r = 0; r < n; ++r) {
        int64_t i = order[r].i;
        int coupled = 0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1] && !coupled; ++p) {
            int32_t j = col[p];
            if (!is_seed[j]) continue;
            double d = orc_strength_of(rho[eid[p]], eps);
            if (d >= theta * smax[i] || d >= theta * smax[j]) coupled = 1;
        }
        if (!coupled) is_seed[i] = 1;
    }
    free(order);
    free(smax);
}

/* Aggregate of every vertex under P; returns the number of aggregates. */
int64_t orc_ml_aggregates(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *eid,
                          const int32_t *orig_id, const double *rho, double eps, const uint8_t *is_seed,
                          int32_t *agg)
{
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) rank[i] = is_seed[i] ? nc++ : -1;
    for (int64_t i = 0; i < n; ++i) {
        if (is_seed[i]) { agg[i] = (int32_t)rank[i]; continue; }
        int64_t best = -1;
        double bd = -1.0;
        int32_t bk = 0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int32_t j = col[p];
            if (!is_seed[j]) continue;
            double d = orc_strength_of(rho[eid[p]], eps);
            int32_t key = orig_id ? orig_id[j] : j;
            if (best < 0 || d > bd || (d == bd && key < bk)) { best = j; bd = d; bk = key; }
        }
        agg[i] = best >= 0 ? (int32_t)rank[best] : -1;     /* -1: no seed neighbour (cannot happen) */
    }
    free(rank);
    return nc;
}

typedef struct {
    int32_t R, k, levels;
    double omega, eps, theta;
    int64_t n_min;
    uint64_t seed, graph_id, bin_seed;
    const double *e;             /* [levels], coarsest level first */
    int32_t fit, span, segment;
    double span_value;
} orc_ml_opts;

/* The level-span vector over n_levels levels, coarsest first. */
void orc_ml_level_span(int32_t n_levels, int32_t span, int32_t segment, double value, double *out)
{
    int32_t lo = segment * n_levels / 3, hi = (segment + 1) * n_levels / 3;
    for (int32_t t = 0; t < n_levels; ++t) out[t] = (t >= lo && t < hi && t - lo < span) ? value : -1.0;
}

/* The ratio-vector entry of level l when the coarsest level is D. */
static double orc_ml_entry(const orc_ml_opts *o, int32_t D, int32_t l)
{
    if (o->span > 0) {
        double *v = (double *)malloc(sizeof(double) * (size_t)(D + 1));
        orc_ml_level_span(D + 1, o->span, o->segment, o->span_value, v);
        double x = v[D - l];
        free(v);
        return x;
    }
    return o->e[D - l];
}

/* SparsifyB of one level with its entry x (x < 0: keep everything). */
static void orc_ml_select(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *eid,
                          const int32_t *orig_id, int64_t m, const double *rho, const orc_ml_opts *o,
                          uint64_t gid, double x, uint8_t *keep)
{
    if (x < 0.0) { memset(keep, 1, (size_t)m); return; }
    if (o->fit) orc_fit_exponent_binned(n, row_ptr, col, eid, orig_id, m, rho, o->bin_seed, gid, x, keep, NULL);
    else orc_sparsify_binned(n, row_ptr, col, eid, orig_id, m, rho, o->bin_seed, gid, x, keep);
}

/* keep[m] of graph (n, row_ptr, col, w, eid, orig_id) at level l. */
static void orc_ml_level(int64_t n, const int64_t *row_ptr, const int32_t *col, const float *w,
                         const int32_t *eid, const int32_t *orig_id, int64_t m, const orc_ml_opts *o, int32_t l,
                         uint8_t *keep, int32_t *depth)
{
    uint64_t gid = o->graph_id + (uint64_t)l;
    double *rho = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    orc_algebraic_distance(n, row_ptr, col, w, eid, orig_id, m, o->R, o->k, o->omega, o->seed, gid, NULL, rho,
                           NULL, NULL, NULL);
    if (*depth < l) *depth = l;
    int coarsest = (n <= o->n_min) || (l + 1 >= o->levels) || m == 0;
    uint8_t *is_seed = NULL;
    int32_t *agg = NULL;
    int64_t nc = 0;
    if (!coarsest) {
        is_seed = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
        agg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        orc_ml_seeds(n, row_ptr, col, eid, orig_id, rho, o->eps, o->theta, is_seed);
        nc = orc_ml_aggregates(n, row_ptr, col, eid, orig_id, rho, o->eps, is_seed, agg);
        if ((double)nc > 0.9 * (double)n) coarsest = 1;
    }
    if (coarsest) {
        orc_ml_select(n, row_ptr, col, eid, orig_id, m, rho, o, gid, orc_ml_entry(o, l, l), keep);
        free(rho); free(is_seed); free(agg);
        return;
    }
    /* coarse graph: the fine edges' aggregate pairs, repeats merged with summed weights */
    int32_t *cu = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int32_t *cv = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    float *cw = (float *)malloc(sizeof(float) * (size_t)m);
    int32_t *corig = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            if (col[p] > i) {
                int32_t e = eid[p];
                cu[e] = agg[i];
                cv[e] = agg[col[p]];
                cw[e] = w ? w[p] : 1.0f;
            }
    for (int64_t i = 0; i < n; ++i)
        if (is_seed[i]) corig[agg[i]] = orig_id ? orig_id[i] : (int32_t)i;
    int64_t *crp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
    int32_t *ccol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m));
    float *cwo = (float *)malloc(sizeof(float) * (size_t)(2 * m));
    int32_t *ceid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m));
    int32_t *corig2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    int64_t cdrop = 0;
    int64_t mc = orc_ingest(nc, m, cu, cv, cw, corig, 0, crp, ccol, cwo, ceid, corig2, &cdrop);
    uint8_t *ckeep = (uint8_t *)malloc((size_t)(mc > 0 ? mc : 1));
    orc_ml_level(nc, crp, ccol, cwo, ceid, corig2, mc, o, l + 1, ckeep, depth);
    /* inherit: an edge between aggregates keeps its coarse edge's state */
    uint8_t *inh = (uint8_t *)malloc((size_t)m);
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = cu[e], b = cv[e];
        if (a == b) { inh[e] = 1; continue; }
        int32_t x = a < b ? a : b, y = a < b ? b : a;
        int64_t lo = crp[x], hi = crp[x + 1];
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (ccol[mid] < y) lo = mid + 1; else hi = mid;
        }
        inh[e] = ckeep[ceid[lo]];
    }
    /* the fine graph less the dropped edges: distances again, SparsifyB on it */
    double x = orc_ml_entry(o, *depth, l);
    if (x < 0.0) {
        memcpy(keep, inh, (size_t)m);
        free(rho); free(is_seed); free(agg); free(cu); free(cv); free(cw); free(corig); free(crp); free(ccol);
        free(cwo); free(ceid); free(corig2); free(ckeep); free(inh);
        return;
    }
    int64_t *srp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *scol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m));
    float *sw = w ? (float *)malloc(sizeof(float) * (size_t)(2 * m)) : NULL;
    int32_t *seid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m));
    int32_t *soe = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m));
    int64_t ms = orc_subgraph(n, row_ptr, col, w, eid, m, inh, srp, scol, sw, seid, soe);
    double *srho = (double *)malloc(sizeof(double) * (size_t)(ms > 0 ? ms : 1));
    uint8_t *skeep = (uint8_t *)malloc((size_t)(ms > 0 ? ms : 1));
    orc_algebraic_distance(n, srp, scol, sw, seid, orig_id, ms, o->R, o->k, o->omega, o->seed, gid, NULL, srho,
                           NULL, NULL, NULL);
    if (ms > 0) orc_ml_select(n, srp, scol, seid, orig_id, ms, srho, o, gid, x, skeep);
    memset(keep, 0, (size_t)m);
    for (int64_t p = 0; p < 2 * ms; ++p)
        if (skeep[seid[p]]) keep[soe[p]] = 1;
    free(rho); free(is_seed); free(agg); free(cu); free(cv); free(cw); free(corig); free(crp); free(ccol);
    free(cwo); free(ceid); free(corig2); free(ckeep); free(inh); free(srp); free(scol); free(sw); free(seid);
    free(soe); free(srho); free(skeep);
}

/* Algorithm 6: keep[m] of the finest graph; returns the kept count, and
 * the index of the coarsest level reached in *depth.  e: [levels] ratios,
 * coarsest level first (ignored when span > 0).                            */
int64_t orc_ml_sparsify(int64_t n, const int64_t *row_ptr, const int32_t *col, const float *w,
                        const int32_t *eid, const int32_t *orig_id, int64_t m, int32_t R, int32_t k,
                        double omega, uint64_t seed, uint64_t graph_id, int32_t levels, int64_t n_min,
                        const double *e, int32_t fit, int32_t span, int32_t segment, double span_value,
                        double eps, double theta, uint64_t bin_seed, uint8_t *keep, int32_t *depth)
{
    orc_ml_opts o = {R, k, levels, omega, eps, theta, n_min, seed, graph_id, bin_seed, e, fit, span, segment,
                     span_value};
    int32_t dd = 0;
    if (m > 0) orc_ml_level(n, row_ptr, col, w, eid, orig_id, m, &o, 0, keep, &dd);
    if (depth) *depth = dd;
    int64_t kept = 0;
    for (int64_t q = 0; q < m; ++q) kept += keep[q];
    return kept;
}

/* ------------------------------------------------------------------------ */
/* Reverse-mode derivative of L = sum_e c_e rho_e with respect to the edge
 * weights w_e (w_ij = w_ji = w_e), taken through the k sweeps, the rescale
 * (its min and max as functions of x^(k)) and the distance.  Written by the
 * chain rule from the forward steps above; one vector at a time, storing
 * x^(0..k).  Start vectors do not depend on w.
 *   c      : [m] weights of the loss.
 *   grad_w : [m] output.                                                    */
void orc_grad_weights(int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const float *w, const int32_t *eid, const int32_t *orig_id,
                      int64_t m, int32_t R, int32_t k, double omega, uint64_t seed,
                      uint64_t graph_id, const double *x0, const double *c,
                      double *grad_w)
{
    double *rho = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *xhat = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n * R : 1));
    double *minmax = (double *)malloc(sizeof(double) * (size_t)(2 * R));
    orc_algebraic_distance(n, row_ptr, col, w, eid, orig_id, m, R, k, omega, seed,
                           graph_id, x0, rho, NULL, xhat, minmax);
    double *s = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) acc += w ? (double)w[p] : 1.0;
        s[i] = acc;
    }
    int64_t nnz = row_ptr[n];
    double *g = (double *)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(double)); /* per directed entry */
    double *trace = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(k + 1));
    double *lam = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *lam_prev = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t r = 0; r < R; ++r) {
        /* forward again for this vector, keeping every sweep */
        for (int64_t i = 0; i < n; ++i)
            trace[i] = x0 ? x0[i * R + r]
                          : orc_start_value(seed, graph_id, orig_id ? orig_id[i] : (int32_t)i, r);
        double *xk = trace + (size_t)k * (size_t)n;
        {
            double *tmp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
            memcpy(tmp, trace, sizeof(double) * (size_t)n);
            orc_relax_vector(n, row_ptr, col, w, k, omega, tmp, trace);
            free(tmp);
        }
        double mn = minmax[r], mx = minmax[R + r];
        for (int64_t i = 0; i < n; ++i) lam[i] = 0.0;
        if (!(mx > mn)) continue;          /* xhat == 0: no dependence on w */
        double D = mx - mn;
        /* d rho_e / d xhat_i = (xhat_i - xhat_j) / rho_e  (0 when rho_e = 0) */
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                int32_t j = col[p];
                double re = rho[eid[p]];
                if (re > 0.0) lam[i] += c[eid[p]] * (xhat[i * R + r] - xhat[(int64_t)j * R + r]) / re;
            }
        /* rescale: xhat_i = (x_i - mn)/D - 1/2 over non-isolated vertices */
        int64_t imin = -1, imax = -1;
        for (int64_t i = 0; i < n; ++i) {
            if (row_ptr[i + 1] == row_ptr[i]) continue;
            if (imin < 0 || xk[i] < xk[imin]) imin = i;
            if (imax < 0 || xk[i] > xk[imax]) imax = i;
        }
        double gmin = 0.0, gmax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (row_ptr[i + 1] == row_ptr[i]) continue;
            gmin += lam[i] * (xk[i] - mx) / (D * D);
            gmax += -lam[i] * (xk[i] - mn) / (D * D);
        }
        for (int64_t i = 0; i < n; ++i)
            lam[i] = (row_ptr[i + 1] == row_ptr[i]) ? 0.0 : lam[i] / D;
        lam[imin] += gmin;
        lam[imax] += gmax;
        /* sweeps, last to first */
        for (int32_t t = k; t >= 1; --t) {
            const double *xp = trace + (size_t)(t - 1) * (size_t)n;
            for (int64_t i = 0; i < n; ++i) {
                int64_t beg = row_ptr[i], end = row_ptr[i + 1];
                if (beg == end) continue;
                double y = 0.0;
                for (int64_t p = beg; p < end; ++p) y += (w ? (double)w[p] : 1.0) * xp[col[p]];
                y /= s[i];
                for (int64_t p = beg; p < end; ++p)
                    g[p] += omega * lam[i] * (xp[col[p]] - y) / s[i];
            }
            for (int64_t i = 0; i < n; ++i) {
                int64_t beg = row_ptr[i], end = row_ptr[i + 1];
                if (beg == end) { lam_prev[i] = lam[i]; continue; }
                double acc = 0.0;
                for (int64_t p = beg; p < end; ++p) {
                    int32_t j = col[p];
                    acc += (w ? (double)w[p] : 1.0) * lam[j] / s[j];
                }
                lam_prev[i] = (1.0 - omega) * lam[i] + omega * acc;
            }
            memcpy(lam, lam_prev, sizeof(double) * (size_t)n);
        }
    }
    for (int64_t e = 0; e < m; ++e) grad_w[e] = 0.0;
    for (int64_t p = 0; p < nnz; ++p) grad_w[eid[p]] += g[p];
    free(rho); free(xhat); free(minmax); free(s); free(g); free(trace); free(lam); free(lam_prev);
}
