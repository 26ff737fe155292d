// ad_batch.hip -- many independent graphs in one captured launch sequence.
//
// The graphs are packed once into a block-diagonal CSR (column and edge ids
// offset per graph, orig_id kept graph-local).  Every kernel of the path then
// covers all graphs in one launch: per-graph centring and min/max chunks and
// launch-plan tiles start at each graph's first row, graph g draws its start
// vectors with key word graph_id + g and rescales with its own min/max, and
// ranking is row-local.  Each graph's distances and kept edges therefore equal
// those of ad_relax + ad_edge_dist + ad_sparsify on that graph alone (same
// options), bit for bit.  The whole sequence is captured once into a HIP
// graph and replayed by ad_batch_run.
#include "ad_internal.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace ad {

constexpr int TB = 256;

__global__ void k_pack_rowptr(int64_t n, const int64_t *__restrict__ src, int64_t nnz_base,
                              int64_t *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] + nnz_base;
}

__global__ void k_pack_i32(int64_t count, const int32_t *__restrict__ src, int32_t base, int32_t *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src ? src[i] + base : (int32_t)i + base;
}

__global__ void k_pack_f32(int64_t count, const float *__restrict__ src, float *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src ? src[i] : 1.0f;
}

__global__ void k_fill_graph(int64_t count, int32_t g, int32_t *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = g;
}

// n_kept[g] = sum of keep over graph g's edges.  A wave's 64 consecutive
// edges mostly lie in one graph: lane 0 finds it (binary search over
// edge_off) and the wave sums into it; a wave that straddles graphs falls
// back to a search per lane.
__global__ __launch_bounds__(TB) void k_count_per_graph(int64_t m, const uint8_t *__restrict__ keep,
                                                        const int64_t *__restrict__ edge_off, int G,
                                                        unsigned long long *__restrict__ counts) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t m_pad = ceil_div_dev(m, stride) * stride;
    const int lane = threadIdx.x & (WAVE - 1);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m_pad; e += stride) {
        const bool on = e < m;
        const int64_t e_first = e - lane;                 // the wave's first edge (< m when any lane is on)
        int g0 = 0;
        if (lane == 0 && e_first < m) g0 = seg_find(edge_off, G, e_first);
        g0 = __shfl(g0, 0, WAVE);
        unsigned long long c = (on && keep[e]) ? 1ull : 0ull;
        const bool mine = !on || e < edge_off[g0 + 1];
        if (__all(mine)) {
            for (int d = WAVE / 2; d >= 1; d >>= 1) c += __shfl_down(c, d, WAVE);
            if (lane == 0 && c) atomicAdd(&counts[g0], c);
        } else if (c) {
            atomicAdd(&counts[seg_find(edge_off, G, e)], c);
        }
    }
}

__global__ void k_counts_out(int G, const unsigned long long *__restrict__ c, int64_t *__restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < G) out[g] = (int64_t)c[g];
}

}  // namespace ad

using namespace ad;

struct ad_batch {
    int32_t G = 0;
    ad_relax_opts o{};
    ad_orient orient = AD_LOCAL;
    double e = 0.5;
    int64_t N = 0, M = 0;
    int32_t d_max = 0;
    std::vector<int64_t> row_off, edge_off, chunk_off, tile_off;
    // device memory owned by the batch
    std::vector<void *> owned;
    int64_t *row_ptr = nullptr, *d_row_off = nullptr, *d_edge_off = nullptr, *d_chunk_off = nullptr,
            *d_tile_off = nullptr;
    int32_t *col = nullptr, *eid = nullptr, *orig = nullptr, *col_orig = nullptr, *row_graph = nullptr;
    float *w = nullptr;
    void *x = nullptr;                   // FP32, or FP64 with an FP64 tail
    float *rho = nullptr;
    double *minmax = nullptr, *shift = nullptr;
    // connected components of the packed graph (per-component centring)
    ad_components comps{};
    int32_t *comp_of = nullptr, *members = nullptr;
    int64_t *comp_start = nullptr, *chunk_start = nullptr;
    uint8_t *keep = nullptr;
    int64_t *n_kept = nullptr;
    unsigned long long *counts = nullptr;
    int32_t *budget = nullptr;
    void *ws_relax = nullptr, *ws_dist = nullptr, *ws_sel = nullptr;
    size_t ws_relax_bytes = 0, ws_dist_bytes = 0, ws_sel_bytes = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ad_graph packed() const {
        ad_graph g{};
        g.n = N;
        g.m = M;
        g.row_ptr = row_ptr;
        g.col = col;
        g.w = w;
        g.eid = eid;
        g.orig_id = orig;
        g.d_max = d_max;
        g.col_orig = col_orig;
        return g;
    }
    Segs segs() const {
        Segs s;
        s.G = G;
        s.row_off = d_row_off;
        s.chunk_off = d_chunk_off;
        s.tile_off = d_tile_off;
        s.row_graph = row_graph;
        s.nchunks = chunk_off.back();
        s.ntiles = tile_off.back();
        return s;
    }
    template <typename T>
    ad_status alloc(T **p, size_t count) {
        void *q = nullptr;
        hipError_t err = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (err != hipSuccess) return hip_fail(err, "hipMalloc");
        owned.push_back(q);
        *p = (T *)q;
        return AD_OK;
    }
    ~ad_batch() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (cap) hipStreamDestroy(cap);
        for (void *q : owned) hipFree(q);
    }
};

// The whole per-batch sequence on `st`: relax, distances, fixed-e selection,
// per-graph counts.
static ad_status batch_enqueue(ad_batch *b, hipStream_t st) {
    const ad_graph g = b->packed();
    const Segs sg = b->segs();
    ad_status s = relax_segs(&g, &b->o, nullptr, b->x, b->minmax, b->shift, nullptr, b->ws_relax, b->ws_relax_bytes,
                             sg, st);
    if (s != AD_OK) return s;
    s = edge_dist_segs(&g, b->o.R, b->o.fp64_tail > 0 ? AD_F64 : AD_F32, b->x, b->minmax, AD_F32, b->rho,
                       b->ws_dist, b->ws_dist_bytes, sg, st);
    if (s != AD_OK) return s;
    s = sparsify_fixed(&g, AD_F32, b->rho, b->orient, b->budget, b->keep, b->ws_sel, b->ws_sel_bytes, st);
    if (s != AD_OK) return s;
    s = fill_u64(b->counts, 0, b->G, st);
    if (s != AD_OK) return s;
    if (b->M > 0) {
        hipLaunchKernelGGL(k_count_per_graph, dim3((unsigned)std::min<int64_t>(1024, ceil_div(b->M, TB))), dim3(TB),
                           0, st, b->M, b->keep, b->d_edge_off, b->G, b->counts);
        AD_LAUNCH_CHECK("k_count_per_graph");
    }
    hipLaunchKernelGGL(k_counts_out, dim3((unsigned)ceil_div(b->G, TB)), dim3(TB), 0, st, b->G, b->counts, b->n_kept);
    AD_LAUNCH_CHECK("k_counts_out");
    return AD_OK;
}

static ad_status batch_sizes(ad_batch *b) {
    const ad_graph g = b->packed();
    const Segs sg = b->segs();
    b->ws_relax_bytes = relax_segs_workspace(&g, &b->o, sg);
    b->ws_dist_bytes = edge_dist_segs_workspace(&g, sg);
    b->ws_sel_bytes = sparsify_workspace(&g);
    if (!b->ws_relax_bytes || !b->ws_dist_bytes || !b->ws_sel_bytes)
        return fail(AD_ERR_INTERNAL, "workspace sizing failed");
    return AD_OK;
}

extern "C" ad_status ad_batch_create(int32_t G, const ad_graph *graphs, const ad_relax_opts *o,
                                     const ad_batch_opts *bo, ad_batch **out, hipStream_t stream) {
    if (!out) return fail(AD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (G < 1) return fail(AD_ERR_INVALID_ARG, "G must be >= 1");
    if (!graphs || !o || !bo) return fail(AD_ERR_INVALID_ARG, "graphs, opts or batch opts is NULL");
    if (o->R < 1 || o->R > 64 || o->k < 0 || !(o->omega > 0.0 && o->omega <= 1.0))
        return fail(AD_ERR_INVALID_ARG, "bad relaxation options");
    if (o->store != AD_F32) return fail(AD_ERR_UNSUPPORTED, "batches use FP32 storage");
    if (o->ckpt_every != 0) return fail(AD_ERR_UNSUPPORTED, "batches keep no checkpoints");
    if (o->fp64_tail < 0) return fail(AD_ERR_INVALID_ARG, "fp64_tail must be >= 0");
    if (bo->orient != AD_LOCAL && bo->orient != AD_GLOBAL) return fail(AD_ERR_INVALID_ARG, "unknown orientation");
    if (!(bo->e >= 0.0 && bo->e <= 1.0)) return fail(AD_ERR_INVALID_ARG, "e must be in [0, 1]");
    for (int32_t q = 0; q < G; ++q) {
        ad_status s = check_graph_args(&graphs[q]);
        if (s != AD_OK) return s;
    }
    ad_batch *b = new ad_batch();
    b->G = G;
    b->o = *o;
    b->o.comp = nullptr;          // set below to the packed graph's components
    b->orient = bo->orient;
    b->e = bo->e;
    b->row_off.assign(G + 1, 0);
    b->edge_off.assign(G + 1, 0);
    b->chunk_off.assign(G + 1, 0);
    b->tile_off.assign(G + 1, 0);
    bool any_w = false;
    for (int32_t q = 0; q < G; ++q) {
        b->row_off[q + 1] = b->row_off[q] + graphs[q].n;
        b->edge_off[q + 1] = b->edge_off[q] + graphs[q].m;
        b->chunk_off[q + 1] = b->chunk_off[q] + ceil_div(graphs[q].n, CENTRE_ROWS);
        b->tile_off[q + 1] = b->tile_off[q] + ceil_div(graphs[q].n, PLAN_TILE);
        b->d_max = std::max(b->d_max, graphs[q].d_max);
        any_w = any_w || graphs[q].w != nullptr;
    }
    b->N = b->row_off[G];
    b->M = b->edge_off[G];
    if (b->N > 0x7fffffffLL || b->M > 0x7fffffffLL) {
        delete b;
        return fail(AD_ERR_UNSUPPORTED, "packed sizes must fit in int32");
    }
    const int64_t N = b->N, M = b->M, NNZ = 2 * M, R = o->R;
    ad_status s = AD_OK;
#define AD_TRY(x)              \
    do {                       \
        s = (x);               \
        if (s != AD_OK) {      \
            delete b;          \
            return s;          \
        }                      \
    } while (0)
    AD_TRY(b->alloc(&b->row_ptr, N + 1));
    AD_TRY(b->alloc(&b->col, NNZ));
    if (any_w) AD_TRY(b->alloc(&b->w, NNZ));
    AD_TRY(b->alloc(&b->eid, NNZ));
    AD_TRY(b->alloc(&b->orig, N));
    AD_TRY(b->alloc(&b->col_orig, NNZ));
    AD_TRY(b->alloc(&b->row_graph, N));
    AD_TRY(b->alloc(&b->d_row_off, G + 1));
    AD_TRY(b->alloc(&b->d_edge_off, G + 1));
    AD_TRY(b->alloc(&b->d_chunk_off, G + 1));
    AD_TRY(b->alloc(&b->d_tile_off, G + 1));
    AD_TRY(b->alloc((char **)&b->x, N * R * (o->fp64_tail > 0 ? 8 : 4)));
    AD_TRY(b->alloc(&b->rho, M));
    AD_TRY(b->alloc(&b->minmax, (size_t)G * 2 * R));
    AD_TRY(b->alloc(&b->comp_of, N));
    AD_TRY(b->alloc(&b->members, N));
    AD_TRY(b->alloc(&b->comp_start, N + 1));
    AD_TRY(b->alloc(&b->chunk_start, N + 1));
    AD_TRY(b->alloc(&b->keep, M));
    AD_TRY(b->alloc(&b->n_kept, G));
    AD_TRY(b->alloc(&b->counts, G));
    AD_TRY(b->alloc(&b->budget, (size_t)b->d_max + 1));

    // pack the graphs
    for (int32_t q = 0; q < G; ++q) {
        const ad_graph &gq = graphs[q];
        const int64_t nq = gq.n, nnzq = 2 * gq.m;
        const int64_t r0 = b->row_off[q], p0 = 2 * b->edge_off[q];
        hipLaunchKernelGGL(k_pack_rowptr, dim3(grid_for(nq + 1, TB)), dim3(TB), 0, stream, nq, gq.row_ptr, p0,
                           b->row_ptr + r0);
        if (nnzq > 0) {
            hipLaunchKernelGGL(k_pack_i32, dim3(grid_for(nnzq, TB)), dim3(TB), 0, stream, nnzq, gq.col, (int32_t)r0,
                               b->col + p0);
            hipLaunchKernelGGL(k_pack_i32, dim3(grid_for(nnzq, TB)), dim3(TB), 0, stream, nnzq, gq.eid,
                               (int32_t)b->edge_off[q], b->eid + p0);
            if (any_w)
                hipLaunchKernelGGL(k_pack_f32, dim3(grid_for(nnzq, TB)), dim3(TB), 0, stream, nnzq, gq.w, b->w + p0);
        }
        if (nq > 0) {
            hipLaunchKernelGGL(k_pack_i32, dim3(grid_for(nq, TB)), dim3(TB), 0, stream, nq, gq.orig_id, 0,
                               b->orig + r0);
            hipLaunchKernelGGL(k_fill_graph, dim3(grid_for(nq, TB)), dim3(TB), 0, stream, nq, q, b->row_graph + r0);
        }
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) {
            delete b;
            return hip_fail(err, "packing kernels");
        }
    }
    // per-entry neighbour ids in the graph-local numbering
    {
        const ad_graph pg = b->packed();
        ad_graph tmp = pg;
        tmp.col_orig = nullptr;
        AD_TRY(ad_graph_col_orig(&tmp, b->col_orig, stream));
    }
    std::vector<int32_t> budget;
    budget.assign((size_t)b->d_max + 1, 0);
    AD_TRY(ad_budget_table(b->d_max, b->e, budget.data()));
    hipError_t err = hipMemcpyAsync(b->budget, budget.data(), budget.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                    stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(b->d_row_off, b->row_off.data(), (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(b->d_edge_off, b->edge_off.data(), (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                             stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(b->d_chunk_off, b->chunk_off.data(), (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                             stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(b->d_tile_off, b->tile_off.data(), (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                             stream);
    if (err == hipSuccess) err = hipStreamSynchronize(stream);
    if (err != hipSuccess) {
        delete b;
        return hip_fail(err, "batch set-up copies");
    }

    // connected components of the packed graph: the components of its graphs,
    // grouped in the same relative order as each graph's own
    {
        const ad_graph pg = b->packed();
        const size_t cb = ad_components_workspace_size(&pg);
        if (cb == 0) {
            delete b;
            return fail(AD_ERR_INTERNAL, "component workspace size");
        }
        void *cws = nullptr;
        err = hipMalloc(&cws, cb);
        if (err != hipSuccess) {
            delete b;
            return hip_fail(err, "hipMalloc");
        }
        int64_t nc = 0, nch = 0;
        s = ad_components_build(&pg, b->comp_of, b->members, b->comp_start, b->chunk_start, &nc, &nch, cws, cb,
                                stream);
        (void)hipFree(cws);
        if (s != AD_OK) {
            delete b;
            return s;
        }
        b->comps = ad_components{nc, nch, b->comp_of, b->members, b->comp_start, b->chunk_start};
        b->o.comp = &b->comps;
        AD_TRY(b->alloc(&b->shift, (size_t)std::max<int64_t>(1, nc) * R));
    }

    // workspaces do not depend on the launch shape
    AD_TRY(batch_sizes(b));
    AD_TRY(b->alloc((char **)&b->ws_relax, b->ws_relax_bytes));
    AD_TRY(b->alloc((char **)&b->ws_dist, b->ws_dist_bytes));
    AD_TRY(b->alloc((char **)&b->ws_sel, b->ws_sel_bytes));

    // autotune: rows per wave of the sweep (0 = per-tile plan), timed on this batch
    if (bo->autotune) {
        static const int cand[] = {0, 1, 2, 4, 8, 16, 32};
        const int sprw = sweep_shape((int)R, 4, 0, 0).SPRW;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        err = hipEventCreate(&e0);
        if (err == hipSuccess) err = hipEventCreate(&e1);
        if (err != hipSuccess) {
            delete b;
            return hip_fail(err, "hipEventCreate");
        }
        const ad_graph pg = b->packed();
        float best_ms = 1e30f;
        int best = 0;
        TraceSuppress quiet;
        for (int c : cand) {
            if (c > sprw) continue;
            b->o.rows_per_wave = c;
            float ms = 0.f;
            for (int rep = 0; rep < 3 && s == AD_OK; ++rep) {
                hipEventRecord(e0, stream);
                s = relax_segs(&pg, &b->o, nullptr, b->x, b->minmax, b->shift, nullptr, b->ws_relax,
                               b->ws_relax_bytes, b->segs(), stream);
                hipEventRecord(e1, stream);
                if (s != AD_OK) break;
                hipEventSynchronize(e1);
                float t = 0.f;
                hipEventElapsedTime(&t, e0, e1);
                if (rep > 0) ms += t;     // the first run warms the caches
            }
            if (s != AD_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (s != AD_OK) {
            delete b;
            return s;
        }
        b->o.rows_per_wave = best;
    }

    // capture the sequence once
    err = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (err != hipSuccess) {
        delete b;
        return hip_fail(err, "hipStreamCreateWithFlags");
    }
    TraceSuppress quiet;               // no event records inside the captured graph
    err = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) {
        delete b;
        return hip_fail(err, "hipStreamBeginCapture");
    }
    s = batch_enqueue(b, b->cap);
    hipGraph_t graph = nullptr;
    err = hipStreamEndCapture(b->cap, &graph);
    b->graph = graph;
    if (s != AD_OK) {
        delete b;
        return s;
    }
    if (err != hipSuccess) {
        delete b;
        return hip_fail(err, "hipStreamEndCapture");
    }
    err = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        delete b;
        return hip_fail(err, "hipGraphInstantiate");
    }
#undef AD_TRY
    *out = b;
    return AD_OK;
}

extern "C" ad_status ad_batch_run(ad_batch *b, hipStream_t stream) {
    if (!b || !b->exec) return fail(AD_ERR_INVALID_ARG, "batch is NULL");
    hipError_t err = hipGraphLaunch(b->exec, stream);
    if (err != hipSuccess) return hip_fail(err, "hipGraphLaunch");
    return AD_OK;
}

extern "C" ad_status ad_batch_run_uncaptured(ad_batch *b, hipStream_t stream) {
    if (!b) return fail(AD_ERR_INVALID_ARG, "batch is NULL");
    return batch_enqueue(b, stream);
}

extern "C" ad_status ad_batch_info(const ad_batch *b, int64_t *row_off_host, int64_t *edge_off_host,
                                   int32_t *rows_per_wave_host) {
    if (!b) return fail(AD_ERR_INVALID_ARG, "batch is NULL");
    if (row_off_host) std::copy(b->row_off.begin(), b->row_off.end(), row_off_host);
    if (edge_off_host) std::copy(b->edge_off.begin(), b->edge_off.end(), edge_off_host);
    if (rows_per_wave_host) *rows_per_wave_host = b->o.rows_per_wave;
    return AD_OK;
}

extern "C" ad_status ad_batch_results(const ad_batch *b, const float **rho, const uint8_t **keep,
                                      const int64_t **n_kept, const double **minmax) {
    if (!b) return fail(AD_ERR_INVALID_ARG, "batch is NULL");
    if (rho) *rho = b->rho;
    if (keep) *keep = b->keep;
    if (n_kept) *n_kept = b->n_kept;
    if (minmax) *minmax = b->minmax;
    return AD_OK;
}

extern "C" ad_status ad_batch_copy_results(const ad_batch *b, float *rho, uint8_t *keep, int64_t *n_kept,
                                           double *minmax, hipStream_t stream) {
    if (!b) return fail(AD_ERR_INVALID_ARG, "batch is NULL");
    const int64_t R = b->o.R;
    if (rho && b->M) AD_HIP(hipMemcpyAsync(rho, b->rho, b->M * sizeof(float), hipMemcpyDeviceToDevice, stream));
    if (keep && b->M) AD_HIP(hipMemcpyAsync(keep, b->keep, b->M, hipMemcpyDeviceToDevice, stream));
    if (n_kept) AD_HIP(hipMemcpyAsync(n_kept, b->n_kept, b->G * sizeof(int64_t), hipMemcpyDeviceToDevice, stream));
    if (minmax)
        AD_HIP(hipMemcpyAsync(minmax, b->minmax, b->G * 2 * R * sizeof(double), hipMemcpyDeviceToDevice, stream));
    return AD_OK;
}

extern "C" void ad_batch_destroy(ad_batch *b) { delete b; }
