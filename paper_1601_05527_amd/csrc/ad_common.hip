// ad_common.hip -- error state, status strings, fills, row collection and
// graph validation for libad.
#include "ad_internal.h"

#include <algorithm>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <vector>

namespace ad {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

ad_status fail(ad_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

ad_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return AD_ERR_HIP;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

ad_status fill_u64(unsigned long long *p, unsigned long long v, int64_t count, hipStream_t s) {
    if (count <= 0) return AD_OK;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, 256)), dim3(256), 0, s, p, v, count);
    AD_LAUNCH_CHECK("k_fill_u64");
    return AD_OK;
}
ad_status fill_u8(uint8_t *p, uint8_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return AD_OK;
    // 16 bytes per thread when aligned
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(count, 256)), dim3(256), 0, s, p, v, count);
    AD_LAUNCH_CHECK("k_fill_u8");
    return AD_OK;
}
// ----------------------------------------------------------- plan scans --

constexpr int SCAN_TB = 256;
constexpr int SCAN_EPT = SCAN_PER_BLOCK / SCAN_TB;     // elements per thread

// Block-wide exclusive scan of one value per thread (wave scans, then the
// wave totals); returns the thread's exclusive prefix, *block_total the sum.
template <typename T>
__device__ T block_exclusive(T x, T *wsum, T *block_total) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    T inc = x;
    for (int o = 1; o < WAVE; o <<= 1) {
        const T y = __shfl_up(inc, o, WAVE);
        if (lane >= o) inc += y;
    }
    if (lane == WAVE - 1) wsum[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < SCAN_TB / WAVE; ++i) {
            const T t = wsum[i];
            wsum[i] = run;
            run += t;
        }
        *block_total = run;
    }
    __syncthreads();
    return wsum[w] + inc - x;
}

__global__ __launch_bounds__(SCAN_TB) void k_scan_partials(int64_t count, const unsigned int *__restrict__ v,
                                                           const unsigned long long *__restrict__ w,
                                                           unsigned int *__restrict__ blk_v,
                                                           unsigned long long *__restrict__ blk_w) {
    __shared__ unsigned int sv[SCAN_TB / WAVE];
    __shared__ unsigned long long sw[SCAN_TB / WAVE];
    __shared__ unsigned int tv;
    __shared__ unsigned long long tw;
    const int64_t base = (int64_t)blockIdx.x * SCAN_PER_BLOCK + (int64_t)threadIdx.x * SCAN_EPT;
    unsigned int a = 0;
    unsigned long long b = 0;
    for (int q = 0; q < SCAN_EPT; ++q) {
        const int64_t i = base + q;
        if (i < count) {
            a += v[i];
            if (w) b += w[i];
        }
    }
    block_exclusive(a, sv, &tv);
    if (w) block_exclusive(b, sw, &tw);
    if (threadIdx.x == 0) {
        blk_v[blockIdx.x] = tv;
        blk_w[blockIdx.x] = w ? tw : 0ull;
    }
}

// One block: exclusive scan of the block sums (thread-contiguous chunks).
__global__ __launch_bounds__(SCAN_TB) void k_scan_blocks(int64_t nblk, unsigned int *__restrict__ blk_v,
                                                         unsigned long long *__restrict__ blk_w,
                                                         unsigned int *__restrict__ total,
                                                         unsigned long long *__restrict__ total_w,
                                                         unsigned int *__restrict__ splits) {
    __shared__ unsigned int sv[SCAN_TB / WAVE];
    __shared__ unsigned long long sw[SCAN_TB / WAVE];
    __shared__ unsigned int tv;
    __shared__ unsigned long long tw;
    const int64_t per = ceil_div_dev(nblk, SCAN_TB);
    const int64_t a0 = threadIdx.x * per, a1 = min(nblk, a0 + per);
    unsigned int a = 0;
    unsigned long long b = 0;
    for (int64_t i = a0; i < a1; ++i) {
        a += blk_v[i];
        b += blk_w[i];
    }
    unsigned int pa = block_exclusive(a, sv, &tv);
    unsigned long long pb = block_exclusive(b, sw, &tw);
    for (int64_t i = a0; i < a1; ++i) {
        const unsigned int x = blk_v[i];
        const unsigned long long y = blk_w[i];
        blk_v[i] = pa;
        blk_w[i] = pb;
        pa += x;
        pb += y;
    }
    if (threadIdx.x == 0) {
        *total = tv;
        *total_w = tw;
        if (splits) {
            splits[0] = 0;
            splits[XCDS] = tv;
            for (unsigned int x = 1; x < XCDS; ++x) splits[x] = tw == 0 ? 0u : tv;
        }
    }
}

__global__ __launch_bounds__(SCAN_TB) void k_scan_apply(int64_t count, unsigned int *__restrict__ v,
                                                        const unsigned long long *__restrict__ w,
                                                        const unsigned int *__restrict__ blk_v,
                                                        const unsigned long long *__restrict__ blk_w,
                                                        const unsigned long long *__restrict__ total_w,
                                                        unsigned int *__restrict__ splits) {
    __shared__ unsigned int sv[SCAN_TB / WAVE];
    __shared__ unsigned long long sw[SCAN_TB / WAVE];
    __shared__ unsigned int tv;
    __shared__ unsigned long long tw;
    const int64_t base = (int64_t)blockIdx.x * SCAN_PER_BLOCK + (int64_t)threadIdx.x * SCAN_EPT;
    unsigned int xv[SCAN_EPT];
    unsigned long long xw[SCAN_EPT];
    unsigned int a = 0;
    unsigned long long b = 0;
    for (int q = 0; q < SCAN_EPT; ++q) {
        const int64_t i = base + q;
        xv[q] = i < count ? v[i] : 0u;
        xw[q] = (i < count && w) ? w[i] : 0ull;
        a += xv[q];
        b += xw[q];
    }
    unsigned int pa = blk_v[blockIdx.x] + block_exclusive(a, sv, &tv);
    unsigned long long pb = blk_w[blockIdx.x] + block_exclusive(b, sw, &tw);
    const unsigned long long tot = w ? *total_w : 0ull;
    for (int q = 0; q < SCAN_EPT; ++q) {
        const int64_t i = base + q;
        if (i >= count) break;
        v[i] = pa;
        const unsigned long long nxt = pb + xw[q];
        if (w && splits) {
            // element i holds the point x * tot / XCDS when pb < target <= nxt
            for (unsigned int x = 1; x < XCDS; ++x) {
                const unsigned long long target = tot * x / XCDS;
                if (target > 0 && pb < target && target <= nxt) splits[x] = pa + xv[q];
            }
        }
        pa += xv[q];
        pb = nxt;
    }
}

size_t scan_scratch_blocks(int64_t count) { return (size_t)std::max<int64_t>(1, ceil_div(count, SCAN_PER_BLOCK)); }

ad_status scan_exclusive(int64_t count, unsigned int *v, const unsigned long long *w, unsigned int *total,
                         unsigned int *splits, const ScanScratch &sc, hipStream_t s) {
    const int64_t nblk = (int64_t)scan_scratch_blocks(count);
    hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nblk), dim3(SCAN_TB), 0, s, count, v, w, sc.blk_v, sc.blk_w);
    AD_LAUNCH_CHECK("k_scan_partials");
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_TB), 0, s, nblk, sc.blk_v, sc.blk_w, total, sc.total_w,
                       w ? splits : nullptr);
    AD_LAUNCH_CHECK("k_scan_blocks");
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblk), dim3(SCAN_TB), 0, s, count, v, w, sc.blk_v, sc.blk_w,
                       sc.total_w, w ? splits : nullptr);
    AD_LAUNCH_CHECK("k_scan_apply");
    return AD_OK;
}

ad_status fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return AD_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, 256)), dim3(256), 0, s, p, v, count);
    AD_LAUNCH_CHECK("k_fill_i32");
    return AD_OK;
}

__global__ void k_collect_rows(int64_t n, const int64_t *__restrict__ row_ptr, int64_t lo,
                               int64_t hi, int32_t *__restrict__ list, unsigned int *count) {
    // the loop bound is uniform per wave (blocks are whole waves), so every
    // lane reaches the wave-wide append
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n_pad = ceil_div_dev(n, stride) * stride;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += stride) {
        bool take = false;
        if (i < n) {
            const int64_t d = row_ptr[i + 1] - row_ptr[i];
            take = d > lo && d <= hi;
        }
        const unsigned int at = wave_append(take, count);
        if (take) list[at] = (int32_t)i;
    }
}

ad_status collect_rows(const ad_graph *g, int64_t lo, int64_t hi, int32_t *list,
                       unsigned int *count, hipStream_t s) {
    if (g->n <= 0) return AD_OK;
    hipLaunchKernelGGL(k_collect_rows, dim3(grid_for(g->n, 256)), dim3(256), 0, s, g->n,
                       g->row_ptr, lo, hi, list, count);
    AD_LAUNCH_CHECK("k_collect_rows");
    return AD_OK;
}

__global__ void k_col_orig(int64_t nnz, const int32_t *__restrict__ col, const int32_t *__restrict__ orig_id,
                           int32_t *__restrict__ out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = col[p];
        out[p] = orig_id ? orig_id[j] : j;
    }
}

ad_status check_graph_args(const ad_graph *g) {
    if (!g) return fail(AD_ERR_INVALID_ARG, "graph is NULL");
    if (g->n < 0 || g->m < 0) return fail(AD_ERR_INVALID_ARG, "negative n or m");
    if (g->n > 0x7fffffffLL) return fail(AD_ERR_UNSUPPORTED, "n must fit in int32");
    if (g->m > 0x7fffffffLL) return fail(AD_ERR_UNSUPPORTED, "m must fit in int32");
    if (!g->row_ptr) return fail(AD_ERR_INVALID_ARG, "row_ptr is NULL");
    if (g->m > 0 && (!g->col || !g->eid)) return fail(AD_ERR_INVALID_ARG, "col or eid is NULL");
    if (g->d_max < 0) return fail(AD_ERR_INVALID_ARG, "negative d_max");
    return AD_OK;
}

// ---------------------------------------------------------------- validate --

// Flags: 1 col out of range, 2 self-loop, 4 unsorted/repeat, 8 no mirror,
// 16 mirror eid/weight mismatch, 32 bad weight, 64 eid out of range,
// 128 eid not used exactly twice, 256 row_ptr inconsistent, 512 degree > d_max.
__global__ void k_validate_rows(int64_t n, const int64_t *__restrict__ row_ptr,
                                const int32_t *__restrict__ col, const float *__restrict__ w,
                                const int32_t *__restrict__ eid, int64_t m, int32_t d_max,
                                unsigned int *__restrict__ eid_uses, unsigned int *flags) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = row_ptr[i], e = row_ptr[i + 1];
        unsigned f = 0;
        if (e < b) { atomicOr(flags, 256u); continue; }
        if (e - b > d_max) f |= 512u;
        for (int64_t p = b; p < e; ++p) {
            int32_t j = col[p];
            if (j < 0 || j >= n) { f |= 1u; continue; }
            if (j == i) f |= 2u;
            if (p > b && col[p - 1] >= j) f |= 4u;
            if (w && !(isfinite(w[p]) && w[p] > 0.f)) f |= 32u;
            int32_t id = eid[p];
            if (id < 0 || id >= m) { f |= 64u; continue; }
            atomicAdd(&eid_uses[id], 1u);
            // binary search for i in row j
            int64_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1;
            int64_t found = -1;
            while (lo <= hi) {
                int64_t mid = (lo + hi) >> 1;
                int32_t c = col[mid];
                if (c == (int32_t)i) { found = mid; break; }
                if (c < (int32_t)i) lo = mid + 1; else hi = mid - 1;
            }
            if (found < 0) f |= 8u;
            else if (eid[found] != id || (w && w[found] != w[p])) f |= 16u;
        }
        if (f) atomicOr(flags, f);
    }
}

// Structure of row_ptr alone: 0 <= row_ptr[i] <= row_ptr[i+1] <= nnz.
__global__ void k_validate_rowptr(int64_t n, const int64_t *__restrict__ row_ptr, int64_t nnz,
                                  unsigned int *flags) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = row_ptr[i], e = row_ptr[i + 1];
        if (b < 0 || e < b || e > nnz) atomicOr(flags, 256u);
    }
}

__global__ void k_validate_eids(int64_t m, const unsigned int *__restrict__ eid_uses,
                                unsigned int *flags) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
         q += (int64_t)gridDim.x * blockDim.x)
        if (eid_uses[q] != 2u) atomicOr(flags, 128u);
}

// ------------------------------------------------------------------ trace --

struct TraceRecord {
    std::string name;
    int launches;
    hipEvent_t a, b;
    int dev;
};
static std::atomic<bool> g_trace_on{false};
static std::mutex g_trace_mu;
static std::vector<TraceRecord> g_trace;
// Released events, per device (an event belongs to the device current when
// it was created), reused by later scopes.
struct PooledEvent {
    hipEvent_t ev;
    int dev;
};
static std::vector<PooledEvent> g_event_pool;

static int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        dev = 0;
    }
    return dev;
}

// An event of the current device from the pool (or a new one); g_trace_mu
// must be held.
static hipEvent_t pooled_event() {
    const int dev = current_device();
    for (size_t k = g_event_pool.size(); k-- > 0;) {
        if (g_event_pool[k].dev == dev) {
            hipEvent_t e = g_event_pool[k].ev;
            g_event_pool[k] = g_event_pool.back();
            g_event_pool.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

static thread_local int g_trace_suppress = 0;

TraceSuppress::TraceSuppress() { ++g_trace_suppress; }
TraceSuppress::~TraceSuppress() { --g_trace_suppress; }

TraceScope::TraceScope(const char *n, hipStream_t s, int count) : name(n), stream(s), launches(count) {
    if (!g_trace_on.load(std::memory_order_relaxed) || g_trace_suppress) return;
    {
        std::lock_guard<std::mutex> lk(g_trace_mu);
        a = pooled_event();
        b = a ? pooled_event() : nullptr;
        if (!b) {
            if (a) g_event_pool.push_back({a, current_device()});
            a = b = nullptr;
            return;
        }
        dev = current_device();
    }
    hipEventRecord(a, stream);
}

TraceScope::~TraceScope() {
    if (!a) return;
    hipEventRecord(b, stream);
    std::lock_guard<std::mutex> lk(g_trace_mu);
    g_trace.push_back({name, launches, a, b, dev});
}

}  // namespace ad

using namespace ad;

extern "C" void ad_trace_enable(int32_t on) { g_trace_on.store(on != 0); }

extern "C" void ad_trace_reset(void) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    for (auto &r : g_trace) {
        hipEventSynchronize(r.b);
        g_event_pool.push_back({r.a, r.dev});
        g_event_pool.push_back({r.b, r.dev});
    }
    g_trace.clear();
}

extern "C" ad_status ad_trace_summary(char *buf, size_t len) {
    if (!buf || len == 0) return fail(AD_ERR_INVALID_ARG, "buffer is NULL");
    std::lock_guard<std::mutex> lk(g_trace_mu);
    std::map<std::string, std::pair<long long, double>> agg;
    for (auto &r : g_trace) {
        AD_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        AD_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        auto &e = agg[r.name];
        e.first += r.launches;
        e.second += ms;
    }
    std::string out;
    char line[256];
    for (auto &kv : agg) {
        snprintf(line, sizeof(line), "%s %lld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
        out += line;
    }
    if (out.size() + 1 > len) return fail(AD_ERR_INVALID_ARG, "buffer too small");
    memcpy(buf, out.c_str(), out.size() + 1);
    return AD_OK;
}

extern "C" size_t ad_validate_workspace_size(const ad_graph *g) {
    if (!g) return 0;
    Carver c(nullptr, 0);
    c.take<unsigned int>(g->m > 0 ? g->m : 1);
    c.take<unsigned int>(1);
    return c.used;
}

extern "C" ad_status ad_validate_graph(const ad_graph *g, void *ws, size_t ws_bytes,
                                       hipStream_t stream) {
    ad_status st = check_graph_args(g);
    if (st != AD_OK) return st;
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    Carver c(ws, ws_bytes);
    unsigned int *uses = c.take<unsigned int>(g->m > 0 ? g->m : 1);
    unsigned int *flags = c.take<unsigned int>(1);
    if (!c.ok()) return fail(AD_ERR_WORKSPACE, "workspace too small");
    int64_t rp[2] = {0, 0};
    if (g->n >= 0) {
        AD_HIP(hipMemcpyAsync(&rp[0], g->row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        AD_HIP(hipMemcpyAsync(&rp[1], g->row_ptr + g->n, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        AD_HIP(hipStreamSynchronize(stream));
    }
    if (rp[0] != 0 || rp[1] != 2 * g->m)
        return fail(AD_ERR_GRAPH, "row_ptr[0] != 0 or row_ptr[n] != 2m");
    st = fill_i32((int32_t *)uses, 0, g->m, stream);
    if (st != AD_OK) return st;
    st = fill_i32((int32_t *)flags, 0, 1, stream);
    if (st != AD_OK) return st;
    if (g->n > 0) {
        // row_ptr first: the per-row pass below reads col[] through it.
        hipLaunchKernelGGL(k_validate_rowptr, dim3(grid_for(g->n, 256)), dim3(256), 0, stream,
                           g->n, g->row_ptr, 2 * g->m, flags);
        AD_LAUNCH_CHECK("k_validate_rowptr");
        unsigned int rflags = 0;
        AD_HIP(hipMemcpyAsync(&rflags, flags, sizeof(unsigned int), hipMemcpyDeviceToHost, stream));
        AD_HIP(hipStreamSynchronize(stream));
        if (rflags) return fail(AD_ERR_GRAPH, "invalid graph: row_ptr not monotone within [0, 2m];");
        hipLaunchKernelGGL(k_validate_rows, dim3(grid_for(g->n, 256)), dim3(256), 0, stream, g->n,
                           g->row_ptr, g->col, g->w, g->eid, g->m, g->d_max, uses, flags);
        AD_LAUNCH_CHECK("k_validate_rows");
    }
    if (g->m > 0) {
        hipLaunchKernelGGL(k_validate_eids, dim3(grid_for(g->m, 256)), dim3(256), 0, stream, g->m,
                           uses, flags);
        AD_LAUNCH_CHECK("k_validate_eids");
    }
    unsigned int hflags = 0;
    AD_HIP(hipMemcpyAsync(&hflags, flags, sizeof(unsigned int), hipMemcpyDeviceToHost, stream));
    AD_HIP(hipStreamSynchronize(stream));
    if (hflags == 0) return AD_OK;
    static const char *names[] = {"column out of range", "self-loop", "columns unsorted or repeated",
                                  "missing mirror entry", "mirror eid or weight differs",
                                  "weight not finite and > 0", "eid out of range",
                                  "eid not used exactly twice", "row_ptr decreasing",
                                  "degree above d_max"};
    std::string msg = "invalid graph:";
    for (int b = 0; b < 10; ++b)
        if (hflags & (1u << b)) msg += std::string(" ") + names[b] + ";";
    return fail(AD_ERR_GRAPH, msg);
}

extern "C" ad_status ad_graph_col_orig(const ad_graph *g, int32_t *col_orig, hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (g->m == 0) return AD_OK;
    if (!col_orig) return fail(AD_ERR_INVALID_ARG, "col_orig is NULL");
    const int64_t nnz = 2 * g->m;
    hipLaunchKernelGGL(k_col_orig, dim3(grid_for(nnz, 256)), dim3(256), 0, stream, nnz, g->col, g->orig_id,
                       col_orig);
    AD_LAUNCH_CHECK("k_col_orig");
    return AD_OK;
}

extern "C" const char *ad_status_string(ad_status s) {
    switch (s) {
    case AD_OK: return "AD_OK";
    case AD_ERR_INVALID_ARG: return "AD_ERR_INVALID_ARG";
    case AD_ERR_UNSUPPORTED: return "AD_ERR_UNSUPPORTED";
    case AD_ERR_WORKSPACE: return "AD_ERR_WORKSPACE";
    case AD_ERR_GRAPH: return "AD_ERR_GRAPH";
    case AD_ERR_HIP: return "AD_ERR_HIP";
    case AD_ERR_INTERNAL: return "AD_ERR_INTERNAL";
    }
    return "AD_ERR_UNKNOWN";
}

extern "C" const char *ad_last_error(void) { return ad::g_last_error.c_str(); }

extern "C" int32_t ad_abi_version(void) { return 1; }
