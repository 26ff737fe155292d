// ad_backward.hip -- reverse-mode derivative of L(rho) with respect to the
// edge weights, through the distance, the rescale and the k JOR sweeps of
// Algorithm 1 (FP32).
//
// Forward recap (per vector r; x^(t) below is the relaxation's own value,
// the stored one plus its component's shift, which no sweep changes):
//   x^(t)_i = (1-omega) x^(t-1)_i + omega y^(t)_i,  y^(t)_i = sum_j w_ij x^(t-1)_j / s_i,
//   xhat_i  = (x^(k)_i - m) / (M - m) - 1/2   (m, M: min and max over live rows),
//   rho_e   = sqrt(sum_r (xhat_i - xhat_j)^2).
// Adjoint:
//   xhatbar_i = sum_{e=(i,j)} gbar_e (xhat_i - xhat_j) / rho_e      (0 when rho_e = 0)
//   lambda^(k)_i = xhatbar_i / (M-m), plus
//     sum_i xhatbar_i (x_i - M) / (M-m)^2 at the first row attaining m and
//    -sum_i xhatbar_i (x_i - m) / (M-m)^2 at the first row attaining M;
//   for t = k..1, with w_ij in row i's formula:
//     g_ij += omega * sum_r lambda^(t)_i (x^(t-1)_j - y^(t)_i) / s_i
//     lambda^(t-1) = (1-omega) lambda^(t) + omega W (lambda^(t) / s)
//   dL/dw_e = g_ij + g_ji.
// x^(t-1) for every t comes from the checkpoints: each segment of
// ckpt_every sweeps is recomputed with the forward sweep kernel and launch
// shape, so the recomputed values equal the forward ones bit for bit.
#include "ad_internal.h"

#include <math.h>

#include <algorithm>

namespace ad {

constexpr int BB = 256;
constexpr int PART_ROWS = 1024;

static int lanes_for(double avg) {
    int lpr = 1;
    while (lpr < 64 && lpr < avg) lpr <<= 1;
    return lpr;
}

// xhatbar from grad_rho: one lane per stored entry, LPR lanes per row.  rho
// is recomputed in the forward distance kernel's order: VEC values per chunk
// summed in order, chunks combined by a pairwise tree when their count is a
// power of two, else in order -- so it equals the forward value bit for bit.
template <int RB, int VEC>
__global__ __launch_bounds__(BB) void k_adj_dist(int64_t n, const int64_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col,
                                                 const int32_t *__restrict__ eid,
                                                 const float *__restrict__ x, const double *__restrict__ minmax,
                                                 const float *__restrict__ grad_rho, float *__restrict__ xbh,
                                                 int R, int LPR) {
    __shared__ float inv_l[64];
    if (threadIdx.x < R) {
        double lo = minmax[threadIdx.x], hi = minmax[R + threadIdx.x];
        inv_l[threadIdx.x] = (hi > lo) ? (float)(1.0 / (hi - lo)) : 0.f;
    }
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * (BB / LPR) + threadIdx.x / LPR;
    const int lane = threadIdx.x % LPR;
    float acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = 0.f;
    if (row < n) {
        const int64_t beg = row_ptr[row], end = row_ptr[row + 1];
        const float *xi = x + row * R;
        for (int64_t p = beg + lane; p < end; p += LPR) {
            const float *xj = x + (int64_t)col[p] * R;
            float d[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) d[r] = r < R ? (xi[r] - xj[r]) * inv_l[r] : 0.f;
            constexpr int NC = RB / VEC;
            const int C = R / VEC;
            float part[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                float a = 0.f;
#pragma unroll
                for (int q = 0; q < VEC; ++q) a = fmaf(d[c * VEC + q], d[c * VEC + q], a);
                part[c] = a;
            }
            float ss;
            if ((C & (C - 1)) == 0) {
#pragma unroll
                for (int off = 1; off < NC; off <<= 1) {
#pragma unroll
                    for (int c = 0; c + off < NC; c += 2 * off)
                        if (off < C) part[c] += part[c + off];
                }
                ss = part[0];
            } else {
                ss = part[0];
#pragma unroll
                for (int c = 1; c < NC; ++c)
                    if (c < C) ss += part[c];
            }
            const float rho = sqrtf(ss);
            if (rho > 0.f) {
                const float c = grad_rho[eid[p]] / rho;
#pragma unroll
                for (int r = 0; r < RB; ++r) acc[r] = fmaf(c, d[r], acc[r]);
            }
        }
    }
    for (int off = LPR >> 1; off >= 1; off >>= 1) {
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] += shfl_down(acc[r], off);
    }
    if (row < n && lane == 0) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (r < R) xbh[row * R + r] = acc[r];
    }
}

// First live row attaining the min and the max of each vector (values with
// their shift added back exactly as ad_relax's min / max pass adds it).
__global__ void k_adj_argminmax(int64_t n, int R, const int64_t *__restrict__ row_ptr,
                                const float *__restrict__ x, const double *__restrict__ shift,
                                const int32_t *__restrict__ comp_of, const double *__restrict__ minmax,
                                unsigned long long *__restrict__ arg) {
    const int64_t total = n * R;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / R;
        const int r = (int)(idx - i * R);
        if (row_ptr[i + 1] == row_ptr[i]) continue;
        bool zero;
        const double *sh = row_shift(shift, comp_of, i, 0, R, zero);
        const double v = (double)x[idx] + (zero ? 0.0 : sh[r]);
        if (v == minmax[r]) atomicMin(&arg[r], (unsigned long long)i);
        if (v == minmax[R + r]) atomicMin(&arg[R + r], (unsigned long long)i);
    }
}

// lambda = xhatbar / (M - m) on live rows; partial sums for the min/max terms.
__global__ __launch_bounds__(BB) void k_adj_rescale(int64_t n, int R, const int64_t *__restrict__ row_ptr,
                                                   const float *__restrict__ x, const double *__restrict__ shift,
                                                   const int32_t *__restrict__ comp_of,
                                                   const double *__restrict__ minmax,
                                                   const float *__restrict__ xbh, float *__restrict__ lam,
                                                   double *__restrict__ part) {
    __shared__ double a_l[BB];
    __shared__ double b_l[BB];
    const int t = threadIdx.x;
    const int stride = BB / R;
    const int r = t % R;
    const int row_off = t / R;
    const double lo = minmax[r], hi = minmax[R + r];
    const double D = hi - lo;
    const double inv = D > 0 ? 1.0 / D : 0.0;
    double a = 0.0, b = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * PART_ROWS;
    const int64_t r1 = min(n, r0 + PART_ROWS);
    if (row_off < stride) {
        for (int64_t i = r0 + row_off; i < r1; i += stride) {
            const bool live = row_ptr[i + 1] > row_ptr[i];
            const double xb = live ? (double)xbh[i * R + r] : 0.0;
            lam[i * R + r] = (float)(xb * inv);
            bool zero;
            const double *sh = row_shift(shift, comp_of, i, 0, R, zero);
            const double xv = (double)x[i * R + r] + (zero ? 0.0 : sh[r]);
            a += xb * (xv - hi) * inv * inv;
            b -= xb * (xv - lo) * inv * inv;
        }
    }
    a_l[t] = a;
    b_l[t] = b;
    __syncthreads();
    if (t < R) {
        double sa = 0.0, sb = 0.0;
        for (int q = t; q < stride * R; q += R) {
            sa += a_l[q];
            sb += b_l[q];
        }
        part[(int64_t)blockIdx.x * 2 * R + t] = sa;
        part[(int64_t)blockIdx.x * 2 * R + R + t] = sb;
    }
}

__global__ void k_adj_corner(int R, int64_t nblocks, const double *__restrict__ part,
                             const unsigned long long *__restrict__ arg, const double *__restrict__ minmax,
                             float *__restrict__ lam) {
    const int r = threadIdx.x;
    if (r >= R) return;
    if (!(minmax[R + r] > minmax[r])) return;
    double sa = 0.0, sb = 0.0;
    for (int64_t b = 0; b < nblocks; ++b) {
        sa += part[b * 2 * R + r];
        sb += part[b * 2 * R + R + r];
    }
    const unsigned long long imin = arg[r], imax = arg[R + r];
    // one thread per vector: the two updates of column r never race
    lam[imin * R + r] = (float)((double)lam[imin * R + r] + sa);
    lam[imax * R + r] = (float)((double)lam[imax * R + r] + sb);
}

// g[p] += omega * inv_s_i * sum_r lambda_i,r (x_j,r - y_i,r)
template <int RB>
__global__ __launch_bounds__(BB) void k_adj_grad(int64_t n, const int64_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col, const float *__restrict__ inv_s,
                                                 float omega, const float *__restrict__ xprev,
                                                 const float *__restrict__ y, const float *__restrict__ lam,
                                                 float *__restrict__ g, int R, int LPR) {
    const int64_t row = (int64_t)blockIdx.x * (BB / LPR) + threadIdx.x / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= n) return;
    const int64_t beg = row_ptr[row], end = row_ptr[row + 1];
    if (beg == end) return;
    float li[RB], yi[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        li[r] = r < R ? lam[row * R + r] : 0.f;
        yi[r] = r < R ? y[row * R + r] : 0.f;
    }
    const float sc = omega * inv_s[row];
    for (int64_t p = beg + lane; p < end; p += LPR) {
        const float *xj = xprev + (int64_t)col[p] * R;
        float dot = 0.f;
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (r < R) dot = fmaf(li[r], xj[r] - yi[r], dot);
        g[p] = fmaf(sc, dot, g[p]);
    }
}

__global__ void k_adj_scale_rows(int64_t n, int R, const float *__restrict__ a, const float *__restrict__ s,
                                 float *__restrict__ out) {
    const int64_t total = n * R;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x)
        out[idx] = a[idx] * s[idx / R];
}

// out = (1 - omega) a + omega b
__global__ void k_adj_axpby(int64_t total, float omega, const float *__restrict__ a, const float *__restrict__ b,
                            float *__restrict__ out) {
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x)
        out[idx] = fmaf(omega, b[idx], (1.f - omega) * a[idx]);
}

__global__ void k_edge_to_entries(int64_t nnz, const int32_t *__restrict__ eid, const float *__restrict__ we,
                                  float *__restrict__ out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x)
        out[p] = we[eid[p]];
}

__global__ void k_adj_fold(int64_t nnz, const int32_t *__restrict__ eid, const float *__restrict__ g,
                           float *__restrict__ grad_w) {
    // two addends per edge onto a zeroed slot: the result does not depend on order
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&grad_w[eid[p]], g[p]);
}

struct BwdLayout {
    float *inv_s, *sdeg, *ones;
    SweepPlan plan;
    float *xbh, *lam, *lam2, *mu, *y, *seg, *g;
    double *part;
    unsigned long long *arg;
};

static size_t bwd_layout(const ad_graph *g, const ad_relax_opts *o, void *ws, size_t ws_bytes, BwdLayout *L) {
    Carver c(ws, ws_bytes);
    const int64_t n = std::max<int64_t>(1, g->n);
    const int64_t nnz = std::max<int64_t>(1, 2 * g->m);
    const size_t nR = (size_t)n * o->R;
    const int64_t nb = std::max<int64_t>(1, ceil_div(g->n, PART_ROWS));
    BwdLayout l;
    l.inv_s = c.take<float>(n);
    l.sdeg = c.take<float>(n);
    l.ones = c.take<float>(n);
    sweep_plan_carve(c, n, ceil_div(n, PLAN_TILE), l.plan);
    l.xbh = c.take<float>(nR);
    l.lam = c.take<float>(nR);
    l.lam2 = c.take<float>(nR);
    l.mu = c.take<float>(nR);
    l.y = c.take<float>(nR);
    l.seg = c.take<float>(nR * (size_t)std::max(1, o->ckpt_every));
    l.g = c.take<float>(nnz);
    l.part = c.take<double>(nb * 2 * o->R);
    l.arg = c.take<unsigned long long>(2 * o->R);
    if (L) *L = l;
    return c.ok() ? c.used : 0;
}

template <int RB>
static ad_status launch_rb(const ad_graph *g, const ad_relax_opts *o, const float *x_k, const double *minmax,
                           const float *grad_rho, const BwdLayout &L, int lpr, hipStream_t st) {
    const unsigned nb = (unsigned)ceil_div(g->n, BB / lpr);
    const int R = o->R;
    // the forward distance kernel's vector width for FP32
    const int vec = R % 4 == 0 ? 4 : (R % 2 == 0 ? 2 : 1);
    if (vec == 4)
        hipLaunchKernelGGL((k_adj_dist<RB, 4>), dim3(nb), dim3(BB), 0, st, g->n, g->row_ptr, g->col, g->eid, x_k,
                           minmax, grad_rho, L.xbh, R, lpr);
    else if (vec == 2)
        hipLaunchKernelGGL((k_adj_dist<RB, 2>), dim3(nb), dim3(BB), 0, st, g->n, g->row_ptr, g->col, g->eid, x_k,
                           minmax, grad_rho, L.xbh, R, lpr);
    else
        hipLaunchKernelGGL((k_adj_dist<RB, 1>), dim3(nb), dim3(BB), 0, st, g->n, g->row_ptr, g->col, g->eid, x_k,
                           minmax, grad_rho, L.xbh, R, lpr);
    AD_LAUNCH_CHECK("k_adj_dist");
    return AD_OK;
}

template <int RB>
static ad_status launch_grad(const ad_graph *g, const BwdLayout &L, float omega, const float *xprev,
                             const float *lam, int R, int lpr, hipStream_t st) {
    const unsigned nb = (unsigned)ceil_div(g->n, BB / lpr);
    hipLaunchKernelGGL((k_adj_grad<RB>), dim3(nb), dim3(BB), 0, st, g->n, g->row_ptr, g->col, L.inv_s, omega,
                       xprev, L.y, lam, L.g, R, lpr);
    AD_LAUNCH_CHECK("k_adj_grad");
    return AD_OK;
}

}  // namespace ad

using namespace ad;

extern "C" ad_status ad_edge_to_entries(const ad_graph *g, const float *w_edge, float *w_entries,
                                        hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (g->m == 0) return AD_OK;
    if (!w_edge || !w_entries) return fail(AD_ERR_INVALID_ARG, "w_edge or w_entries is NULL");
    const int64_t nnz = 2 * g->m;
    hipLaunchKernelGGL(k_edge_to_entries, dim3(grid_for(nnz, BB)), dim3(BB), 0, stream, nnz, g->eid, w_edge,
                       w_entries);
    AD_LAUNCH_CHECK("k_edge_to_entries");
    return AD_OK;
}

extern "C" size_t ad_relax_backward_workspace_size(const ad_graph *g, const ad_relax_opts *o) {
    if (check_graph_args(g) != AD_OK || !o || o->R < 1 || o->R > 64 || o->ckpt_every < 1) return 0;
    return bwd_layout(g, o, nullptr, 0, nullptr);
}

extern "C" ad_status ad_relax_backward(const ad_graph *g, const ad_relax_opts *o, const void *ckpt,
                                       const void *x_k, const double *minmax, const double *shift,
                                       const float *grad_rho, float *grad_w, void *ws, size_t ws_bytes,
                                       hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (!o) return fail(AD_ERR_INVALID_ARG, "opts is NULL");
    if (o->R < 1 || o->R > 64) return fail(AD_ERR_INVALID_ARG, "R must be in [1, 64]");
    if (o->k < 0) return fail(AD_ERR_INVALID_ARG, "k must be >= 0");
    if (!(o->omega > 0.0 && o->omega <= 1.0)) return fail(AD_ERR_INVALID_ARG, "omega must be in (0, 1]");
    if (o->store != AD_F32) return fail(AD_ERR_UNSUPPORTED, "the adjoint needs FP32 storage");
    if (o->fp64_tail != 0) return fail(AD_ERR_UNSUPPORTED, "the adjoint needs fp64_tail == 0");
    if (o->ckpt_every < 1) return fail(AD_ERR_INVALID_ARG, "the adjoint needs ckpt_every >= 1");
    if (g->m > 0 && (!x_k || !minmax || !shift || !grad_rho || !grad_w))
        return fail(AD_ERR_INVALID_ARG, "x_k, minmax, shift, grad_rho or grad_w is NULL");
    if (o->comp && o->comp->n_comp > 0 && !o->comp->comp_of)
        return fail(AD_ERR_INVALID_ARG, "component arrays are NULL");
    const int32_t *comp_of = o->comp ? o->comp->comp_of : nullptr;
    if (o->k > 0 && g->m > 0 && !ckpt) return fail(AD_ERR_INVALID_ARG, "ckpt is NULL");
    if (!ws) return fail(AD_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(AD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    BwdLayout L;
    if (bwd_layout(g, o, ws, ws_bytes, &L) == 0) return fail(AD_ERR_WORKSPACE, "workspace too small");
    if (g->m == 0) return AD_OK;

    const int R = o->R;
    const int64_t n = g->n, nnz = 2 * g->m;
    const size_t nR = (size_t)n * R;
    const double avg = (double)nnz / (double)n;
    const int lpr = lanes_for(avg);
    const float omega = (float)o->omega;
    const float *xk = (const float *)x_k;

    SweepPlan plan = L.plan;
    plan.sh = sweep_shape(R, sizeof(float), o->rows_per_wave, o->hub_degree);
    s = sweep_plan_build(g, plan, true, Segs(), stream);
    if (s != AD_OK) return s;
    s = weighted_degree_f32(g, L.inv_s, L.sdeg, plan, stream);
    if (s != AD_OK) return s;
    s = fill_i32((int32_t *)L.ones, 0x3f800000, n, stream);   // 1.0f
    if (s != AD_OK) return s;
    s = fill_i32((int32_t *)L.g, 0, nnz, stream);
    if (s != AD_OK) return s;
    s = fill_i32((int32_t *)grad_w, 0, g->m, stream);
    if (s != AD_OK) return s;

    // distance adjoint
    if (R <= 8) s = launch_rb<8>(g, o, xk, minmax, grad_rho, L, lpr, stream);
    else if (R <= 16) s = launch_rb<16>(g, o, xk, minmax, grad_rho, L, lpr, stream);
    else if (R <= 32) s = launch_rb<32>(g, o, xk, minmax, grad_rho, L, lpr, stream);
    else s = launch_rb<64>(g, o, xk, minmax, grad_rho, L, lpr, stream);
    if (s != AD_OK) return s;

    // rescale adjoint
    s = fill_u64(L.arg, ~0ull, 2 * R, stream);
    if (s != AD_OK) return s;
    hipLaunchKernelGGL(k_adj_argminmax, dim3(grid_for((int64_t)nR, BB)), dim3(BB), 0, stream, n, R, g->row_ptr,
                       xk, shift, comp_of, minmax, L.arg);
    AD_LAUNCH_CHECK("k_adj_argminmax");
    const int64_t nb = std::max<int64_t>(1, ceil_div(n, PART_ROWS));
    hipLaunchKernelGGL(k_adj_rescale, dim3((unsigned)nb), dim3(BB), 0, stream, n, R, g->row_ptr, xk, shift,
                       comp_of, minmax, L.xbh, L.lam, L.part);
    AD_LAUNCH_CHECK("k_adj_rescale");
    hipLaunchKernelGGL(k_adj_corner, dim3(1), dim3(64), 0, stream, R, nb, L.part, L.arg, minmax, L.lam);
    AD_LAUNCH_CHECK("k_adj_corner");

    // reverse sweeps, one checkpoint segment at a time
    const int c = o->ckpt_every;
    const int nseg = ad_relax_num_checkpoints(o);
    float *lam = L.lam, *lam_next = L.lam2;
    for (int q = nseg - 1; q >= 0; --q) {
        const int t0 = q * c;
        const int t1 = std::min(o->k, (q + 1) * c);
        const float *base = (const float *)ckpt + (size_t)q * nR;
        // seg[u] = x^(t0 + u), u = 0 .. t1 - t0 - 1
        for (int u = 1; u < t1 - t0; ++u) {
            const float *src = u == 1 ? base : L.seg + (size_t)(u - 1) * nR;
            s = sweep_f32(g, L.inv_s, omega, src, L.seg + (size_t)u * nR, R, plan, stream);
            if (s != AD_OK) return s;
        }
        for (int t = t1; t > t0; --t) {
            const int u = t - 1 - t0;
            const float *xprev = u == 0 ? base : L.seg + (size_t)u * nR;
            // y = S^-1 W x^(t-1): the sweep kernel with omega = 1
            s = sweep_f32(g, L.inv_s, 1.0f, xprev, L.y, R, plan, stream);
            if (s != AD_OK) return s;
            if (R <= 8) s = launch_grad<8>(g, L, omega, xprev, lam, R, lpr, stream);
            else if (R <= 16) s = launch_grad<16>(g, L, omega, xprev, lam, R, lpr, stream);
            else if (R <= 32) s = launch_grad<32>(g, L, omega, xprev, lam, R, lpr, stream);
            else s = launch_grad<64>(g, L, omega, xprev, lam, R, lpr, stream);
            if (s != AD_OK) return s;
            // lambda^(t-1) = (1 - omega) lambda + omega W (lambda / s)
            hipLaunchKernelGGL(k_adj_scale_rows, dim3(grid_for((int64_t)nR, BB)), dim3(BB), 0, stream, n, R, lam,
                               L.inv_s, L.mu);
            AD_LAUNCH_CHECK("k_adj_scale_rows");
            s = sweep_f32(g, L.ones, 1.0f, L.mu, L.y, R, plan, stream);
            if (s != AD_OK) return s;
            hipLaunchKernelGGL(k_adj_axpby, dim3(grid_for((int64_t)nR, BB)), dim3(BB), 0, stream, (int64_t)nR,
                               omega, lam, L.y, lam_next);
            AD_LAUNCH_CHECK("k_adj_axpby");
            std::swap(lam, lam_next);
        }
    }
    hipLaunchKernelGGL(k_adj_fold, dim3(grid_for(nnz, BB)), dim3(BB), 0, stream, nnz, g->eid, L.g, grad_w);
    AD_LAUNCH_CHECK("k_adj_fold");
    return AD_OK;
}
