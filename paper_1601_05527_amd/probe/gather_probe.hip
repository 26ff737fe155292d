// Measurement aid, not part of the method: the rate at which the memory
// system delivers random rows when nothing else is asked of it.
//
// Every entry q of idx[0, nnz) gathers row idx[q] of a row-major array of
// rows of `row_bytes` bytes (16, 32, 64 or 128), one 16-byte piece per lane,
// and adds it into a per-lane sum; nothing is written but one 16-byte sum
// per thread.  Given the column array of a graph and a vector block of the
// sweep's row size, the time of one launch is the floor that gathering the
// sweep's neighbour rows, in the sweep's order, can reach on this device:
// the sweep also streams its columns and weights and writes its output rows.
//
// Built into its own library (libad_probe.so); the method's library does
// not use it.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int PROBE_BLOCK = 256;
constexpr int PROBE_UNROLL = 8;

template <int LPR>
__global__ __launch_bounds__(PROBE_BLOCK) void k_gather_probe(const float4 *__restrict__ x,
                                                              const int32_t *__restrict__ idx, int64_t nnz,
                                                              float4 *__restrict__ sums) {
    constexpr int SPW = 64 / LPR;    // rows per wave per gather instruction
    const int lane = threadIdx.x & 63;
    const int slot = lane / LPR, piece = lane % LPR;
    const int64_t wave = ((int64_t)blockIdx.x * PROBE_BLOCK + threadIdx.x) >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * (PROBE_BLOCK / 64);
    const int64_t per = (int64_t)SPW * PROBE_UNROLL;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t b = wave * per; b < nnz; b += nwaves * per) {
        int32_t j[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            const int64_t q = b + (int64_t)u * SPW + slot;
            j[u] = q < nnz ? idx[q] : -1;
        }
        float4 v[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u)
            v[u] = j[u] >= 0 ? x[(int64_t)j[u] * LPR + piece] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    sums[(int64_t)blockIdx.x * PROBE_BLOCK + threadIdx.x] = acc;
}

}  // namespace

extern "C" {

// Number of threads of one probe launch: `sums` holds that many 16-byte values.
int64_t ad_probe_threads(int blocks) { return (int64_t)blocks * PROBE_BLOCK; }

// x: device, n_rows rows of row_bytes bytes, 16-byte aligned.  idx: device,
// nnz row ids, each in [0, n_rows) (not checked on the device: the caller
// passes a valid column array).  sums: device, ad_probe_threads(blocks)
// float4.  Returns 0, -1 for bad arguments, or the HIP error of the launch.
int ad_probe_gather(const void *x, int64_t n_rows, int row_bytes, const int32_t *idx, int64_t nnz, void *sums,
                    int blocks, hipStream_t stream) {
    if (!x || !idx || !sums || n_rows < 1 || nnz < 0 || blocks < 1) return -1;
    if (nnz == 0) return 0;
    const float4 *X = (const float4 *)x;
    float4 *S = (float4 *)sums;
    switch (row_bytes) {
    case 16: hipLaunchKernelGGL(k_gather_probe<1>, dim3(blocks), dim3(PROBE_BLOCK), 0, stream, X, idx, nnz, S); break;
    case 32: hipLaunchKernelGGL(k_gather_probe<2>, dim3(blocks), dim3(PROBE_BLOCK), 0, stream, X, idx, nnz, S); break;
    case 64: hipLaunchKernelGGL(k_gather_probe<4>, dim3(blocks), dim3(PROBE_BLOCK), 0, stream, X, idx, nnz, S); break;
    case 128: hipLaunchKernelGGL(k_gather_probe<8>, dim3(blocks), dim3(PROBE_BLOCK), 0, stream, X, idx, nnz, S); break;
    default: return -1;
    }
    return (int)hipGetLastError();
}

}  // extern "C"
