// Field-point ordering: points are sorted along a Morton (Z-order) curve so that the
// points of one wavefront lie close together, mostly choose the same rule level for a
// given element (rule choice by distance ratio) and are near the same elements.  Results
// are stored back in the caller's order by the evaluation's last kernel (finish_points_kernel).
#include <hipcub/hipcub.hpp>

#include "bemc_internal.h"

namespace bemc {

namespace {

constexpr int kBlock = 256;

__global__ void bbox_partial_kernel(const double* __restrict__ pts, int64_t n, double* __restrict__ part)
{
    __shared__ double smin[3][kBlock], smax[3][kBlock];
    double lo[3] = { 1e300, 1e300, 1e300 }, hi[3] = { -1e300, -1e300, -1e300 };
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = pts[c * n + i];
            lo[c] = fmin(lo[c], v);
            hi[c] = fmax(hi[c], v);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        smin[c][threadIdx.x] = lo[c];
        smax[c][threadIdx.x] = hi[c];
    }
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                smin[c][threadIdx.x] = fmin(smin[c][threadIdx.x], smin[c][threadIdx.x + w]);
                smax[c][threadIdx.x] = fmax(smax[c][threadIdx.x], smax[c][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            part[6 * blockIdx.x + c] = smin[c][0];
            part[6 * blockIdx.x + 3 + c] = smax[c][0];
        }
}

__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void morton_kernel(const double* __restrict__ pts, int64_t n, const double* __restrict__ part, int nparts,
                              uint32_t* __restrict__ keys, uint32_t* __restrict__ idx)
{
    double lo[3] = { 1e300, 1e300, 1e300 }, hi[3] = { -1e300, -1e300, -1e300 };
    for (int b = 0; b < nparts; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], part[6 * b + c]);
            hi[c] = fmax(hi[c], part[6 * b + 3 + c]);
        }
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double ext = hi[c] - lo[c];
        double u = ext > 0.0 ? (pts[c * n + i] - lo[c]) / ext : 0.0;
        u = fmin(fmax(u, 0.0), 1.0);  // also maps NaN to 0
        q[c] = min(1023u, (uint32_t)(u * 1024.0));
    }
    keys[i] = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
    idx[i] = (uint32_t)i;
}

__global__ void gather_kernel(const double* __restrict__ pts, int64_t n, const uint32_t* __restrict__ perm,
                              double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * n + i] = pts[c * n + j];
}

}  // namespace

size_t order_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                             (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)n, 0, 30);
    return bytes;
}

hipError_t order_points(const double* pts, int64_t n, const OrderWork& w, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int nparts = (int)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
    bbox_partial_kernel<<<nparts, kBlock, 0, s>>>(pts, n, w.bbox);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    morton_kernel<<<blocks, kBlock, 0, s>>>(pts, n, w.bbox, nparts, w.keys_in, w.idx_in);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    size_t bytes = w.temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(w.temp, bytes, w.keys_in, w.keys_out, w.idx_in, w.perm, (int)n, 0, 30, s);
    if (e != hipSuccess) return e;
    gather_kernel<<<blocks, kBlock, 0, s>>>(pts, n, w.perm, w.pts);
    return hipGetLastError();
}

}  // namespace bemc
