// Deterministic near-field accumulation.
//
// The list pass appends near pairs to a list in an order that depends on scheduling.
// Before the near kernel runs, each pair gets a result slot in (point, element) order:
// pairs are regrouped by field point (counts per point, an exclusive scan, a scatter) and
// each point's segment is ordered by element index.  The near kernel walks the pairs in
// the list's order (neighbouring points and the same element: similar subdivision trees
// side by side) and writes each pair's result record to its slot; one thread per point
// then adds its segment in element order to the point's far-field result.  The outcome
// does not depend on how the GPU scheduled the work.  No step needs the pair count on the
// host: the kernels read it from the device counters.
#include <hipcub/hipcub.hpp>

#include "bemc_internal.h"

namespace bemc {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ unsigned long long pair_total(const DevCounters* ctr, unsigned long long cap)
{
    const unsigned long long c = ctr->near_count;
    return c < cap ? c : cap;
}

__global__ void zero_u32_kernel(uint32_t* __restrict__ a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) a[i] = 0u;
}

__global__ void count_kernel(const NearPair* __restrict__ list, const DevCounters* __restrict__ ctr,
                             unsigned long long cap, uint32_t* __restrict__ count)
{
    const unsigned long long total = pair_total(ctr, cap);
    for (unsigned long long i = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (unsigned long long)gridDim.x * kBlock)
        atomicAdd(&count[list[i].point], 1u);
}

__global__ void scatter_pairs_kernel(const NearPair* __restrict__ list, const DevCounters* __restrict__ ctr,
                                     unsigned long long cap, const uint32_t* __restrict__ start,
                                     uint32_t* __restrict__ cursor, NearPair* __restrict__ grouped,
                                     uint32_t* __restrict__ origin)
{
    const unsigned long long total = pair_total(ctr, cap);
    for (unsigned long long i = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (unsigned long long)gridDim.x * kBlock) {
        const NearPair pr = list[i];
        const uint32_t pos = start[pr.point] + atomicAdd(&cursor[pr.point], 1u);
        grouped[pos] = pr;
        origin[pos] = (uint32_t)i;
    }
}

// Sorts each point's segment by element index, one wavefront per point: every entry's
// place is the number of entries of the segment with a smaller element index (the
// elements of a segment are distinct).  Segments hold the elements within near_dr L of
// the point: tens of entries, rarely thousands.
constexpr int kWavesPerBlock = kBlock / 64;

__global__ void rank_sort_kernel(const uint32_t* __restrict__ start, const uint32_t* __restrict__ count, int64_t n,
                                 const NearPair* __restrict__ in, const uint32_t* __restrict__ origin,
                                 NearPair* __restrict__ out, uint32_t* __restrict__ slot)
{
    const int64_t p = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / 64;  // same for the whole wavefront
    if (p >= n) return;
    const uint32_t s = start[p], k = count[p];
    for (uint32_t i = threadIdx.x % 64; i < k; i += 64) {
        const NearPair v = in[s + i];
        uint32_t rank = 0;
        for (uint32_t j = 0; j < k; ++j) rank += in[s + j].elem < v.elem ? 1u : 0u;
        out[s + rank] = v;
        slot[origin[s + i]] = s + rank;  // where the pair at this list index puts its result
    }
}

// Adds each point's near-pair results, in element order, to its far-field result.
// mode kNearEval: records (phi, Ex, Ey, Ez) (already scaled); kNearGrad: records of the six
// gradient rows (scaled); kNearColloc: one unscaled value per pair, multiplied here by
// K q_r(element) per density r.
__global__ void reduce_pairs_kernel(const uint32_t* __restrict__ start, const uint32_t* __restrict__ count,
                                    int64_t n, const NearPair* __restrict__ sorted, const double* __restrict__ res,
                                    int mode, double* __restrict__ phi,
                                    double* __restrict__ E, double* __restrict__ G, const double* __restrict__ q,
                                    int64_t ne, int n_rhs, double K)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const uint32_t s = start[p], k = count[p];
    if (k == 0) return;
    if (mode == kNearColloc) {
        for (int r = 0; r < n_rhs; ++r) {
            double acc = 0.0;
            for (uint32_t m = 0; m < k; ++m) acc += q[(int64_t)r * ne + sorted[s + m].elem] * res[s + m];
            phi[(int64_t)r * ne + p] += K * acc;
        }
        return;
    }
    const int rec = mode == kNearGrad ? 6 : 4;  // result record of a pair (see near_kernel)
    const int rows = mode == kNearGrad ? 6 : (E ? 4 : 1);
    for (int c = 0; c < rows; ++c) {
        double acc = 0.0;
        for (uint32_t m = 0; m < k; ++m) acc += res[(unsigned long long)(s + m) * rec + c];
        if (mode == kNearGrad) G[(int64_t)c * n + p] += acc;
        else if (c == 0) phi[p] += acc;
        else E[(int64_t)(c - 1) * n + p] += acc;
    }
}

unsigned grid_for(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

}  // namespace

void near_work_free(NearWork& w)
{
    for (void* ptr : { (void*)w.count, (void*)w.start, (void*)w.cursor, (void*)w.grouped, (void*)w.origin,
                       (void*)w.sorted, (void*)w.slot, (void*)w.res, w.temp })
        if (ptr) (void)hipFree(ptr);
    w = NearWork{};
}

hipError_t near_work_alloc(NearWork& w, int64_t n, unsigned long long pairs, int rows)
{
    near_work_free(w);
    const size_t np = (size_t)std::max<int64_t>(n, 1), npairs = (size_t)std::max<unsigned long long>(pairs, 1);
    w.temp_bytes = near_scan_temp_bytes(std::max<int64_t>(n, 1));
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&w.count), np * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.start), np * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.cursor), np * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.grouped), npairs * sizeof(NearPair));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.origin), npairs * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.sorted), npairs * sizeof(NearPair));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.slot), npairs * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.res), npairs * (size_t)rows * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&w.temp, std::max<size_t>(w.temp_bytes, 1));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        const size_t tb = w.temp_bytes;
        near_work_free(w);
        w.temp_bytes = tb;
    }
    return e;
}

size_t near_scan_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)n);
    return bytes;
}

hipError_t near_order(const NearPair* list, const DevCounters* ctr, unsigned long long cap, int64_t n,
                      const NearWork& w, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    zero_u32_kernel<<<grid_for(n), kBlock, 0, s>>>(w.count, n);
    zero_u32_kernel<<<grid_for(n), kBlock, 0, s>>>(w.cursor, n);
    count_kernel<<<grid_for((int64_t)std::min<unsigned long long>(cap, 1ull << 40)), kBlock, 0, s>>>(list, ctr, cap,
                                                                                                  w.count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = w.temp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(w.temp, bytes, w.count, w.start, (int)n, s);
    if (e != hipSuccess) return e;
    scatter_pairs_kernel<<<grid_for((int64_t)std::min<unsigned long long>(cap, 1ull << 40)), kBlock, 0, s>>>(
        list, ctr, cap, w.start, w.cursor, w.grouped, w.origin);
    const int64_t blocks = (n + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    rank_sort_kernel<<<(unsigned)blocks, kBlock, 0, s>>>(w.start, w.count, n, w.grouped, w.origin, w.sorted, w.slot);
    return hipGetLastError();
}

hipError_t near_reduce(const NearWork& w, int64_t n, int mode, double* phi, double* E,
                       double* G, const double* q, int64_t ne, int n_rhs, double K, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    reduce_pairs_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        w.start, w.count, n, w.sorted, w.res, mode, phi, E, G, q, ne, n_rhs, K);
    return hipGetLastError();
}

}  // namespace bemc
