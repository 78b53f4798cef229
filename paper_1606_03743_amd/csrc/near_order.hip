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
//
// The near kernel's lanes take pairs from a shared cursor, most expensive first: a pair's
// subdivision has a number of leaves that grows with log2(L / d), d the distance from the
// point to the element (from a few leaves at distance ratio 3 to thousands a thousandth of
// L above the element).  The list indices are bucketed by an estimate of that depth
// (counting sort over cost classes, order within a class arbitrary), so the lanes of a
// wavefront walk trees of similar size and the long walks start first.
#include <hipcub/hipcub.hpp>

#include "bemc_internal.h"
#include "on_element.h"

namespace bemc {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ unsigned long long pair_total(const DevCounters* ctr, unsigned long long cap)
{
    const unsigned long long c = ctr->near_count;
    return c < cap ? c : cap;
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

// The call's counters, copied by the first threads of the last kernel of an evaluation into
// the host's pinned record of the call (out: its device address; null: the host copies them).
__device__ __forceinline__ void copy_counters(const DevCounters* __restrict__ ctr, DevCounters* __restrict__ out)
{
    constexpr int kWords = (int)(sizeof(DevCounters) / sizeof(unsigned long long));
    if (out && blockIdx.x == 0 && threadIdx.x < kWords) {
        reinterpret_cast<unsigned long long*>(out)[threadIdx.x] =
            reinterpret_cast<const unsigned long long*>(ctr)[threadIdx.x];
        __threadfence_system();
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
                                    int64_t ne, int n_rhs, double K, const DevCounters* __restrict__ ctr,
                                    DevCounters* __restrict__ ctr_out)
{
    copy_counters(ctr, ctr_out);
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

// The final value of each point (field or gradient rows): its far field (K times the element
// chunks' partial sums in chunk order, or the far kernel's own row) plus its near-pair records
// in element order, stored at the point's place in the caller's order.  The same operations
// in the same order as the separate chunk reduction, ordered sums and unordering, in one pass.
__global__ void finish_points_kernel(const uint32_t* __restrict__ start, const uint32_t* __restrict__ count,
                                     int64_t n, const double* __restrict__ res, int rec, int rows, int prow,
                                     const double* __restrict__ partial, int n_split, const double* __restrict__ far,
                                     double K, const uint32_t* __restrict__ perm, double* __restrict__ d0,
                                     double* __restrict__ d1, const DevCounters* __restrict__ ctr,
                                     DevCounters* __restrict__ ctr_out)
{
#pragma clang fp contract(off)
    copy_counters(ctr, ctr_out);
    // one thread per (row, point)
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)rows * n) return;
    const int c = (int)(i / n);
    const int64_t p = i - (int64_t)c * n;
    const uint32_t s = start[p], k = count[p];
    double v;
    if (n_split > 1) {  // the row summed in chunk order
        v = 0.0;
#pragma unroll 4
        for (int j = 0; j < n_split; ++j) v += partial[((int64_t)j * prow + c) * n + p];
        v = K * v;
    } else {
        v = far[(int64_t)c * n + p];
    }
    if (k > 0) {
        double acc = 0.0;
        for (uint32_t m = 0; m < k; ++m) acc += res[(unsigned long long)(s + m) * rec + c];
        v = v + acc;
    }
    const int64_t q = perm ? (int64_t)perm[p] : p;
    (c == 0 ? d0 : d1 + (int64_t)(c - 1) * n)[q] = v;
}

__device__ __forceinline__ double dot3(const double* a, const double* b) { return fma(a[0], b[0], fma(a[1], b[1], a[2] * b[2])); }

// Squared distance from p to the triangle (0, b, c) (p, b, c relative to its first vertex):
// the closest point by the Voronoi regions of the vertices, the edges and the face.
__device__ __forceinline__ double triangle_distance2(const double (&p)[3], const double* b, const double* c)
{
    double q[3];  // the closest point
    const double d1 = dot3(b, p), d2 = dot3(c, p);
    const double bp[3] = { p[0] - b[0], p[1] - b[1], p[2] - b[2] };
    const double d3 = dot3(b, bp), d4 = dot3(c, bp);
    const double cp[3] = { p[0] - c[0], p[1] - c[1], p[2] - c[2] };
    const double d5 = dot3(b, cp), d6 = dot3(c, cp);
    const double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
    if (d1 <= 0.0 && d2 <= 0.0) {
        q[0] = q[1] = q[2] = 0.0;
    } else if (d3 >= 0.0 && d4 <= d3) {
        q[0] = b[0]; q[1] = b[1]; q[2] = b[2];
    } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        const double t = d1 / (d1 - d3);
        q[0] = t * b[0]; q[1] = t * b[1]; q[2] = t * b[2];
    } else if (d6 >= 0.0 && d5 <= d6) {
        q[0] = c[0]; q[1] = c[1]; q[2] = c[2];
    } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        const double t = d2 / (d2 - d6);
        q[0] = t * c[0]; q[1] = t * c[1]; q[2] = t * c[2];
    } else if (va <= 0.0 && d4 - d3 >= 0.0 && d5 - d6 >= 0.0) {
        const double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        q[0] = fma(t, c[0] - b[0], b[0]); q[1] = fma(t, c[1] - b[1], b[1]); q[2] = fma(t, c[2] - b[2], b[2]);
    } else {
        const double den = 1.0 / (va + vb + vc), v = vb * den, w = vc * den;
        q[0] = fma(v, b[0], w * c[0]); q[1] = fma(v, b[1], w * c[1]); q[2] = fma(v, b[2], w * c[2]);
    }
    const double r[3] = { p[0] - q[0], p[1] - q[1], p[2] - q[2] };
    return dot3(r, r);
}

// Cost class of a near pair (higher = more subdivision leaves expected): 4 steps per octave of
// L / d, d the distance from the point to the element (its closest point), the costliest step
// where d vanishes without the point lying on the element.  Deep pairs (d <= L / 16: a near
// region at some five levels or more) come first, walked by a wavefront each; then the
// others.  Rectangles come before triangles in each group: the near kernel's wavefronts take
// windows of the order far apart in time, and a wavefront whose lanes mix both kinds runs
// both rule loops.
__device__ __forceinline__ int cost_class(const double* __restrict__ pts, int64_t n, const Elements& el, NearPair pr)
{
    const int64_t e = pr.elem, p = pr.point;
    const bool tri = e < el.n_tri;
    const double X[3] = { pts[p], pts[n + p], pts[2 * n + p] };
    double G[9], P[3];
    if (point_on_element(el, e, tri, X, G, P)) return kOnElementClass;
    double d2;
    if (tri) {
        const double b[3] = { G[3] - G[0], G[4] - G[1], G[5] - G[2] };
        const double c[3] = { G[6] - G[0], G[7] - G[1], G[8] - G[2] };
        d2 = triangle_distance2(P, b, c);
    } else {  // P0 + u e1 + v e2 with u, v clamped to [0, 1] (orthogonal sides)
        const double* e1 = G + 3;
        const double* e2 = G + 6;
        const double u = fmin(fmax(dot3(P, e1) / dot3(e1, e1), 0.0), 1.0);
        const double v = fmin(fmax(dot3(P, e2) / dot3(e2, e2), 0.0), 1.0);
        const double r[3] = { P[0] - u * e1[0] - v * e2[0], P[1] - u * e1[1] - v * e2[1], P[2] - u * e1[2] - v * e2[2] };
        d2 = dot3(r, r);
    }
    const double L = el.L[e];
    int c = 63;
    if (d2 > 1e-24 * L * L) c = min(63, max(1, (int)floor(4.0 * (log2(L) - 0.5 * log2(d2)) + 16.0)));
    return (c >= kDeepCost ? kDeepClass : 0) + (tri ? 0 : 64) + c;
}

// Clears the per-class counts and cursors (buckets) and the per-point counts and cursors.
__global__ void clear_order_kernel(uint32_t* __restrict__ buckets, uint32_t* __restrict__ count,
                                   uint32_t* __restrict__ cursor, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        count[i] = 0u;
        cursor[i] = 0u;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < 3 * kCostClasses; i += kBlock) buckets[i] = 0u;
}

// An evaluation's first launch: its device counters, and the clears of the near stage's order
// (per-point counts and cursors, per-class buckets), which nothing touches before that stage.
__global__ void clear_call_kernel(DevCounters* __restrict__ ctr, uint32_t* __restrict__ buckets,
                                  uint32_t* __restrict__ count, uint32_t* __restrict__ cursor, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        count[i] = 0u;
        cursor[i] = 0u;
    }
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < 3 * kCostClasses; i += kBlock) buckets[i] = 0u;
        unsigned long long* c = reinterpret_cast<unsigned long long*>(ctr);
        for (int i = threadIdx.x; i < (int)(sizeof(DevCounters) / sizeof(unsigned long long)); i += kBlock) c[i] = 0ull;
    }
}

// The class of every list index and the per-class counts (per-workgroup histograms in LDS,
// one global atomic per class and workgroup); the near pairs of each point.
__global__ void cost_count_kernel(const NearPair* __restrict__ list, const DevCounters* __restrict__ ctr,
                                  unsigned long long cap, const double* __restrict__ pts, int64_t n, Elements el,
                                  uint8_t* __restrict__ cost, uint32_t* __restrict__ buckets,
                                  uint32_t* __restrict__ count)
{
    __shared__ uint32_t hist[kCostClasses];
    hist[threadIdx.x] = 0u;  // kBlock == kCostClasses
    __syncthreads();
    const unsigned long long total = pair_total(ctr, cap);
    for (unsigned long long i = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (unsigned long long)gridDim.x * kBlock) {
        const NearPair pr = list[i];
        const int c = cost_class(pts, n, el, pr);
        cost[i] = (uint8_t)c;
        atomicAdd(&hist[c], 1u);
        atomicAdd(&count[pr.point], 1u);
    }
    __syncthreads();
    if (hist[threadIdx.x]) atomicAdd(&buckets[threadIdx.x], hist[threadIdx.x]);
}

// Both scatters of the list.  By cost: order[start[class] + rank] = list index, ranks within
// a workgroup's chunk from LDS atomics, one global atomic per class and chunk (each workgroup
// forms the class starts itself, most expensive class first; the first one stores them).  By
// point: each pair to its point's segment (start from the scan of the per-point counts),
// with its list index.
constexpr int kCostItems = 8;  // list entries per thread and chunk
__global__ void scatter_kernel(const NearPair* __restrict__ list, const DevCounters* __restrict__ ctr,
                               unsigned long long cap, const uint8_t* __restrict__ cost,
                               uint32_t* __restrict__ buckets, uint32_t* __restrict__ order,
                               NearPair* __restrict__ opair,
                               const uint32_t* __restrict__ start, uint32_t* __restrict__ cursor,
                               NearPair* __restrict__ grouped, uint32_t* __restrict__ origin)
{
    __shared__ uint32_t hist[kCostClasses], base[kCostClasses], first[kCostClasses];
    __shared__ uint32_t wave_total[kWavesPerBlock];
    {
        // the class starts: the counts of all higher classes (a suffix sum, by the wavefronts'
        // shuffles and their totals)
        const uint32_t v = buckets[threadIdx.x];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        uint32_t inc = v;  // v and the counts of the higher classes of this wavefront
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_down(inc, o);
            if (lane + o < 64) inc += t;
        }
        if (lane == 0) wave_total[wave] = inc;
        __syncthreads();
        uint32_t st = inc - v;
        for (int w = wave + 1; w < kWavesPerBlock; ++w) st += wave_total[w];
        first[threadIdx.x] = st;
        if (blockIdx.x == 0) buckets[kCostClasses + threadIdx.x] = st;
        __syncthreads();
    }
    const unsigned long long total = pair_total(ctr, cap);
    const unsigned long long chunk = (unsigned long long)kBlock * kCostItems;
    for (unsigned long long c0 = (unsigned long long)blockIdx.x * chunk; c0 < total;
         c0 += (unsigned long long)gridDim.x * chunk) {
        hist[threadIdx.x] = 0u;
        __syncthreads();
        int cls[kCostItems];
        uint32_t rank[kCostItems];
        NearPair prs[kCostItems];
#pragma unroll
        for (int k = 0; k < kCostItems; ++k) {
            const unsigned long long i = c0 + (unsigned long long)k * kBlock + threadIdx.x;
            cls[k] = -1;
            if (i < total) {
                cls[k] = cost[i];
                rank[k] = atomicAdd(&hist[cls[k]], 1u);
                const NearPair pr = list[i];
                prs[k] = pr;
                const uint32_t pos = start[pr.point] + atomicAdd(&cursor[pr.point], 1u);
                grouped[pos] = pr;
                origin[pos] = (uint32_t)i;
            }
        }
        __syncthreads();
        const uint32_t cnt = hist[threadIdx.x];
        base[threadIdx.x] = cnt ? first[threadIdx.x] + atomicAdd(&buckets[2 * kCostClasses + threadIdx.x], cnt) : 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCostItems; ++k) {
            const unsigned long long i = c0 + (unsigned long long)k * kBlock + threadIdx.x;
            if (cls[k] >= 0) {
                order[base[cls[k]] + rank[k]] = (uint32_t)i;
                opair[base[cls[k]] + rank[k]] = prs[k];
            }
        }
        __syncthreads();
    }
}

unsigned grid_for(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}


}  // namespace

hipError_t clear_call(DevCounters* ctr, const NearWork& w, int64_t n, hipStream_t s)
{
    static_assert(sizeof(DevCounters) % sizeof(unsigned long long) == 0, "counters are 64-bit words");
    clear_call_kernel<<<grid_for(std::max<int64_t>(n, 1)), kBlock, 0, s>>>(ctr, w.buckets, w.count, w.cursor,
                                                                           std::max<int64_t>(n, 0));
    return hipGetLastError();
}

void near_work_free(NearWork& w)
{
    for (void* ptr : { (void*)w.count, (void*)w.start, (void*)w.cursor, (void*)w.grouped, (void*)w.origin,
                       (void*)w.sorted, (void*)w.slot, (void*)w.res, (void*)w.cost, (void*)w.order, (void*)w.opair,
                       (void*)w.buckets, w.temp })
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
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.cost), npairs);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.order), npairs * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.opair), npairs * sizeof(NearPair));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&w.buckets), 3 * kCostClasses * sizeof(uint32_t));
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
                      const double* pts, const Elements& el, const NearWork& w, bool cleared, hipStream_t s)
{
    static_assert(kBlock == kCostClasses, "one thread per cost class");
    if (n <= 0) {  // no pairs: the walk's share (near_walk_end) is empty
        if (!cleared) clear_order_kernel<<<1, kBlock, 0, s>>>(w.buckets, w.count, w.cursor, 0);
        return hipGetLastError();
    }
    const unsigned lgrid = grid_for((int64_t)std::min<unsigned long long>(cap, 1ull << 40));
    if (!cleared) clear_order_kernel<<<grid_for(n), kBlock, 0, s>>>(w.buckets, w.count, w.cursor, n);
    cost_count_kernel<<<lgrid, kBlock, 0, s>>>(list, ctr, cap, pts, n, el, w.cost, w.buckets, w.count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = w.temp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(w.temp, bytes, w.count, w.start, (int)n, s);
    if (e != hipSuccess) return e;
    scatter_kernel<<<std::max(1u, lgrid / kCostItems), kBlock, 0, s>>>(list, ctr, cap, w.cost, w.buckets, w.order,
                                                                       w.opair, w.start, w.cursor, w.grouped,
                                                                       w.origin);
    const int64_t blocks = (n + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    rank_sort_kernel<<<(unsigned)blocks, kBlock, 0, s>>>(w.start, w.count, n, w.grouped, w.origin, w.sorted, w.slot);
    return hipGetLastError();
}

hipError_t near_finish(const NearWork& w, int64_t n, int mode, int rows, const double* partial, int n_split,
                       int prow, const double* far, double K, const uint32_t* perm, double* d0, double* d1,
                       const DevCounters* ctr, DevCounters* ctr_out, hipStream_t s)
{
    if (n <= 0 || rows <= 0) return hipSuccess;
    if (mode == kNearColloc) return hipErrorInvalidValue;
    const int64_t threads = (int64_t)rows * n;
    if ((threads + kBlock - 1) / kBlock > 0x7fffffff) return hipErrorInvalidValue;
    finish_points_kernel<<<(unsigned)((threads + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        w.start, w.count, n, w.res, mode == kNearGrad ? 6 : 4, rows, prow, partial, n_split, far, K, perm, d0, d1,
        ctr, ctr_out);
    return hipGetLastError();
}

hipError_t near_reduce(const NearWork& w, int64_t n, int mode, double* phi, double* E,
                       double* G, const double* q, int64_t ne, int n_rhs, double K, const DevCounters* ctr, DevCounters* ctr_out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    reduce_pairs_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        w.start, w.count, n, w.sorted, w.res, mode, phi, E, G, q, ne, n_rhs, K, ctr, ctr_out);
    return hipGetLastError();
}

}  // namespace bemc
