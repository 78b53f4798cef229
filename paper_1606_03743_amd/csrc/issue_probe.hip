// Issue rates of the instruction classes the far-field kernels are made of, measured on the
// device: the FP64 fused multiply-add, the FP64 reciprocal square root, a stream of one
// reciprocal square root per eight FMAs, and the same three in FP32 (unpacked).  The
// benchmark uses them to state the ceiling of a kernel's instruction mix beside the published
// peak.  Measurement code only, built as a library of its own: no part of the evaluation path
// calls it.
//
// Each kernel runs 16 independent chains per lane (enough to cover the latency of every
// instruction) over 4,096 workgroups of 256, and stores one value per lane so that nothing is
// optimised away.  A rate is wavefront instructions per second, from HIP events around the
// second of two launches.
#include <hip/hip_runtime.h>

namespace {

constexpr int kChains = 16;
constexpr int kBlocks = 4096;
constexpr int kThreads = 256;
constexpr int kIters = 2000;

template <typename T>
__device__ __forceinline__ T rsq(T x);
template <>
__device__ __forceinline__ double rsq<double>(double x) { return __builtin_amdgcn_rsq(x); }
template <>
__device__ __forceinline__ float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// kind 0: x = x a + b; kind 1: x = rsq(x); kind 2: x = rsq(x), then eight times x = x a + b
template <typename T, int KIND>
__global__ __launch_bounds__(kThreads) void chains_kernel(T* out, int iters, T a, T b)
{
    T x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = T(1.5) + T(1e-3) * T(k) + T(1e-6) * T(threadIdx.x);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            if (KIND == 0) {
                x[k] = fma(x[k], a, b);
            } else {
                T y = rsq<T>(x[k]);
                if (KIND == 2) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) y = fma(y, a, b);
                }
                x[k] = y;
            }
        }
    }
    T s = T(0);
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

template <typename T, int KIND>
hipError_t time_kernel(T* out, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double& rate)
{
    // the mixed stream runs a quarter of the iterations, nine instructions each
    const int iters = KIND == 2 ? kIters / 4 : kIters;
    const double per_lane = (double)iters * kChains * (KIND == 2 ? 9.0 : 1.0);
    float ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {
        hipError_t e = hipEventRecord(e0, st);
        if (e != hipSuccess) return e;
        chains_kernel<T, KIND><<<kBlocks, kThreads, 0, st>>>(out, iters, T(0.999999), T(1e-7));
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
    }
    const double waves = (double)kBlocks * kThreads / 64.0;
    rate = ms > 0.0f ? waves * per_lane / (1e-3 * ms) : 0.0;
    return hipSuccess;
}

}  // namespace

// rates[6], wavefront instructions per second: FP64 FMA, FP64 reciprocal square root, FP64
// one-in-nine stream, FP32 FMA, FP32 reciprocal square root, FP32 one-in-nine stream.
// Runs on `device` (made current for the call; the previous current device is restored).
// Returns 0, or -1 for a null pointer, or the HIP error code of the failing call.
extern "C" int issue_probe_rates(int device, double* rates)
{
    if (!rates) return -1;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    if (e != hipSuccess) return (int)e;
    void* out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipMalloc(&out, (size_t)kBlocks * kThreads * sizeof(double));
    if (e == hipSuccess) e = hipStreamCreate(&st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double* d = static_cast<double*>(out);
    float* f = static_cast<float*>(out);
    if (e == hipSuccess) e = time_kernel<double, 0>(d, st, e0, e1, rates[0]);
    if (e == hipSuccess) e = time_kernel<double, 1>(d, st, e0, e1, rates[1]);
    if (e == hipSuccess) e = time_kernel<double, 2>(d, st, e0, e1, rates[2]);
    if (e == hipSuccess) e = time_kernel<float, 0>(f, st, e0, e1, rates[3]);
    if (e == hipSuccess) e = time_kernel<float, 1>(f, st, e0, e1, rates[4]);
    if (e == hipSuccess) e = time_kernel<float, 2>(f, st, e0, e1, rates[5]);
    if (st) (void)hipStreamSynchronize(st);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (st) (void)hipStreamDestroy(st);
    if (out) (void)hipFree(out);
    (void)hipSetDevice(prev);
    return (int)e;
}
