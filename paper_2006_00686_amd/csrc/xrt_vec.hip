// Batched vector kernels of the iterative solvers (CGLS, Landweber): dot products with
// FP64 accumulation in a fixed order (deterministic) and updates whose scalar is a ratio
// of two device-resident FP64 values, so a solver iteration never waits on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "xrt_internal.h"

namespace xrt {
namespace {

constexpr int kVBlock = 256;
constexpr int kDotBlocks = 64;   // partial sums per batch member

// partial[b][blk] = sum over the block's grid-stride share of a[b][i] * b[b][i]
__global__ __launch_bounds__(kVBlock) void k_dot_partial(const float* __restrict__ a, const float* __restrict__ b,
                                                         int64_t n, double* __restrict__ partial)
{
    __shared__ double red[kVBlock];
    const int64_t off = (int64_t)blockIdx.y * n;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVBlock + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kVBlock)
        s = fma((double)a[off + i], (double)b[off + i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kVBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * kDotBlocks + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kDotBlocks) void k_dot_final(const double* __restrict__ partial, double* __restrict__ out)
{
    __shared__ double red[kDotBlocks];
    red[threadIdx.x] = partial[(int64_t)blockIdx.x * kDotBlocks + threadIdx.x];
    __syncthreads();
    for (int w = kDotBlocks / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// y[b] += sign * (num[b] / den[b]) * x[b]   (a zero denominator adds nothing)
__global__ __launch_bounds__(kVBlock) void k_axpy_ratio(const double* __restrict__ num, const double* __restrict__ den,
                                                        double sign, const float* __restrict__ x,
                                                        float* __restrict__ y, int64_t n)
{
    const int64_t off = (int64_t)blockIdx.y * n;
    const double d = den[blockIdx.y];
    const float a = d != 0.0 ? (float)(sign * num[blockIdx.y] / d) : 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
        y[off + i] = fmaf(a, x[off + i], y[off + i]);
}

// p[b] = s[b] + (num[b] / den[b]) * p[b]
__global__ __launch_bounds__(kVBlock) void k_xpby_ratio(const double* __restrict__ num, const double* __restrict__ den,
                                                        const float* __restrict__ s, float* __restrict__ p, int64_t n)
{
    const int64_t off = (int64_t)blockIdx.y * n;
    const double d = den[blockIdx.y];
    const float beta = d != 0.0 ? (float)(num[blockIdx.y] / d) : 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
        p[off + i] = fmaf(beta, p[off + i], s[off + i]);
}

// y = a x + b y
__global__ __launch_bounds__(kVBlock) void k_axpby(double a, const float* __restrict__ x, double b,
                                                   float* __restrict__ y, int64_t n)
{
    const float af = (float)a, bf = (float)b;
    for (int64_t i = (int64_t)blockIdx.x * kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
        y[i] = fmaf(af, x[i], bf * y[i]);
}

unsigned grid_for(int64_t n)
{
    int64_t g = (n + kVBlock - 1) / kVBlock;
    return (unsigned)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

// w[i] = exp(-x[i]): the transmission of a ray through an attenuation map, from its line
// integral (the PET weight of the generalised transform).
__global__ __launch_bounds__(kVBlock) void k_transmission(float* w, const float* x, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
        w[i] = expf(-x[i]);
}

// Partial sums of the allocation-free dot product: a file-scope device array (each GPU
// the library runs on holds its own copy, at its own address, until the process ends).
// Host code never names it as a kernel argument: kernels get the per-device address that
// hipGetSymbolAddress returns (scratch_on).
constexpr int32_t kNoAllocBatch = 1024;
static __device__ __align__(256) double scratch[kDotBlocks * kNoAllocBatch];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::atomic<double*> g_scratch_addr[kMaxDevices];

// Device address of `scratch` on device dev, looked up once per device with that device
// current.
xrt_status scratch_on(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d outside the %d devices the static scratch supports", dev, kMaxDevices);
        return XRT_E_ARG;
    }
    double* p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (p == nullptr) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_addr[dev].load(std::memory_order_relaxed);
        if (p == nullptr) {
            DeviceGuard guard(dev);
            if (!guard.ok) return hip_fail(hipErrorInvalidDevice, "hipSetDevice for the static scratch");
            void* addr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || addr == nullptr)
                return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress of the static scratch");
            p = static_cast<double*>(addr);
            g_scratch_addr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return XRT_OK;
}

// The two kernels of a batched dot product: 64 partial sums per member into work, then
// their fixed-order sum into out.
xrt_status launch_dot(int64_t n, int32_t batch, const float* a, const float* b, double* work, double* out,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks, (unsigned)batch), dim3(kVBlock), 0, s, a, b, n, work);
    hipLaunchKernelGGL(k_dot_final, dim3((unsigned)batch), dim3(kDotBlocks), 0, s, (const double*)work, out);
    return hip_fail(hipGetLastError(), "dot product launch");
}

}  // namespace

xrt_status launch_transmission(float* w, const float* x, int64_t n, hipStream_t s)
{
    if (n <= 0) return XRT_OK;
    const int64_t blocks = std::min<int64_t>((n + kVBlock - 1) / kVBlock, 65536);
    hipLaunchKernelGGL(k_transmission, dim3((unsigned)blocks), dim3(kVBlock), 0, s, w, x, n);
    return hip_fail(hipGetLastError(), "transmission launch");
}
}  // namespace xrt

using namespace xrt;

extern "C" {

xrt_status xrt_vec_dot(int64_t n, int32_t batch, const float* d_a, const float* d_b, double* d_work,
                       double* d_out, void* stream)
{
    if (!d_a || !d_b || !d_work || !d_out || n < 1 || batch < 1 || batch > 65535) {
        set_error("xrt_vec_dot: bad argument");
        return XRT_E_ARG;
    }
    return launch_dot(n, batch, d_a, d_b, d_work, d_out, (hipStream_t)stream);
}

xrt_status xrt_vec_dot_noalloc(int64_t n, int32_t batch, const float* d_a, const float* d_b, double* d_out,
                               void* stream)
{
    if (!d_a || !d_b || !d_out || n < 1 || batch < 1) {
        set_error("xrt_vec_dot_noalloc: bad argument");
        return XRT_E_ARG;
    }
    if (batch > kNoAllocBatch) {
        set_error("xrt_vec_dot_noalloc: batch %d exceeds the %d members of the static scratch", batch,
                  kNoAllocBatch);
        return XRT_E_SIZE;
    }
    const hipStream_t s = (hipStream_t)stream;
    int dev = -1;
    const hipError_t e = s != nullptr ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "xrt_vec_dot_noalloc: device of the stream");
    double* work = nullptr;
    const xrt_status st = scratch_on(dev, &work);
    if (st != XRT_OK) return st;
    DeviceGuard guard(dev);
    return launch_dot(n, batch, d_a, d_b, work, d_out, s);
}

xrt_status xrt_vec_axpy_ratio(int64_t n, int32_t batch, const double* d_num, const double* d_den, double sign,
                              const float* d_x, float* d_y, void* stream)
{
    if (!d_num || !d_den || !d_x || !d_y || n < 1 || batch < 1 || batch > 65535) {
        set_error("xrt_vec_axpy_ratio: bad argument");
        return XRT_E_ARG;
    }
    hipLaunchKernelGGL(k_axpy_ratio, dim3(grid_for(n), (unsigned)batch), dim3(kVBlock), 0, (hipStream_t)stream, d_num,
                       d_den, sign, d_x, d_y, n);
    return hip_fail(hipGetLastError(), "xrt_vec_axpy_ratio launch");
}

xrt_status xrt_vec_xpby_ratio(int64_t n, int32_t batch, const double* d_num, const double* d_den, const float* d_s,
                              float* d_p, void* stream)
{
    if (!d_num || !d_den || !d_s || !d_p || n < 1 || batch < 1 || batch > 65535) {
        set_error("xrt_vec_xpby_ratio: bad argument");
        return XRT_E_ARG;
    }
    hipLaunchKernelGGL(k_xpby_ratio, dim3(grid_for(n), (unsigned)batch), dim3(kVBlock), 0, (hipStream_t)stream, d_num,
                       d_den, d_s, d_p, n);
    return hip_fail(hipGetLastError(), "xrt_vec_xpby_ratio launch");
}

xrt_status xrt_vec_axpby(int64_t n, double a, const float* d_x, double b, float* d_y, void* stream)
{
    if (!d_x || !d_y || n < 1) {
        set_error("xrt_vec_axpby: bad argument");
        return XRT_E_ARG;
    }
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kVBlock), 0, (hipStream_t)stream, a, d_x, b, d_y, n);
    return hip_fail(hipGetLastError(), "xrt_vec_axpby launch");
}

}  // extern "C"
