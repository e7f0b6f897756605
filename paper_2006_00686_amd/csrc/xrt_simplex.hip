// The transform on a simplex basis for gfx950: forward projection and its transpose
// (ray-driven scatter with float atomics).  The per-ray work is the slab walk of
// xrt_walk.h; each hit unit's piece of the ray is cut into its simplex pieces by
// xrt_simplex.h.  One lane per ray; images hold S = 2 (2D) or 6 (3D) float32 values per
// unit ([batch][nz][ny][nx][S]); line integrals accumulate in FP64.
#include "xrt_simplex.h"

namespace xrt {
namespace {

constexpr int kBlock = 256;

template <int DIM>
struct SimplexFwd : SimplexWalker<DIM, SimplexFwd<DIM>> {
    const float* img;
    double acc = 0.0;
    __device__ __forceinline__ void simplex(int64_t T, double l) { acc = fma((double)img[T], l, acc); }
};

template <int DIM>
struct SimplexScatter : SimplexWalker<DIM, SimplexScatter<DIM>> {
    float* img;
    double gw;
    __device__ __forceinline__ void simplex(int64_t T, double l) { unsafeAtomicAdd(img + T, (float)(gw * l)); }
};

template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_forward_simplex(DevPlan P, const float* __restrict__ img,
                                                             float* __restrict__ sino)
{
    const int32_t r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (r >= P.n_rays) return;
    const int64_t b = blockIdx.y;
    Ray R;
    make_ray<DIM, MODE>(P, r, R);
    SimplexFwd<DIM> v;
    simplex_walker_init(v, P, R);
    v.img = img + b * P.n_units * kSimplices<DIM>;
    walk<DIM>(P, R, v);
    sino[b * P.n_rays + r] = (float)(v.acc * R.scale);
}

template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_adjoint_simplex(DevPlan P, const float* __restrict__ sino,
                                                             float* __restrict__ img)
{
    const int32_t r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (r >= P.n_rays) return;
    const int64_t b = blockIdx.y;
    const float g = sino[b * P.n_rays + r];
    if (g == 0.0f) return;
    Ray R;
    make_ray<DIM, MODE>(P, r, R);
    SimplexScatter<DIM> v;
    simplex_walker_init(v, P, R);
    v.img = img + b * P.n_units * kSimplices<DIM>;
    v.gw = (double)g * R.scale;
    walk<DIM>(P, R, v);
}

template <template <int, int> class K, class... Args>
xrt_status dispatch_simplex(const DevPlan& P, dim3 grid, hipStream_t s, Args... args)
{
    auto go = [&](auto kern) -> xrt_status {
        hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, P, args...);
        return hip_fail(hipGetLastError(), "simplex kernel launch");
    };
    if (P.dim == 2) {
        switch (P.mode) {
            case MODE_PARALLEL: return go(K<2, MODE_PARALLEL>::fn());
            case MODE_DIVERGENT: return go(K<2, MODE_DIVERGENT>::fn());
            case MODE_ARC: return go(K<2, MODE_ARC>::fn());
            default: return go(K<2, MODE_LIST>::fn());
        }
    }
    switch (P.mode) {
        case MODE_PARALLEL: return go(K<3, MODE_PARALLEL>::fn());
        case MODE_DIVERGENT: return go(K<3, MODE_DIVERGENT>::fn());
        case MODE_ARC: return go(K<3, MODE_ARC>::fn());
        default: return go(K<3, MODE_LIST>::fn());
    }
}

template <int D, int M> struct SFwdK { static auto fn() { return k_forward_simplex<D, M>; } };
template <int D, int M> struct SAdjK { static auto fn() { return k_adjoint_simplex<D, M>; } };

}  // namespace

xrt_status launch_forward_simplex(const xrt_plan* p, const float* img, float* sino, int batch, hipStream_t s)
{
    const DevPlan& P = p->dp;
    const dim3 grid((unsigned)((P.n_rays + kBlock - 1) / kBlock), (unsigned)batch);
    return dispatch_simplex<SFwdK>(P, grid, s, img, sino);
}

xrt_status launch_adjoint_simplex(const xrt_plan* p, const float* sino, float* img, int batch, hipStream_t s)
{
    const DevPlan& P = p->dp;
    const int64_t n = P.n_units * (P.dim == 3 ? 6 : 2) * (int64_t)batch;
    xrt_status st = launch_fill_zero(img, n, s);
    if (st != XRT_OK) return st;
    const dim3 grid((unsigned)((P.n_rays + kBlock - 1) / kBlock), (unsigned)batch);
    return dispatch_simplex<SAdjK>(P, grid, s, sino, img);
}

}  // namespace xrt
