// Batches of plans (one persistent forward launch over all members) and the launch-shape
// settings of a plan.
#include <algorithm>
#include <cmath>
#include <new>

#include "xrt_internal.h"

using namespace xrt;

namespace {

// Relative cost of one ray of a plan: the number of unit faces a ray crossing the whole
// grid passes, so the queue starts with the members whose rays are longest.
double ray_cost(const DevPlan& P) { return (double)P.nx + P.ny + (P.dim == 3 ? P.nz : 0); }

void free_batch(xrt_batch* b)
{
    if (b->d_plans) (void)hipFree(b->d_plans);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
}

}  // namespace

extern "C" {

xrt_status xrt_plan_set_tuning(xrt_plan* plan, const xrt_tuning* t)
{
    if (!plan || !t) { set_error("null argument"); return XRT_E_ARG; }
    if (!(t->packet_cols == 0 || t->packet_cols == 1 || t->packet_cols == 16 || t->packet_cols == 32 ||
          t->packet_cols == 64) ||
        (t->xcd_remap != 0 && t->xcd_remap != 1)) {
        set_error("packet_cols must be 0, 1, 16, 32 or 64 and xcd_remap 0 or 1");
        return XRT_E_ARG;
    }
    const int32_t pc = plan->dp.mode == MODE_LIST ? 0 : t->packet_cols;
    if (pc == 1 && plan->dp.dim == 3 && plan->d_imgZ == nullptr) {
        // column packets read a z-fastest copy of the image (plan workspace, kept)
        DeviceGuard guard(plan->device);
        void* ws = nullptr;
        if (hipMalloc(&ws, (size_t)plan->dp.n_units * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of the %lld-float column-packet workspace failed", (long long)plan->dp.n_units);
            return XRT_E_NOMEM;
        }
        plan->d_imgZ = (float*)ws;
    }
    plan->dp.packet_cols = pc;
    plan->dp.xcd_remap = t->xcd_remap;
    return XRT_OK;
}

xrt_status xrt_plan_get_tuning(const xrt_plan* plan, xrt_tuning* t)
{
    if (!plan || !t) { set_error("null argument"); return XRT_E_ARG; }
    t->packet_cols = plan->dp.packet_cols;
    t->xcd_remap = plan->dp.xcd_remap;
    return XRT_OK;
}

xrt_status xrt_batch_create(xrt_plan* const* plans, int32_t n, xrt_batch** out)
{
    if (!out) { set_error("out is NULL"); return XRT_E_ARG; }
    *out = nullptr;
    if (!plans || n < 1 || n > kMaxBatch) {
        set_error("a batch holds 1 to %d plans", kMaxBatch);
        return XRT_E_ARG;
    }
    for (int32_t m = 0; m < n; ++m) {
        if (!plans[m]) { set_error("plan %d is NULL", m); return XRT_E_ARG; }
        const DevPlan &P = plans[m]->dp, &P0 = plans[0]->dp;
        if (plans[m]->device != plans[0]->device || P.dim != P0.dim || P.mode != P0.mode || P.mode == MODE_LIST) {
            set_error("batch members must share the device, the dimension and the ray mode (no ray lists)");
            return XRT_E_UNSUPPORTED;
        }
    }
    xrt_batch* b = new (std::nothrow) xrt_batch{};
    if (!b) { set_error("host allocation failed"); return XRT_E_NOMEM; }
    b->device = plans[0]->device;
    b->n = n;
    for (int32_t m = 0; m < n; ++m) {
        b->plans[m] = plans[m];
        b->hp[m] = plans[m]->dp;
        b->order[m] = m;
    }
    std::stable_sort(b->order, b->order + n,
                     [&](int32_t a, int32_t c) { return ray_cost(b->hp[a]) > ray_cost(b->hp[c]); });
    DeviceGuard guard(b->device);
    if (!guard.ok) { delete b; set_error("hipSetDevice(%d) failed", plans[0]->device); return XRT_E_HIP; }
    if (hipMalloc((void**)&b->d_plans, sizeof(DevPlan) * n) != hipSuccess ||
        hipMalloc((void**)&b->d_counter, sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        free_batch(b);
        set_error("device allocation for the batch failed");
        return XRT_E_NOMEM;
    }
    xrt_status st = hip_fail(hipMemcpy(b->d_plans, b->hp, sizeof(DevPlan) * n, hipMemcpyHostToDevice), "hipMemcpy");
    if (st != XRT_OK) { free_batch(b); return st; }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        cus = 256;
    }
    b->grid = (uint32_t)cus * forward_batch_blocks_per_cu();
    *out = b;
    return XRT_OK;
}

xrt_status xrt_batch_destroy(xrt_batch* batch)
{
    if (!batch) return XRT_OK;
    DeviceGuard guard(batch->device);
    (void)hipDeviceSynchronize();
    free_batch(batch);
    return XRT_OK;
}

xrt_status xrt_batch_forward(xrt_batch* batch, const float* const* d_imgs, float* const* d_sinos, void* stream)
{
    if (!batch || !d_imgs || !d_sinos) { set_error("null argument"); return XRT_E_ARG; }
    float* imgT[kMaxBatch];
    float* imgZ[kMaxBatch];
    for (int32_t m = 0; m < batch->n; ++m) {
        if (!d_imgs[m] || !d_sinos[m]) { set_error("null buffer for member %d", m); return XRT_E_ARG; }
        imgT[m] = batch->plans[m]->d_imgT;
        imgZ[m] = batch->plans[m]->d_imgZ;
    }
    DeviceGuard guard(batch->device);
    return launch_forward_batch(batch->hp, imgT, imgZ, batch->d_plans, batch->n, batch->order, d_imgs, d_sinos,
                                batch->d_counter, batch->grid, (hipStream_t)stream);
}

xrt_status xrt_batch_adjoint(xrt_batch* batch, const float* const* d_sinos, float* const* d_imgs, int32_t mode,
                             void* stream)
{
    if (!batch || !d_imgs || !d_sinos) { set_error("null argument"); return XRT_E_ARG; }
    for (int32_t m = 0; m < batch->n; ++m)
        if (!d_imgs[m] || !d_sinos[m]) { set_error("null buffer for member %d", m); return XRT_E_ARG; }
    for (int32_t k = 0; k < batch->n; ++k) {
        const int32_t m = batch->order[k];
        xrt_status st = xrt_adjoint(batch->plans[m], d_sinos[m], d_imgs[m], 1, mode, stream);
        if (st != XRT_OK) return st;
    }
    return XRT_OK;
}

}  // extern "C"
