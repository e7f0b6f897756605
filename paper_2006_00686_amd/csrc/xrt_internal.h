// Internal types shared by the host side (plan construction) and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/xrt.h"

namespace xrt {

// How a ray (point p, direction d, both FP64, physical units) is built from its
// (view, row, col) in the kernels.  Every geometry of the paper reduces to one of these
// (Sec. 4.2: the transform depends only on each ray's geometric parameters).
enum RayMode : int32_t {
    MODE_PARALLEL = 0,    // p = A + u B + v C,  d = E            (PAR2D, PAR3D)
    MODE_DIVERGENT = 1,   // p = A (source),     d = E + u B + v C (flat fan / cone)
    MODE_ARC = 2,         // p = A, d = cb (ca E + sa B) + sb C    (equiangular fan / cone)
    MODE_LIST = 3         // p, d read per ray from a table        (ray lists)
};

struct ViewGeom {         // FP64 per-view vectors, see RayMode
    double A[3], B[3], C[3], E[3];
};

// Everything a projection kernel needs, passed by value as a kernel argument.
constexpr int kMaxBatch = 32;   // members of one xrt_batch
// floats after the gather's transposed sinogram: its 8-byte row-pair loads may read one
// element past the last ray (the value is then discarded)
constexpr int kGatherPad = 64;

struct DevPlan {
    int32_t dim;          // 2 or 3
    int32_t mode;         // RayMode
    int32_t nx, ny, nz;   // nz = 1 in 2D
    int32_t n_views, n_rows, n_cols;
    int64_t n_rays;
    int64_t n_units;
    // index-space transform: q = (p_x*ax + bx, -p_y*ay + by, -p_z*az + bz),
    // direction w = (d_x*ax, -d_y*ay, -d_z*az); unit (k,j,i) = [i,i+1)x[j,j+1)x[k,k+1)
    double ax, bx, ay, by, az, bz;
    double du, ubase, dv, vbase;      // u = c*du + ubase, v = r*dv + vbase
    double sdd;                       // source-to-detector distance (flat detectors)
    // physical unit boundaries: x of index plane 0, y of row plane 0 (top), z of layer
    // plane 0 (top); unit side lengths
    double px0, py0, pz0, pdx, pdy, pdz;
    const ViewGeom* views;            // [n_views]
    const double* col_cs;             // MODE_ARC: [n_cols][2] (cos, sin) of the column angle
    const double* row_cs;             // MODE_ARC: [n_rows][2]
    const double* rays;               // MODE_LIST: [n_rays][6] (p, d)
    // 2D gather: (|d|/d_x, |d|/d_y) of every (view, column) ray (MODE_DIVERGENT, MODE_ARC:
    // [n_views][n_cols][2]) or of every view's common direction (MODE_PARALLEL:
    // [n_views][2]).  A zero component (ray parallel to that axis's grid lines) is 0 for
    // parallel beams, and +1e300 (x) / -1e300 (y) for rays from a source, where it makes
    // the clip of a unit in front of the source the half-open membership test
    const double* ray2d;
    // half-width in bins by which the gathers widen a candidate column range: covers the
    // hardware FP64 reciprocal (relative error below 2^-20) at the largest |u| of the
    // detector
    double uslack;
    // 2D gather, rays from a flat-detector source: candidate bins from the pixel centre's
    // detector coordinate u_c and the half-width (sdd^2 + max(g2_umax2, u_c^2)) g2_r / D of
    // the shadow of the pixel's circumscribed disc (D = E . (centre - source)); g2_r = 0:
    // use the four corners instead
    double g2_umax2, g2_r;
    // forward launch shape (tuning; no effect on results): packet_cols = 0 enumerates
    // rays linearly, 64 / 32 / 16 gives each wavefront a packet of packet_cols detector
    // columns x (64 / packet_cols) rows of one view; xcd_remap = 1 hands each XCD a
    // contiguous range of packets (workgroups are dealt to the 8 XCDs round robin)
    int32_t packet_cols = 0;
    int32_t xcd_remap = 0;
    // 3D forward projections (plain and attenuated): walk form (0 flat, 1 nested; no
    // effect on results), set at plan creation
    int32_t nest_z = 0;
};

}  // namespace xrt

struct xrt_plan {
    int device;
    xrt::DevPlan dp;
    void* d_views;
    void* d_col;
    void* d_row;
    void* d_rays;
    void* d_ray2d;      // DevPlan::ray2d (2D plans with the gather), or NULL
    int32_t kind;
    // voxel-driven cone adjoint (flat detector): per-row 1/v table and a sinogram
    // workspace [view][col][row] of one batch member, owned by the plan
    void* d_invwz;
    float* d_gT;
    int32_t zero_row;   // index of a row with v = 0 (ray in a z plane), or -1
    int32_t gather_ok;  // every unit lies in front of every source position
    int32_t gather_nr;  // bound on the detector rows one voxel's shadow covers per column
    int32_t gather_lgs; // log2 of the gather's column slots per view (0..6)
    int32_t helical;    // the source moves along z between views
    double sz0;         // source height of the first view (of every view when !helical)
    // y-fastest copy of one image for the forward projection of views whose detector
    // u axis runs along y (owned by the plan; 2D plans use it for one image per call), or NULL
    float* d_imgT;
    // z-fastest copy ([y][x][z]) of one image for the column-packet launch shape
    // (packet_cols = 1: a wavefront takes 64 rows of one detector column), allocated when
    // that shape is selected, or NULL
    float* d_imgZ;
    int32_t gather2d_ok;   // 2D scan whose image lies in front of every source position
    // (f, mu) pairs of one image for the attenuated forward, allocated by its first call
    // (2 n_units floats), or NULL
    float* d_att;
};

// Several plans (same dimension and ray mode) projected together; the plans stay owned
// by the caller and must outlive the batch.  Their launch shapes are taken at creation.
struct xrt_batch {
    int device;
    int32_t n;
    xrt_plan* plans[xrt::kMaxBatch];
    xrt::DevPlan hp[xrt::kMaxBatch];        // snapshots of the plans' device descriptors
    int32_t order[xrt::kMaxBatch];          // queue order: longest rays first
    xrt::DevPlan* d_plans;                  // device copies of hp
    unsigned long long* d_counter;          // work-queue counter (reset by a kernel per launch)
    uint32_t grid;                          // persistent workgroups
};

namespace xrt {
// Host-side result of validating and expanding a grid + scan (device pointers unset).
struct HostTables {
    DevPlan dp;
    int32_t kind;
    std::vector<ViewGeom> views;
    std::vector<double> col, row, rays;
};

// Validate and expand in FP64 on the host (no HIP calls).
xrt_status build_tables(const xrt_grid* grid, const xrt_scan* scan, HostTables& out);

// Makes a device current for the lifetime of the guard, restoring the previous one.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Set by failing entry points; read by xrt_last_error().
void set_error(const char* fmt, ...);
xrt_status hip_fail(hipError_t e, const char* what);

// Launchers (xrt_project.hip).
// wt (optional): per-ray weights, wt_stride floats apart per image (0: shared)
xrt_status launch_forward(const xrt_plan* p, const float* img, float* sino, int batch,
                          hipStream_t s, const float* wt = nullptr, int64_t wt_stride = 0);
// One persistent launch over the members of a batch (host plan snapshots hp, device
// copies d_plans, queue order, per-member images and sinograms).
xrt_status launch_forward_batch(const DevPlan* hp, float* const* imgT, float* const* imgZ, const DevPlan* d_plans,
                                int32_t n, const int32_t* order, const float* const* imgs, float* const* sinos,
                                unsigned long long* counter, uint32_t grid, hipStream_t s);
xrt_status launch_transpose_xy(const DevPlan& P, const float* img, float* imgT, hipStream_t s);
xrt_status launch_transpose_zfast(const DevPlan& P, const float* img, float* imgZ, hipStream_t s);
xrt_status launch_forward_att(const xrt_plan* p, const float* img, const float* mu, int64_t mu_stride, float* sino,
                              int batch, hipStream_t s);
// muT: n_units floats of workspace for the map's y-fastest copy, or NULL
xrt_status launch_adjoint_att(const xrt_plan* p, const float* sino, const float* mu, int64_t mu_stride, float* img,
                              int batch, hipStream_t s, float* muT = nullptr);
uint32_t forward_batch_blocks_per_cu();
xrt_status launch_adjoint_scatter(const xrt_plan* p, const float* sino, float* img, int batch,
                                  hipStream_t s, const float* wt = nullptr, int64_t wt_stride = 0);
xrt_status launch_hit_counts(const xrt_plan* p, int64_t first, int64_t n, double eps,
                             int32_t* counts, hipStream_t s);
xrt_status launch_hits(const xrt_plan* p, int64_t first, int64_t n, double eps,
                       const int64_t* offsets, int32_t* idx, float* len, hipStream_t s);
xrt_status launch_fill_zero(float* dst, int64_t n, hipStream_t s);
// Simplex basis (xrt_simplex.hip): images of S = 2 (2D) or 6 (3D) values per unit.
xrt_status launch_forward_simplex(const xrt_plan* p, const float* img, float* sino, int batch, hipStream_t s);
xrt_status launch_adjoint_simplex(const xrt_plan* p, const float* sino, float* img, int batch, hipStream_t s);
// Voxel-driven gather adjoint for flat-detector cone beams (xrt_gather.hip).
xrt_status launch_adjoint_cone_gather(const xrt_plan* p, const float* sino, float* img, int batch,
                                      hipStream_t s, const float* wt = nullptr, int64_t wt_stride = 0);
// w[i] = exp(-x[i]) for n floats (in place allowed)
xrt_status launch_transmission(float* w, const float* x, int64_t n, hipStream_t s);
// batch-in-lanes forward (any 2D plan) and gather adjoint (2D gather plans): images
// [unit][image], sinograms [ray][image], 1 <= batch <= 64
xrt_status launch_forward_il(const xrt_plan* p, const float* img, float* sino, int batch, hipStream_t s);
xrt_status launch_adjoint_gather2d_il(const xrt_plan* p, const float* sino, float* img, int batch, hipStream_t s);
// attenuated forward reading (f, mu) pairs from p->d_att (8 n_units bytes within 32-bit
// offsets), one image after the other
xrt_status launch_forward_att_pairs(const xrt_plan* p, const float* img, const float* mu, int64_t mu_stride,
                                    float* sino, int batch, hipStream_t s);
// Voxel-driven gather adjoint for 2D scans (xrt_gather.hip).
xrt_status launch_adjoint_gather2d(const xrt_plan* p, const float* sino, float* img, int batch, hipStream_t s,
                                   const float* wt = nullptr, int64_t wt_stride = 0);
}  // namespace xrt
