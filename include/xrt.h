/*
 * xrt.h -- C ABI of libxrt.so, the MI355X (gfx950) implementation of the discrete
 * X-ray transform of a pixel/voxel image and of its adjoint.
 *
 * Reference: C. Chen, R. Wang, C. Bajaj, O. Oktem, "A Fast and Adaptive Algorithm to
 * Compute the X-ray Transform" (arXiv 2006.00686).
 *
 * What is computed (Introduction, eq. Xray_transform_image; Secs. 2.2.1 and 3.2.1):
 *   image f = sum_I f_I b_I with b_I the indicator of unit I (pixel or voxel);
 *   for every ray r,  g_r = sum_I f_I * len(r, I),  len = length of the ray inside
 *   unit I; the adjoint is f_I = sum_r g_r * len(r, I) (the transpose of the
 *   projection matrix, Introduction).  For each ray only the units that the paper's
 *   sufficient-and-necessary condition (eqs. conditions_2D_1, conditions_3D_1) admits
 *   are visited, and len = C_up - C_low (eqs. range_length, range_length_3D).
 *
 * Image layout: unit (k, j, i) has centre (cx + (i - (nx-1)/2) dx, cy + ((ny-1)/2 - j) dy,
 *   cz + ((nz-1)/2 - k) dz) (Secs. 2.1 and 3.1 with scale and offset, Sec. 4.2); the
 *   1D index is I = (k*ny + j)*nx + i (the paper's kNyNx + jNy + i for non-square
 *   grids).  Buffers are float32, contiguous, [batch][nz][ny][nx] ([batch][ny][nx] in 2D).
 * Sinogram layout: float32 [batch][view][row][col] (2D kinds: [batch][view][col];
 *   ray lists: [batch][ray]).
 * Grid-aligned rays (Sec. 4.1): a ray lying on a grid line/plane is given to the unit
 *   with the bigger 1D index (half-open units: x in [lo,hi), y in (lo,hi], z in (lo,hi]),
 *   also at the outer border of the image.
 *
 * Ownership: the caller allocates and owns every buffer passed in (device pointers
 *   marked d_, host pointers otherwise).  A plan owns its device tables; destroy frees
 *   them.  Host arrays referenced by xrt_scan are copied during xrt_plan_create.
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *   asynchronously; no call below synchronises the host except plan create/destroy and
 *   the first attenuated call (xrt_forward_attenuated or xrt_adjoint_attenuated) on a
 *   plan outside stream capture (it allocates that plan's workspace).  Nothing allocates
 *   during stream capture.
 * Concurrency: a plan's device workspaces (the cone gather's transposed sinogram, the
 *   y-fastest copy of an image, the attenuated transform's workspace) are shared by its
 *   calls, so
 *   calls on one plan must be ordered: one stream, or events between streams.  Different
 *   plans are independent.
 * Errors: every call returns an xrt_status.  Arguments are validated before any work
 *   is enqueued, so a failed call writes nothing.  XRT_E_HIP carries the HIP runtime
 *   message in xrt_last_error() (per thread).
 */
#ifndef XRT_H
#define XRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum xrt_status {
    XRT_OK = 0,
    XRT_E_ARG = -1,          /* null pointer, unknown enum value, batch < 1, bad ray range */
    XRT_E_GEOM = -2,         /* invalid geometry: non-positive sizes or spacings, SOD/SDD <= 0,
                                source inside the image box, non-finite parameters */
    XRT_E_SIZE = -3,         /* more than 2^29-4 units or 2^31-1 rays per image, or sizes beyond
                                the library's limits */
    XRT_E_HIP = -4,          /* a HIP runtime call failed (see xrt_last_error) */
    XRT_E_NOMEM = -5,        /* device or host allocation failed */
    XRT_E_UNSUPPORTED = -6   /* valid request that this build does not implement */
} xrt_status;

/* Scan kinds.  Bin centres are u_c = (c - (n_cols-1)/2)*du + u0 and
 * v_r = (r - (n_rows-1)/2)*dv + v0 (v grows with +z). */
typedef enum xrt_kind {
    XRT_PAR2D = 1,      /* 2D parallel beam (Sec. 2.2.1): view angle phi, bin = s          */
    XRT_FAN2D_FLAT = 2, /* equispaced fan (Sec. 2.2.2, eq. 2Dparalleltofan_2): view angle
                           alpha (source at sod*(-sin a, cos a)), flat detector at sdd     */
    XRT_FAN2D_ARC = 3,  /* equiangular fan (eq. 2Dparalleltofan): bin = gamma [rad]      */
    XRT_PAR3D = 4,      /* 3D parallel beam (Sec. 3.2.1): view (phi1, phi2), bins (s1, s2) */
    XRT_CONE_FLAT = 5,  /* equispaced circular/helical cone (Secs. 3.2.2-3.2.3): view
                           angle phi1' (source at -sod*(cos p, sin p, 0) + (0,0,H)),
                           flat detector at sdd with u along (-sin p, cos p, 0), v along z */
    XRT_CONE_ARC = 6,   /* equiangular cone: bins (alpha, beta) [rad]                     */
    XRT_RAYLIST2D = 7,  /* explicit rays (s, phi) (Sec. 4.2: any ray given by its
                           parallel-beam parameters)                                       */
    XRT_RAYLIST3D = 8   /* explicit rays (s1, s2, phi1, phi2)                              */
} xrt_kind;

typedef struct xrt_grid {
    int32_t nx, ny, nz;     /* units per axis; nz = 0 selects a 2D image               */
    double dx, dy, dz;      /* unit side lengths (> 0); dz ignored in 2D                 */
    double cx, cy, cz;      /* centre of the image box                                   */
} xrt_grid;

typedef struct xrt_scan {
    int32_t kind;                  /* xrt_kind                                         */
    int32_t n_views, n_rows, n_cols; /* n_rows = 1 for 2D kinds; ignored for ray lists  */
    double du, dv, u0, v0;         /* bin spacing and offset (radians for ARC kinds)    */
    double sod, sdd;               /* source-to-centre, source-to-detector (divergent)  */
    const double* view_angle;      /* host [n_views]: phi, alpha, phi1 or phi1'         */
    const double* view_z;          /* host [n_views] or NULL: source height H (cone);
                                      non-NULL makes the cone helical                  */
    const double* view_phi2;       /* host [n_views]: elevation phi2 (PAR3D only)       */
    const double* ray_params;      /* host [n_rays][2 or 4] (RAYLIST kinds only)        */
    int64_t n_rays;                /* RAYLIST kinds only                                */
} xrt_scan;

typedef struct xrt_plan xrt_plan;

/* Adjoint algorithms (Introduction: the adjoint is the transpose of the projection
 * matrix).  SCATTER walks the rays with the forward traversal and adds g_r * len into
 * the image with float atomics (order-dependent rounding); GATHER visits every unit
 * and sums over the rays that hit it, in a fixed order (deterministic); AUTO takes
 * the faster one for the plan's geometry. */
typedef enum xrt_adjoint_mode {
    XRT_ADJ_AUTO = 0,
    XRT_ADJ_SCATTER = 1,
    XRT_ADJ_GATHER = 2
} xrt_adjoint_mode;

/* Build a plan: validates grid and scan, expands the geometry in FP64 on the host
 * (Secs. 2.2.2, 3.2.2, 3.2.3 transforms, applied as the equivalent source-to-detector
 * construction), snaps direction components of magnitude <= 1e-12 to exactly 0, and
 * uploads the per-view tables to `device`.  Synchronous.  *out is NULL on failure. */
xrt_status xrt_plan_create(const xrt_grid* grid, const xrt_scan* scan, int device,
                           xrt_plan** out);

/* Free the plan's device tables.  Synchronises the plan's device.  NULL is accepted. */
xrt_status xrt_plan_destroy(xrt_plan* plan);

/* Number of rays (= sinogram elements per batch member) and of units (image elements
 * per batch member). */
xrt_status xrt_plan_sizes(const xrt_plan* plan, int64_t* n_rays, int64_t* n_units);

/* Which adjoint algorithm XRT_ADJ_AUTO runs on this plan, and for the voxel-driven cone
 * gather (flat detector, circular or helical) the kernel variant the plan selects: the
 * voxels along z each lane sums (1 for nz <= 64, 2 for nz <= 128, else 4 with further
 * z chunks), the bound on the detector rows a voxel's shadow covers in one column (the
 * candidate rows per voxel and record: 2, 3, 4, 6 or 8), the column slots per view of a
 * record pass, whether the source moves along z (helical: the kernel skips blocks of
 * voxels no ray of a record reaches), and the detector row with v = 0 (-1 if none).
 * Fields that do not apply are 0 (zero_row -1).  No GPU work. */
typedef struct {
    int32_t algorithm;        /* XRT_ADJ_SCATTER or XRT_ADJ_GATHER */
    int32_t voxels_per_lane;
    int32_t row_bound;
    int32_t column_slots;
    int32_t helical;
    int32_t zero_row;
} xrt_adjoint_info;

xrt_status xrt_plan_adjoint_info(const xrt_plan* plan, xrt_adjoint_info* out);

/* Forward transform: d_sino[b][r] = sum_I d_img[b][I] * len(r, I) for b < batch.
 * Overwrites d_sino.  d_img and d_sino must not overlap. */
xrt_status xrt_forward(xrt_plan* plan, const float* d_img, float* d_sino, int32_t batch,
                       void* stream);

/* Adjoint: d_img[b][I] = sum_r d_sino[b][r] * len(r, I).  Overwrites d_img (the
 * library clears it with its own kernel first).  mode: xrt_adjoint_mode.  The sinogram
 * is expected finite: the cone gather multiplies the values of a voxel's candidate rows
 * by lengths clamped at 0, so a NaN or infinity can also reach voxels next to those its
 * ray crosses. */
xrt_status xrt_adjoint(xrt_plan* plan, const float* d_sino, float* d_img, int32_t batch,
                       int32_t mode, void* stream);

/* Number of hit units of rays [first, first+n): d_counts[r] = #{I : len(first+r, I) > eps}
 * (eps >= 0; eps = 0 is the paper's strict condition C_low < C_up). */
xrt_status xrt_ray_hit_counts(xrt_plan* plan, int64_t first, int64_t n, double eps,
                              int32_t* d_counts, void* stream);

/* Hit lists of rays [first, first+n) (Algorithms 1 and 2: the 1D indices and
 * intersection lengths of each ray).  d_offsets is an int64 CSR row pointer [n+1]
 * (normally the exclusive prefix sum of xrt_ray_hit_counts with the same eps); row r
 * occupies d_idx/d_len[d_offsets[r] .. d_offsets[r+1]) and is sorted by increasing 1D
 * index, the order of the paper's lists (Tables 1-5).  No row writes past
 * d_offsets[r+1]; a row with more room than hits leaves the tail unwritten. */
xrt_status xrt_ray_hits(xrt_plan* plan, int64_t first, int64_t n, double eps,
                        const int64_t* d_offsets, int32_t* d_idx, float* d_len, void* stream);

/* ---------------------------------------------------------------------------------
 * Batched vector kernels of the iterative reconstructions built on the transform (CGLS,
 * Landweber; the paper's motivation in the Introduction).  Vectors are float32
 * [batch][n] contiguous; scalars are FP64, device-resident, one per batch member, so a
 * solver iteration never synchronises with the host.
 * --------------------------------------------------------------------------------- */

/* d_out[b] = sum_i d_a[b][i] * d_b[b][i], accumulated in FP64 in a fixed order
 * (deterministic).  d_work: device scratch of at least 64 * batch doubles. */
xrt_status xrt_vec_dot(int64_t n, int32_t batch, const float* d_a, const float* d_b, double* d_work,
                       double* d_out, void* stream);

/* xrt_vec_dot for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same kernels and the same result
 * bit for bit, with the partial sums in a static device array of the library instead of
 * a workspace argument (64 * 1024 doubles, 512 KiB, held by every GPU the library runs
 * on until the process ends).  The kernels run on the device of `stream` (the current
 * device for NULL); the first call on a device looks up that device's copy of the array
 * (no allocation, no GPU work).  batch <= 1024 (XRT_E_SIZE beyond).  Every call on one
 * GPU shares the array, so calls that overlap on one GPU (different streams without
 * ordering between them) race; calls ordered on one stream do not. */
xrt_status xrt_vec_dot_noalloc(int64_t n, int32_t batch, const float* d_a, const float* d_b, double* d_out,
                               void* stream);

/* d_y[b] += sign * (d_num[b] / d_den[b]) * d_x[b]; a zero denominator adds nothing. */
xrt_status xrt_vec_axpy_ratio(int64_t n, int32_t batch, const double* d_num, const double* d_den, double sign,
                              const float* d_x, float* d_y, void* stream);

/* d_p[b] = d_s[b] + (d_num[b] / d_den[b]) * d_p[b]; a zero denominator gives d_s[b]. */
xrt_status xrt_vec_xpby_ratio(int64_t n, int32_t batch, const double* d_num, const double* d_den, const float* d_s,
                              float* d_p, void* stream);

/* d_y = a * d_x + b * d_y over n elements. */
xrt_status xrt_vec_axpby(int64_t n, double a, const float* d_x, double b, float* d_y, void* stream);

/* ---------------------------------------------------------------------------------
 * 3x3 convolutions of the learned preconditioner's CNN (stride 1, zero padding 1, no
 * bias): BF16 operands (weights and inputs rounded to BF16), FP32 accumulation.
 * Tensors with one channel are float32 [batch][height][width]; tensors with 32 channels
 * are BF16 NHWC [batch][height][width][32].  A layer cin -> cout stores FP32 weights
 * W[cout][3][3][cin] (row kh, column kw).  Supported layers: 1->32, 32->32, 32->1.
 *   transposed = 0: out[p][co] = sum_{kh,kw,ci} W[co][kh][kw][ci] * in[p + (kh-1, kw-1)][ci]
 *   transposed = 1: the adjoint of that layer, out[p][ci] = sum W[co][kh][kw][ci] *
 *                   in[p - (kh-1, kw-1)][co]; (cin, cout) still name the layer, so the
 *                   input then has cout channels and the output cin channels.
 * The 32->32 layer runs on MFMA (v_mfma_f32_32x32x16_bf16).
 * --------------------------------------------------------------------------------- */

/* Convolution (or its adjoint) of one layer.  d_residual (float32, single-channel outputs
 * only, or NULL) is added to the result.  out_bf16 = 0 writes a 32-channel output as
 * float32 NHWC instead of BF16 (single-channel outputs are always float32). */
xrt_status xrt_conv3x3(int32_t cin, int32_t cout, int32_t transposed, int32_t batch, int32_t height, int32_t width,
                       const void* d_in, const float* d_weight, const float* d_residual, void* d_out,
                       int32_t out_bf16, void* stream);

/* The learned preconditioner in one launch: y = x + C3 C2 C1 x, or with transposed != 0
 * its adjoint y = x + C1^T C2^T C3^T x, for float32 images x, y [batch][height][width]
 * (C1: 1 -> 32, C2: 32 -> 32, C3: 32 -> 1 channels; weights d_w1 [32][3][3][1],
 * d_w2 [32][3][3][32], d_w3 [1][3][3][32] float32, rounded to BF16).  The result equals
 * the three xrt_conv3x3 calls with BF16 hidden activations and the residual x, up to
 * FP32 summation order; the hidden activations never leave the chip.  d_y must not
 * overlap d_x (XRT_E_ARG). */
xrt_status xrt_precond_apply(int32_t transposed, int32_t batch, int32_t height, int32_t width, const float* d_x,
                             const float* d_w1, const float* d_w2, const float* d_w3, float* d_y, void* stream);

/* Floats of device workspace xrt_conv3x3_wgrad needs for layer (cin, cout); -1 if the
 * layer is not supported. */
int64_t xrt_conv3x3_wgrad_workspace(int32_t cin, int32_t cout);

/* Weight gradient of layer (cin, cout): d_dweight[co][kh][kw][ci] = sum over batch and
 * pixels of dout[p][co] * in[p + (kh-1, kw-1)][ci] (in: cin channels, dout: cout
 * channels, both rounded to BF16), summed in a fixed order (deterministic). */
xrt_status xrt_conv3x3_wgrad(int32_t cin, int32_t cout, int32_t batch, int32_t height, int32_t width,
                             const void* d_in, const void* d_dout, float* d_work, int64_t work_floats,
                             float* d_dweight, void* stream);

/* Attenuated transform (Introduction, eq. generalizedRadontransform, SPECT case): each
 * point of a ray is weighted by exp(-integral of mu from the point to the detector side
 * of the ray; for divergent beams the side away from the source, for parallel beams the
 * +theta side).  d_mu: attenuation per unit length, float32 with the image layout, one map
 * for all images (mu_per_image = 0) or one per image.  Every hit piece of length len
 * contributes f exp(-A) (1 - exp(-mu len)) / mu (f len where mu = 0), A the attenuation
 * between the piece and the detector.  The adjoint is the exact transpose (ray-driven,
 * atomics: summation order not fixed).  Same layouts and errors as xrt_forward.  The
 * first attenuated call on a plan outside stream capture allocates a workspace of
 * 2 n_units floats that the plan keeps (XRT_E_NOMEM if that fails): the forward
 * interleaves each image with its map there, so that a candidate takes one 8-byte load;
 * the adjoint of a 3D plan keeps a y-fastest copy of the map there for the views whose
 * atomics it adds into the y-fastest layout.  A call during capture on a plan without it
 * allocates nothing and takes the paths that need none (same results up to the adjoint's
 * summation order). */
xrt_status xrt_forward_attenuated(xrt_plan* plan, const float* d_img, const float* d_mu, int32_t mu_per_image,
                                  float* d_sino, int32_t batch, void* stream);
xrt_status xrt_adjoint_attenuated(xrt_plan* plan, const float* d_sino, const float* d_mu, int32_t mu_per_image,
                                  float* d_img, int32_t batch, void* stream);

/* The transform on a simplex basis (the paper's polygonal / polyhedral extension:
 * Introduction "Contributions", Sec. 4.2).  The image lives on the simplices of a
 * structured triangulation of the plan's grid: in index coordinates (unit (k,j,i) =
 * [i,i+1) x [j,j+1) x [k,k+1)) every pixel is cut into 2 triangles by the plane
 * x - y = const, every voxel into 6 tetrahedra by the planes x - y, y - z, x - z = const.
 * Simplex s of a unit holds the points whose local coordinates, sorted largest first,
 * come in the s-th axis order: 2D (x,y) = 0, (y,x) = 1; 3D (x,y,z) = 0, (x,z,y) = 1,
 * (y,x,z) = 2, (y,z,x) = 3, (z,x,y) = 4, (z,y,x) = 5; equal coordinates rank the later
 * axis first, so a ray inside a diagonal face is given to the simplex with the bigger
 * index (Sec. 4.1's resolution carried to the new faces).  d_img: float32
 * [batch][nz][ny][nx][S] ([batch][ny][nx][2] in 2D), S = 6 (3D) or 2 (2D), i.e. simplex
 * index I * S + s.  A simplex is hit iff C_low < C_up over its facets, len = C_up - C_low.
 * Forward: d_sino[b][r] = sum_T d_img[b][T] len(r, T), overwriting d_sino.  Adjoint: its
 * transpose, ray-driven with float atomics (summation order not fixed), overwriting d_img.
 * Every ray kind of the plan; same sinogram layout and errors as xrt_forward. */
xrt_status xrt_forward_simplex(xrt_plan* plan, const float* d_img, float* d_sino, int32_t batch, void* stream);
xrt_status xrt_adjoint_simplex(xrt_plan* plan, const float* d_sino, float* d_img, int32_t batch, void* stream);

/* Per-ray weighted transform (Introduction, eq. generalizedRadontransform, PET case: the
 * weight does not depend on the position along the ray, so the generalised transform is
 * the X-ray transform times a weight given per ray).  d_w: float32 weights in sinogram
 * layout, one set for all images (w_per_image = 0) or one per image.
 * Forward: d_sino = w * (A d_img), the weight applied to the FP64 line integral before
 * rounding.  Adjoint: d_img = A^T (w * d_sino), the weight applied where each kernel reads
 * a sinogram value (mode as in xrt_adjoint, same summation order).  Same layouts and
 * errors as xrt_forward / xrt_adjoint; d_w must not be NULL (XRT_E_ARG). */
xrt_status xrt_forward_weighted(xrt_plan* plan, const float* d_img, const float* d_w, int32_t w_per_image,
                                float* d_sino, int32_t batch, void* stream);
xrt_status xrt_adjoint_weighted(xrt_plan* plan, const float* d_sino, const float* d_w, int32_t w_per_image,
                                float* d_img, int32_t batch, int32_t mode, void* stream);

/* Batch in the lanes (Sec. 4.3: rays independent; a batch shares every ray's walk).
 * d_img float [n_units][batch] and d_sino float [n_rays][batch] hold 1..64 problems
 * interleaved (unit-major; xrt_interleave converts).  One wavefront walks one ray (forward)
 * or gathers one pixel (adjoint) for the whole batch, each lane one problem, so the
 * batch's values of a unit or ray are one contiguous load.  Each problem's result equals
 * that of xrt_forward / xrt_adjoint (gather) bit for bit.  The forward takes any plan;
 * the adjoint needs a 2D plan that has the voxel-driven gather (XRT_E_UNSUPPORTED
 * otherwise).  batch outside [1, 64]: XRT_E_ARG; batch * n_units (or n_rays) * 4 bytes
 * beyond 31 bits: XRT_E_SIZE. */
xrt_status xrt_forward_interleaved(xrt_plan* plan, const float* d_img, float* d_sino, int32_t batch, void* stream);
xrt_status xrt_adjoint_interleaved(xrt_plan* plan, const float* d_sino, float* d_img, int32_t batch, void* stream);

/* Transmission of every ray through attenuation maps: d_w[b][ray] = exp(-(A d_mu[b])[ray]),
 * the PET attenuation weight of a map given per unit length in the image layout (batch
 * maps in, batch sets of weights out).  The line integral is rounded to float32 before
 * the exponential (relative error below |integral| * 6e-8).  Errors as xrt_forward. */
xrt_status xrt_ray_transmission(xrt_plan* plan, const float* d_mu, float* d_w, int32_t batch, void* stream);

/* ---- launch shape of the forward projection (tuning; results do not depend on it) ----
 * packet_cols = 0: a wavefront takes 64 consecutive rays in (view, row, column) order;
 * 64, 32 or 16: a wavefront takes a packet of packet_cols detector columns x
 * (64 / packet_cols) rows of one view; 1 (3D plans): column packets, 64 rows of one
 * detector column, which read a z-fastest copy of the image that the plan allocates
 * (n_units floats, kept; XRT_E_NOMEM if that fails) -- the rays of a cone's detector
 * column share their xy path, so the lanes step through the same x/y slabs.  Ignored for
 * ray lists.  xcd_remap = 1 gives each of the 8 XCDs a contiguous range of packets
 * (shared L2 working set).  A new cone plan with at least 64 detector rows starts with
 * column packets (1, 0), every other plan linear (0, 0); the best shape depends on the
 * geometry and is found by timing (the package's autotuner). */
typedef struct {
    int32_t packet_cols;
    int32_t xcd_remap;
} xrt_tuning;

xrt_status xrt_plan_set_tuning(xrt_plan* plan, const xrt_tuning* tuning);   /* XRT_E_ARG: bad value */
xrt_status xrt_plan_get_tuning(const xrt_plan* plan, xrt_tuning* tuning);

/* ---- batches: several plans projected by one persistent launch ----
 * 1..32 plans of one device that share the dimension and the ray mode (no ray lists;
 * XRT_E_UNSUPPORTED otherwise).  The caller keeps the plans alive while the batch
 * exists; their launch shapes are taken at creation.  The forward of all members is one
 * persistent kernel whose workgroups draw chunks of rays from a queue ordered by ray
 * length (longest first), after one small reset kernel (and the y-fastest copies of
 * the images of plans that use them); no allocation, copy or host synchronisation
 * happens in xrt_batch_forward / xrt_batch_adjoint, so both can be captured in a graph.
 * The rays of one member match xrt_forward of its plan bit for bit.  Host arrays of n
 * device pointers: images [nz][ny][nx] and sinograms of each member. */
typedef struct xrt_batch xrt_batch;

xrt_status xrt_batch_create(xrt_plan* const* plans, int32_t n, xrt_batch** out);
xrt_status xrt_batch_destroy(xrt_batch* batch);
xrt_status xrt_batch_forward(xrt_batch* batch, const float* const* d_imgs, float* const* d_sinos, void* stream);
/* Adjoint of every member (xrt_adjoint of its plan with the given mode, members in
 * queue order, each overwriting its image). */
xrt_status xrt_batch_adjoint(xrt_batch* batch, const float* const* d_sinos, float* const* d_imgs, int32_t mode,
                             void* stream);

/* ---- the projection matrix in sparse storage ----
 * The paper notes that the method can output the projection matrix in sparse storage: a
 * row of A is the hit list of one ray (unit index, length), as xrt_ray_hits writes it for
 * consecutive rays with row offsets from xrt_ray_hit_counts.  Stored, A and its transpose
 * turn every product into one gather and one multiply-add per nonzero and image. */

/* int64 elements of workspace xrt_offsets_from_counts needs for n counts (-1: n < 0). */
int64_t xrt_scan_workspace(int64_t n);

/* d_offsets[i] = d_counts[0] + ... + d_counts[i-1] for i = 0..n (int64 [n+1]); counts are
 * int32 [n].  Deterministic.  d_work: int64 [xrt_scan_workspace(n)]. */
xrt_status xrt_offsets_from_counts(int64_t n, const int32_t* d_counts, int64_t* d_offsets, int64_t* d_work,
                                   void* stream);

/* int64 elements of workspace xrt_csr_transpose needs (-1: n_cols < 0). */
int64_t xrt_csr_transpose_workspace(int64_t n_cols);

/* Transpose of a CSR matrix with n_rows rows, n_cols columns and nnz nonzeros (d_off int64
 * [n_rows+1], d_col int32 [nnz] in [0, n_cols), d_val float [nnz]) into d_t_off int64
 * [n_cols+1], d_t_col int32 [nnz], d_t_val float [nnz]; the entries of every transposed
 * row are sorted by column, so the result is unique (deterministic).  Entries whose
 * column lies outside [0, n_cols) are dropped (d_t_off[n_cols] then counts the others).
 * d_off must be a valid row-offset array for d_col / d_val.  Sizes up to 2^31-1 rows and
 * columns; d_work int64 [work_len >= xrt_csr_transpose_workspace(n_cols)]. */
xrt_status xrt_csr_transpose(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t* d_off, const int32_t* d_col,
                             const float* d_val, int64_t* d_t_off, int32_t* d_t_col, float* d_t_val, int64_t* d_work,
                             int64_t work_len, void* stream);

/* d_y[b][r] = sum over row r of val * d_x[b][col] for b < batch (d_x float [batch][n_cols],
 * d_y float [batch][n_rows]); one wavefront per row and 8 images per pass, FP64 partial
 * sums reduced in a fixed order (deterministic).  A column index outside [0, n_cols)
 * reads 0.  batch * n_cols * 4 bytes must fit in 31 bits (XRT_E_ARG otherwise). */
xrt_status xrt_csr_spmv(int64_t n_rows, int64_t n_cols, const int64_t* d_off, const int32_t* d_col, const float* d_val,
                        int32_t batch, const float* d_x, float* d_y, void* stream);

/* [batch][n] -> [n][batch] (to_interleaved != 0) or back, batch in [1, 64]; d_in and
 * d_out must be distinct. */
xrt_status xrt_interleave(int64_t n, int32_t batch, int32_t to_interleaved, const float* d_in, float* d_out,
                          void* stream);

/* xrt_csr_spmv on batch-interleaved vectors: d_y_il[r][b] = sum over row r of
 * val * d_x_il[col][b] (d_x_il float [n_cols][batch], d_y_il float [n_rows][batch], batch in
 * [1, 64]); one wavefront per row with the images in its lanes, so each nonzero reads the
 * batch's values of one unit from contiguous memory; FP64 accumulation in the row's
 * order (deterministic). */
xrt_status xrt_csr_spmv_interleaved(int64_t n_rows, int64_t n_cols, const int64_t* d_off, const int32_t* d_col,
                                   const float* d_val, int32_t batch, const float* d_x_il, float* d_y_il, void* stream);

/* Human-readable name of a status code (static storage). */
const char* xrt_status_str(int32_t status);

/* Message of the last failed call on this thread ("" if none). */
const char* xrt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* XRT_H */
