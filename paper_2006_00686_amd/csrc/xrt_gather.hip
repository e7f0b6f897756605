// Voxel-driven (gather) adjoint of the X-ray transform for flat-detector cone beams,
// circular or helical (Secs. 3.2.2-3.2.3), on gfx950.
//
// f_I = sum_r g_r len(r, I): every unit sums over the rays that hit it, in a fixed order
// (deterministic, no atomics).  Rays are enumerated from the unit's shadow on the
// detector, and each candidate's length is the paper's per-unit condition
// C_low < C_up, len = C_up - C_low (eqs. conditions_3D_1, range_length_3D), with the
// interval of every axis taken along the candidate ray.
//
// The flat detector is vertical (u horizontal, v along z), so all rays of one detector
// column c share their projection on the xy plane.  For a voxel column (i, j) and a view,
// the x and y intervals (the pixel's C_low/C_up in xy) are therefore computed once per
// column c; each voxel k then only adds the z interval of its 1-3 candidate rows.
//
// Work layout: one wavefront per voxel column (i, j) and z chunk, lane = voxel along z,
// KB voxels per lane.  The per-(view, column) xy intervals are computed by the lanes in
// parallel, 16 views x 4 column slots at a time, into records in LDS that the voxel loop
// reads uniformly.  The sinogram is first transposed to [view][col][row] and scaled by
// |d| (the ray parameter tau runs along d = detector cell - source, len = |d| dtau), so
// the lanes of a wave read consecutive rows of one column, two rows per 8-byte load.
#include "xrt_walk.h"

namespace xrt {
namespace {

constexpr int kTile = 32;
constexpr int kBlock = 256;

// gT[v][c][r] = g[v][r][c] * w[v][r][c] * |d_{c,r}|, |d|^2 = sdd^2 + u_c^2 + v_r^2 (orthogonal
// frame); w: per-ray weights (the PET form of the generalised transform), or none.
__global__ __launch_bounds__(kBlock) void k_cone_sino_prep(DevPlan P, const float* __restrict__ g,
                                                           float* __restrict__ gT, int32_t rblocks,
                                                           const float* __restrict__ wt)
{
    __shared__ float tile[kTile][kTile + 1];
    const int32_t v = blockIdx.y / rblocks;
    const int32_t r0 = (blockIdx.y - v * rblocks) * kTile;
    const int32_t c0 = blockIdx.x * kTile;
    const int32_t tx = threadIdx.x & (kTile - 1), ty = threadIdx.x >> 5;
    const double sdd2 = P.sdd * P.sdd;
    for (int32_t yy = ty; yy < kTile; yy += kBlock / kTile) {
        const int32_t r = r0 + yy, c = c0 + tx;
        if (r < P.n_rows && c < P.n_cols) {
            const double u = fma((double)c, P.du, P.ubase);
            const double w = fma((double)r, P.dv, P.vbase);
            const int64_t ray = ((int64_t)v * P.n_rows + r) * P.n_cols + c;
            const double x = (double)g[ray] * (wt != nullptr ? (double)wt[ray] : 1.0);
            tile[yy][tx] = (float)(x * sqrt(sdd2 + u * u + w * w));
        }
    }
    __syncthreads();
    for (int32_t yy = ty; yy < kTile; yy += kBlock / kTile) {
        const int32_t c = c0 + yy, r = r0 + tx;
        if (r < P.n_rows && c < P.n_cols) gT[((int64_t)v * P.n_cols + c) * P.n_rows + r] = tile[tx][yy];
    }
}

// floor/ceil of x as an index clamped to [-1, hi] (no out-of-range conversion).
__device__ __forceinline__ int32_t ifloor(double x, int32_t hi)
{
    return (int32_t)floor(fmin(fmax(x, -1.0), (double)hi));
}
__device__ __forceinline__ int32_t iceil(double x, int32_t hi)
{
    return (int32_t)ceil(fmin(fmax(x, -1.0), (double)hi));
}

// 1/x: the hardware estimate (relative error below 2^-20; 2^-24.4 measured on gfx950),
// and that estimate refined by one Newton step (error squared: full FP64 precision).
__device__ __forceinline__ double rcp_fast(double x)
{
    return __builtin_amdgcn_rcp(x);
}
__device__ __forceinline__ double rcp_full(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// Interval of the ray parameter inside one axis slab, for a ray s + tau*d whose
// offsets to the slab faces are a0 = lo - s, a1 = hi - s; a ray that does not move
// along the axis is in the slab iff the unit owns its coordinate (half-open faces).
__device__ __forceinline__ void axis_interval(double a0, double a1, double d, bool bigger_low, double& tin,
                                              double& tout)
{
    if (d != 0.0) {
        const double id = rcp_full(d);
        const double t0 = a0 * id, t1 = a1 * id;
        tin = fmax(tin, fmin(t0, t1));
        tout = fmin(tout, fmax(t0, t1));
    } else {
        // a0 <= 0 < a1: s in [lo, hi);  a0 < 0 <= a1: s in (lo, hi]
        const bool in = bigger_low ? (a0 <= 0.0 && a1 > 0.0) : (a0 < 0.0 && a1 >= 0.0);
        if (!in) tout = -kInf;
    }
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int64_t bytes)
{
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0,
                                             __builtin_amdgcn_readfirstlane((int32_t)bytes), 0x00020000);
}

constexpr int32_t kOutOfRange = (int32_t)0xFFFFFFF0u;
// Where a block of 64 voxels lies against the source height Sz: every voxel above it
// (z - Sz >= 0 on the bottom face), every voxel below it (z - Sz <= 0 on the top face), or
// mixed.  Rays leave the source at parameters tau > 0, so only rows with v > 0 can hit a
// voxel above and only rows with v < 0 a voxel below: there the order of the two face
// parameters rel / v and of the two row bounds is known, and the min / max that sort
// them drop out.
constexpr int32_t kAbove = 0, kBelow = 1, kMixed = 2;
// widening of candidate row ranges (in bins); column ranges, which come from the
// hardware reciprocal's estimate (relative error below 2^-20; 2^-24.4 measured on gfx950),
// are widened by the plan's uslack instead
constexpr double kRangeSlack = 1e-7;

// The rays of one (view, detector column) that can cross a wave's pixel column, as
// every lane of the wave needs them: the pixel's xy interval (tin, tout) of the ray
// parameter, 1/tin and 1/tout in row bins, the source height and the column's offset in
// the transposed sinogram.  One wave fills up to 64 records at once, one lane per
// (view, column slot), and then walks them in lane order.
struct ColRecs {
    double tin[64], tout[64], sin[64], sout[64], sz[64];
    int32_t g[64];
    int32_t klo[64], khi[64];   // helical scans: voxel indices k the record's rays can reach
};
constexpr int kWaves = kBlock / 64;

// One wave per voxel column (i, j) and z chunk; lane = voxel along z, KB per lane.
// NR: bound on the rows a voxel's shadow covers in one detector column (from the plan).
// ZR: the detector has a row with v = 0, whose rays lie in the plane z = Sz.
// CULL (helical scans, where the detector sees a band of z at a time): a wave skips a
// block of 64 voxels when none of them has a candidate row on the detector; skipped
// voxels are exactly the ones that would add nothing.  With 4 voxels per lane (BAND) the
// blocks follow each record's band [klo, khi] of reachable voxels: 64 consecutive voxels
// from klo (lane = voxel - block start), with the wave's voxel sums in LDS -- the band,
// about as tall as the detector's shadow, then takes 1.5 blocks on average instead of 2
// fixed ones.  Every voxel adds its records in record order either way.  Without CULL
// (circular scans) every source sits at the height sz0, and voxel heights are taken
// relative to it once.
// lg_slots: log2 of the column slots per view in one record pass (a bound on the
// columns of a pixel's shadow, from the plan; wider shadows take further passes).
// vmin, vmax: range of the detector rows' v, idz = 1 / pdz (helical culling); vb_lo1,
// vb_hi: row coordinate of v = 0 in bins, -vbase / dv, minus (plus one) and plus the
// candidate rows' slack of kRangeSlack bins (kernel arguments, so they stay in scalar
// registers).
template <int KB, int NR, bool ZR, bool CULL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_cone_gather(
    DevPlan P, const float* __restrict__ gT, float* __restrict__ img, const double* __restrict__ inv_v,
    int32_t zero_row, int32_t nzc, int32_t nlogical, int32_t lg_slots, double vmin, double vmax, double idz,
    double vb_lo1, double vb_hi, double sz0)
{
    // 1/v of every row followed by NR entries 0 for rows past the detector (their z
    // interval (0, 0) lies before tin > 0, so they are never hit), then the per-wave
    // records; the table comes first so that its addresses need no base
    extern __shared__ double s_dyn[];
    double* const s_iv = s_dyn;
    ColRecs* const s_rec = reinterpret_cast<ColRecs*>(s_dyn + ((P.n_rows + NR + 1) & ~1));
    // helical scans: each wave's voxel sums (64 KB doubles) after the records
    double* const s_accs = reinterpret_cast<double*>(s_rec + kWaves);
    constexpr bool BAND = CULL && KB == 4;
    for (int32_t r = threadIdx.x; r < P.n_rows + NR; r += kBlock) s_iv[r] = r < P.n_rows ? inv_v[r] : 0.0;
    __syncthreads();

    // XCD-aware order: hardware block b runs on XCD b % 8; each XCD gets a contiguous
    // range of logical blocks, so neighbouring voxel columns (whose shadows overlap)
    // share that XCD's L2.
    const int32_t per = (int32_t)(gridDim.x >> 3);
    const int32_t L = (int32_t)(blockIdx.x & 7) * per + (int32_t)(blockIdx.x >> 3);
    if (L >= nlogical) return;
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int64_t colid = (int64_t)L * kWaves + wave;
    if (colid >= (int64_t)P.nx * P.ny * nzc) return;
    const int32_t zc = (int32_t)(colid % nzc);
    const int64_t ij = colid / nzc;
    const int32_t i = (int32_t)(ij % P.nx), j = (int32_t)(ij / P.nx);
    ColRecs& R = s_rec[wave];

    // unit (k, j, i): x in [xa, xb), y in (ya, yb], z in (za, zb]  (Sec. 4.1 resolution)
    const double xa = fma((double)i, P.pdx, P.px0), xb = xa + P.pdx;
    const double yb = P.py0 - (double)j * P.pdy, ya = yb - P.pdy;
    const double sdd2 = P.sdd * P.sdd, idu = 1.0 / P.du, idv = 1.0 / P.dv;

    const int32_t kfirst = zc * 64 * KB, kbase = kfirst + lane;
    const __amdgpu_buffer_rsrc_t gsrc = make_rsrc(gT, (P.n_rays + kGatherPad) * 4);

    // top face of the lane's voxel q; for a circular scan (every source at height sz0)
    // already taken relative to the source, z - Sz
    // (BAND: slot 0 holds the voxel of the current block, kq its index)
    double acc[KB], zb0[KB];
    int32_t kq[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
        acc[q] = 0.0;
        kq[q] = kbase + 64 * q;
        zb0[q] = P.pz0 - (double)kq[q] * P.pdz;
        if constexpr (!CULL) zb0[q] = zb0[q] - sz0;
    }
    const int32_t kend = min(kfirst + 64 * KB, P.nz);
    double* const s_acc = s_accs + wave * 64 * KB;
    if constexpr (BAND) {
#pragma unroll
        for (int q = 0; q < KB; ++q) s_acc[lane + 64 * q] = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // Circular scans: the class of each block against sz0 is fixed for the whole scan.
    // When the wave's blocks are a run above sz0 followed by a run below it (every valid
    // lane's voxel; lanes past the volume compute values that are never stored), the
    // voxel loop is compiled for that split; otherwise, and for helical scans, every
    // block takes the general form.  Below sz0 needs z - Sz < 0 on the top face when the
    // detector has a row with v = 0 (that row's plane z = Sz belongs to a voxel whose top
    // face it is).
    int32_t split = -1;
    if constexpr (!CULL) {
        int32_t m = 0;
        bool ok = true;
#pragma unroll
        for (int q = 0; q < KB; ++q) {
            const uint64_t valid = __builtin_amdgcn_ballot_w64(kbase + 64 * q < P.nz);
            const double rel1 = zb0[q], rel0 = rel1 - P.pdz;
            const bool above = (__builtin_amdgcn_ballot_w64(!(rel0 >= 0.0)) & valid) == 0;
            const bool below = (__builtin_amdgcn_ballot_w64(!(ZR ? rel1 < 0.0 : rel1 <= 0.0)) & valid) == 0;
            if (above && m == q)
                m = q + 1;
            else if (!below)
                ok = false;
        }
        split = ok ? m : -1;
    }
    auto run = [&](auto S) {
        constexpr int32_t kSplit = decltype(S)::value;
        // class of block q (a constant once the loops over q are unrolled)
        auto cls_of = [](int q) { return kSplit < 0 ? kMixed : q < kSplit ? kAbove : kBelow; };

        const int32_t slot = lane & ((1 << lg_slots) - 1), vlane = lane >> lg_slots;
        for (int32_t v0 = 0; v0 < P.n_views; v0 += 64 >> lg_slots)
            for (int32_t pass = 0;; ++pass) {
                // this lane's view: detector columns whose rays can cross the pixel, from u of
                // the four corners seen from the source, u = sdd^2 ((P - S).B) / ((P - S).E);
                // recomputed per pass so that none of it stays live across the voxel loop
                const int32_t v = v0 + vlane;
                const bool vok = v < P.n_views;
                const ViewGeom& V = P.views[vok ? v : P.n_views - 1];
                const double Sx = V.A[0], Sy = V.A[1];
                const double Ex = V.E[0], Ey = V.E[1], Bx = V.B[0], By = V.B[1];
                const double ax0 = xa - Sx, ax1 = xb - Sx, ay0 = ya - Sy, ay1 = yb - Sy;
                double umin = kInf, umax = -kInf;
#pragma unroll
                for (int cnr = 0; cnr < 4; ++cnr) {
                    const double px = (cnr & 1) ? ax1 : ax0, py = (cnr & 2) ? ay1 : ay0;
                    const double u = sdd2 * fma(px, Bx, py * By) * rcp_fast(fma(px, Ex, py * Ey));
                    umin = fmin(umin, u);
                    umax = fmax(umax, u);
                }
                const int32_t c0 = max(iceil(fma(umin - P.ubase, idu, -P.uslack), P.n_cols), 0);
                const int32_t c1 = min(ifloor(fma(umax - P.ubase, idu, P.uslack), P.n_cols), P.n_cols - 1);
                const int32_t cb = c0 + (pass << lg_slots);
                if (__builtin_amdgcn_ballot_w64(vok && cb <= c1) == 0) break;
                // C_low / C_up of the pixel in xy, shared by every ray of column c
                const int32_t c = cb + slot;
                bool ok = vok && c <= c1;
                double tin = -kInf, tout = kInf;
                if (ok) {
                    const double u = fma((double)c, P.du, P.ubase);
                    axis_interval(ax0, ax1, fma(u, Bx, Ex), true, tin, tout);
                    axis_interval(ay0, ay1, fma(u, By, Ey), false, tin, tout);
                    ok = tin < tout;
                }
                const uint64_t live = __builtin_amdgcn_ballot_w64(ok);
                if (ok) {
                    const int32_t at = __builtin_amdgcn_mbcnt_hi((uint32_t)(live >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)live, 0));
                    R.tin[at] = tin;
                    R.tout[at] = tout;
                    // 1/tau in row bins for the candidate rows: refined, so that a row range of
                    // a few hundred bins stays within the rows' 1e-7-bin slack
                    R.sin[at] = rcp_full(tin) * idv;
                    R.sout[at] = rcp_full(tout) * idv;
                    R.sz[at] = V.A[2];
                    R.g[at] = (int32_t)(((int64_t)v * P.n_cols + c) * P.n_rows) * 4;
                    if constexpr (BAND) {
                        // heights z = Sz + tau v over tau in (tin, tout) and v in [vmin, vmax]
                        // (bilinear: extremes at the corners), widened by a hundredth of a
                        // unit; voxel k spans z in (pz0 - (k + 1) dz, pz0 - k dz]
                        const double zlo = V.A[2] + fmin(tin * vmin, tout * vmin) - 0.01 * P.pdz;
                        const double zhi = V.A[2] + fmax(tin * vmax, tout * vmax) + 0.01 * P.pdz;
                        R.klo[at] = (int32_t)floor(fmin(fmax((P.pz0 - zhi) * idz, -2.0), (double)P.nz + 1.0));
                        R.khi[at] = (int32_t)floor(fmin(fmax((P.pz0 - zlo) * idz, -2.0), (double)P.nz + 1.0));
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int32_t nrec = __builtin_popcountll(live);
                for (int32_t e = 0; e < nrec; ++e) {
                    const double tin_ = R.tin[e], tout_ = R.tout[e], sin_ = R.sin[e], sout = R.sout[e], Sz = R.sz[e];
                    const int32_t gcol4 = R.g[e];
                    // C_up - C_low of row r in the voxel between z offsets rel0 < rel1: positive
                    // iff C_low < C_up (hit), else finite and non-positive (lanes past the
                    // volume, k >= nz, compute values that are never stored).  Above Sz a row
                    // with v > 0 crosses the faces at rel0 / v < rel1 / v; a row with v <= 0
                    // (1/v <= 0, the zero row and the padding rows store 0) gets an upper end
                    // <= 0 < tin, so a non-positive value as it should.  Below Sz likewise with
                    // the faces swapped.  Hits get the same value as from the general form.
                    auto len = [&](int32_t r, double rel0, double rel1, int32_t cls) {
                        double lo = tin_, hi = tout_;
                        if (cls == kAbove) {
                            const double iv = s_iv[r];
                            lo = fmax(lo, rel0 * iv);
                            hi = fmin(hi, rel1 * iv);
                        } else if (cls == kBelow) {
                            const double iv = s_iv[r];
                            lo = fmax(lo, rel1 * iv);
                            hi = fmin(hi, rel0 * iv);
                        } else if (ZR && r == zero_row) {
                            if (!(rel0 < 0.0 && rel1 >= 0.0)) hi = lo;   // plane z = Sz not in (za, zb]
                        } else {
                            const double iv = s_iv[r];
                            const double t0 = rel0 * iv, t1 = rel1 * iv;
                            lo = fmax(lo, fmin(t0, t1));
                            hi = fmin(hi, fmax(t0, t1));
                        }
                        return hi - lo;
                    };
                    // per voxel q of the lane: rows r0 and r0 + 1 (one 8-byte load, out of range
                    // when neither row is hit; a row that is not hit contributes 0), then the
                    // rows beyond where some shadow reaches them
                    int32_t r0[KB];
                    double l0[KB], l1[KB];
                    float g0[KB], g1[KB];
                    bool more[KB];
                    auto head = [&](int q, int32_t cls) {
                        // first candidate row: the smallest v = rel / tau of the voxel over
                        // tau in (tin, tout), in bin units (1/tin > 1/tout > 0: above Sz the
                        // smallest at tout, below it at tin, and the largest the other way)
                        const double rel1 = CULL ? zb0[q] - Sz : zb0[q], rel0 = rel1 - P.pdz;
                        // plus one: r0 = trunc(vlo + 1) is ceil(vlo), or one more where vlo is an
                        // integer m -- that row then lies below the voxel's rows by the slack
                        const double vlo1 = cls == kAbove   ? fma(rel0, sout, vb_lo1)
                                            : cls == kBelow ? fma(rel0, sin_, vb_lo1)
                                                            : fmin(fma(rel0, sin_, vb_lo1), fma(rel0, sout, vb_lo1));
                        // rows outside the voxel's range fail C_low < C_up below on their own
                        // (clamped so that r0 + NR - 1 stays inside the padded 1/v table)
                        r0[q] = min(max((int32_t)vlo1, 0), P.n_rows);
                        const double vhi = cls == kAbove   ? fma(rel1, sin_, vb_hi)
                                           : cls == kBelow ? fma(rel1, sout, vb_hi)
                                                           : fmax(fma(rel1, sin_, vb_hi), fma(rel1, sout, vb_hi));
                        more[q] = NR > 2 && vhi >= (double)(r0[q] + 2);
                        if constexpr (CULL) {
                            // rows past the detector are zero padding; a voxel whose rows all
                            // lie above the first row (by half a bin, far beyond the error of
                            // the estimates) has no hit in rows r0 = 0 ..
                            const bool any = kq[q] < P.nz && r0[q] < P.n_rows && vhi >= -0.5 + kRangeSlack;
                            if (__builtin_amdgcn_ballot_w64(any) == 0) return false;
                        }
                        l0[q] = len(r0[q], rel0, rel1, cls);
                        l1[q] = len(r0[q] + 1, rel0, rel1, cls);
                        const bool h0 = l0[q] > 0.0, h1 = l1[q] > 0.0;
                        const int32_t off = h0 || h1 ? gcol4 + 4 * r0[q] : kOutOfRange;
                        const uint32_t a = __builtin_amdgcn_raw_buffer_load_b32(gsrc, off, 0, 0);
                        const uint32_t b = __builtin_amdgcn_raw_buffer_load_b32(gsrc, off + 4, 0, 0);
                        // a row that is not hit adds its value times a length clamped to
                        // 0 (both rows out of range read 0)
                        g0[q] = __builtin_bit_cast(float, a);
                        g1[q] = __builtin_bit_cast(float, b);
                        return true;
                    };
                    auto body = [&](int q) {
                        acc[q] = fma((double)g0[q], fmax(l0[q], 0.0), acc[q]);
                        acc[q] = fma((double)g1[q], fmax(l1[q], 0.0), acc[q]);
                    };
                    // only where some lane's shadow spans more than one bin (whole waves skip it
                    // often enough that evaluating it always is slower)
                    auto tail = [&](int q, int32_t cls) {
                        if (NR > 2 && more[q]) {
                            const double rel1 = CULL ? zb0[q] - Sz : zb0[q], rel0 = rel1 - P.pdz;
#pragma unroll
                            for (int ei = 2; ei < NR; ++ei) {
                                const int32_t r = r0[q] + ei;
                                const double le = len(r, rel0, rel1, cls);
                                // a row that is not hit reads 0 (out of range)
                                const float ge = __builtin_bit_cast(
                                    float, __builtin_amdgcn_raw_buffer_load_b32(
                                               gsrc, le > 0.0 ? gcol4 + 4 * r : kOutOfRange, 0, 0));
                                acc[q] = fma((double)ge, le, acc[q]);
                            }
                        }
                    };
                    if constexpr (BAND) {
                        // the record's band of voxels in blocks of 64 from
                        // klo (scalar bounds), each skipped by the vote in head() when no
                        // voxel of it has a candidate row
                        const int32_t klo = __builtin_amdgcn_readfirstlane(R.klo[e]);
                        const int32_t kstop = min(__builtin_amdgcn_readfirstlane(R.khi[e]), kend - 1);
                        for (int32_t kb = max(klo, kfirst); kb <= kstop; kb += 64) {
                            kq[0] = kb + lane;
                            zb0[0] = P.pz0 - (double)kq[0] * P.pdz;
                            // the block's class against this record's source height (lanes
                            // past the volume do not count), one copy of the block's code
                            // per class
                            const uint64_t valid = __builtin_amdgcn_ballot_w64(kq[0] < P.nz);
                            const double rel1 = zb0[0] - Sz, rel0 = rel1 - P.pdz;
                            const bool above = (__builtin_amdgcn_ballot_w64(!(rel0 >= 0.0)) & valid) == 0;
                            const bool below =
                                (__builtin_amdgcn_ballot_w64(!(ZR ? rel1 < 0.0 : rel1 <= 0.0)) & valid) == 0;
                            auto block = [&](int32_t cls) {
                                if (head(0, cls)) {
                                    // lanes past the wave's voxels compute values never stored
                                    const bool mine = kq[0] < kend;
                                    const int32_t at = kq[0] - kfirst;
                                    acc[0] = mine ? s_acc[at] : 0.0;
                                    body(0);
                                    tail(0, cls);
                                    if (mine) s_acc[at] = acc[0];
                                }
                            };
                            if (above)
                                block(kAbove);
                            else if (below)
                                block(kBelow);
                            else
                                block(kMixed);
                        }
                        // the next record's blocks give these voxels to other lanes
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    } else if constexpr (CULL) {
                        // shorter chunks: the fixed blocks, culled by the vote in head()
#pragma unroll
                        for (int q = 0; q < KB; ++q) {
                            if (head(q, kMixed)) {
                                body(q);
                                tail(q, kMixed);
                            }
                        }
                    } else {
                        // the loads of every voxel of the lane in flight together
#pragma unroll
                        for (int q = 0; q < KB; ++q) head(q, cls_of(q));
#pragma unroll
                        for (int q = 0; q < KB; ++q) body(q);
#pragma unroll
                        for (int q = 0; q < KB; ++q) tail(q, cls_of(q));
                    }
                }
                // every lane has read the records before the next pass rewrites them
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
    };
    using std::integral_constant;
    if (CULL || split < 0)
        run(integral_constant<int32_t, -1>{});
    else if (split == 0)
        run(integral_constant<int32_t, 0>{});
    else if (KB == 1 || split == 1)
        run(integral_constant<int32_t, 1>{});
    else if (KB == 2 || split == 2)
        run(integral_constant<int32_t, 2>{});
    else if (split == 3)
        run(integral_constant<int32_t, 3>{});
    else
        run(integral_constant<int32_t, 4>{});
#pragma unroll
    for (int q = 0; q < KB; ++q) {
        const int32_t k = kbase + 64 * q;
        if (k < P.nz) img[((int64_t)k * P.ny + j) * P.nx + i] = (float)(BAND ? s_acc[lane + 64 * q] : acc[q]);
    }
}

// ---------------------------------------------------------------------------------
// 2D gather adjoint (every 2D scan kind): one lane per pixel, BB images per lane, and
// the views split over the kG2Waves waves of a block (wave w takes views w, w + kG2Waves,
// ...), whose sums are added in wave order at the end (deterministic: fixed view, bin
// and wave order).  Per view the pixel's shadow on the detector gives the candidate
// bins; each candidate ray is clipped against the pixel (C_low < C_up of eq.
// conditions_2D_1, half-open faces) and adds g * len.
//
// The clip takes the ray parameter in physical length: with J = |d| / d per axis (the
// plan's ray2d table, 0 for a zero component), the pixel's x interval is
// (x - o_x) J_x over x in {xa, xb}, so len = C_up - C_low directly.  Every candidate's
// work is four products, six min / max and one multiply-add per image.
// wt: per-ray weights applied to the sinogram values (the PET form), or none.
// Eight waves per block: a 512^2 image has 4096 pixel blocks, too few to hide the
// candidates' load latency with four (fan2d_512 step 0.894 -> 0.878 ms).
constexpr int kG2Waves = 8;

// C_up - C_low of a ray from a source (origin offsets a0 = xa - S_x, a1 = xb - S_x,
// b0 = ya - S_y, b1 = yb - S_y, every unit at positive ray parameter) with J from the
// plan's table.  A ray parallel to x grid lines has J_x = +1e300: its x interval is then
// (-inf, +inf) for a0 < 0 < a1, [0, inf) for a0 = 0 and (-inf, 0] for a1 = 0 -- with the
// unit's positive parameters, exactly the membership x in [xa, xb); J_y = -1e300 gives
// y in (ya, yb] the same way.  No branch, no division.
__device__ __forceinline__ double clip2d_src(double a0, double a1, double b0, double b1, double jx, double jy)
{
    const double t0 = a0 * jx, t1 = a1 * jx, u0 = b0 * jy, u1 = b1 * jy;
    return fmin(fmax(t0, t1), fmax(u0, u1)) - fmax(fmin(t0, t1), fmin(u0, u1));
}

// C_up - C_low of a parallel-beam ray with origin offsets a0 = xa - o_x, a1 = xb - o_x,
// b0 = ya - o_y, b1 = yb - o_y and J (0: the ray runs along that axis's grid lines, where
// the pixel owns x in [xa, xb) and y in (ya, yb]; J is the view's, so such a branch is
// taken by the whole wavefront)
__device__ __forceinline__ double clip2d(double a0, double a1, double b0, double b1, double jx, double jy)
{
    double lo = -kInf, hi = kInf;
    if (jx != 0.0) {
        const double t0 = a0 * jx, t1 = a1 * jx;
        lo = fmin(t0, t1);
        hi = fmax(t0, t1);
    } else if (!(a0 <= 0.0 && a1 > 0.0)) {
        hi = -kInf;
    }
    if (jy != 0.0) {
        const double t0 = b0 * jy, t1 = b1 * jy;
        lo = fmax(lo, fmin(t0, t1));
        hi = fmin(hi, fmax(t0, t1));
    } else if (!(b0 < 0.0 && b1 >= 0.0)) {
        hi = -kInf;
    }
    return hi - lo;
}

// Detector bins [cb, ce] whose rays can cross the pixel with corner offsets a0, a1 (x)
// and c0y, c1y (y) from the view's origin.  Hits and lengths come from the exact clip; a
// range only has to contain every bin that hits, and its slack covers the rounding of the
// hardware reciprocal.  Rays from a flat-detector source (when the plan allows): the
// centre's coordinate u_c = sdd^2 (B . p) / (E . p) and the half-width of the shadow of
// the pixel's circumscribed disc (see DevPlan::g2_r); otherwise the four corners.
template <int MODE>
__device__ __forceinline__ void candidate_bins(const DevPlan& P, double a0, double a1, double c0y, double c1y,
                                               double Bx, double By, double Ex, double Ey, double idu, int32_t& cb,
                                               int32_t& ce)
{
    double umin = kInf, umax = -kInf;
    if (MODE == MODE_DIVERGENT && P.g2_r > 0.0) {
        const double px = 0.5 * (a0 + a1), py = 0.5 * (c0y + c1y);
        const double e2 = Ex * Ex + Ey * Ey;                     // |E|^2 = sdd^2
        const double r = rcp_fast(fma(px, Ex, py * Ey));
        const double uc = e2 * fma(px, Bx, py * By) * r;
        const double hw = (e2 + fmax(P.g2_umax2, uc * uc)) * P.g2_r * r * P.du;
        umin = uc - hw;
        umax = uc + hw;
    } else {
#pragma unroll
        for (int cnr = 0; cnr < 4; ++cnr) {
            const double px = (cnr & 1) ? a1 : a0, py = (cnr & 2) ? c1y : c0y;
            double u;
            if constexpr (MODE == MODE_PARALLEL) {
                u = fma(px, Bx, py * By);                        // p = u B (+ t E)
            } else if constexpr (MODE == MODE_DIVERGENT) {
                const double e2 = Ex * Ex + Ey * Ey;
                u = e2 * fma(px, Bx, py * By) * rcp_fast(fma(px, Ex, py * Ey));
            } else {
                u = atan2(fma(px, Bx, py * By), fma(px, Ex, py * Ey));   // equiangular gamma
            }
            umin = fmin(umin, u);
            umax = fmax(umax, u);
        }
    }
    cb = max(iceil(fma(umin - P.ubase, idu, -P.uslack), P.n_cols), 0);
    ce = min(ifloor(fma(umax - P.ubase, idu, P.uslack), P.n_cols), P.n_cols - 1);
}

template <int MODE, int BB, bool WT>
__global__ __launch_bounds__(64 * kG2Waves) void k_gather2d(DevPlan P, const float* __restrict__ sino,
                                                             float* __restrict__ img, int32_t batch,
                                                             const float* __restrict__ wt, int64_t wt_stride)
{
    __shared__ double part[kG2Waves - 1][BB][64];
    const int32_t lane = threadIdx.x & 63;
    const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t pix = (int32_t)blockIdx.x * 64 + lane;
    const bool live = pix < P.nx * P.ny;
    const int32_t b0 = blockIdx.y * BB;
    const int32_t i = live ? pix % P.nx : 0, j = live ? pix / P.nx : 0;
    const double xa = fma((double)i, P.pdx, P.px0), xb = xa + P.pdx;
    const double yb = P.py0 - (double)j * P.pdy, ya = yb - P.pdy;
    const double idu = 1.0 / P.du;
    double acc[BB];
#pragma unroll
    for (int q = 0; q < BB; ++q) acc[q] = 0.0;
    auto value = [&](int q, int64_t r) {
        double g = (double)sino[(int64_t)(b0 + q) * P.n_rays + r];
        if constexpr (WT) g *= (double)wt[(int64_t)(b0 + q) * wt_stride + r];
        return g;
    };
    for (int32_t v = wv; v < P.n_views && live; v += kG2Waves) {
        const ViewGeom& V = P.views[v];
        const double Ax = V.A[0], Ay = V.A[1], Bx = V.B[0], By = V.B[1], Ex = V.E[0], Ey = V.E[1];
        // corner offsets from the view's origin (the source for rays that fan out)
        const double a0 = xa - Ax, a1 = xb - Ax, c0y = ya - Ay, c1y = yb - Ay;
        int32_t cb, ce;
        candidate_bins<MODE>(P, a0, a1, c0y, c1y, Bx, By, Ex, Ey, idu, cb, ce);
        if constexpr (MODE == MODE_PARALLEL) {
            const double jx = P.ray2d[2 * v], jy = P.ray2d[2 * v + 1];
            for (int32_t c = cb; c <= ce; ++c) {
                // origin A + u B moves with the bin; the direction is the view's
                const double u = fma((double)c, P.du, P.ubase);
                const double ox = u * Bx, oy = u * By;
                const double len = clip2d(a0 - ox, a1 - ox, c0y - oy, c1y - oy, jx, jy);
                if (!(len > 0.0)) continue;
                const int64_t r = (int64_t)v * P.n_cols + c;
#pragma unroll
                for (int q = 0; q < BB; ++q)
                    if (BB == 1 || b0 + q < batch) acc[q] = fma(value(q, r), len, acc[q]);
            }
        } else {
            for (int32_t c = cb; c <= ce; ++c) {
                const int64_t r = (int64_t)v * P.n_cols + c;
                const double2 J = *reinterpret_cast<const double2*>(P.ray2d + 2 * r);
                const double len = clip2d_src(a0, a1, c0y, c1y, J.x, J.y);
                if (!(len > 0.0)) continue;
#pragma unroll
                for (int q = 0; q < BB; ++q)
                    if (BB == 1 || b0 + q < batch) acc[q] = fma(value(q, r), len, acc[q]);
            }
        }
    }
    if (wv > 0) {
#pragma unroll
        for (int q = 0; q < BB; ++q) part[wv - 1][q][lane] = acc[q];
    }
    __syncthreads();
    if (wv == 0 && live) {
#pragma unroll
        for (int q = 0; q < BB; ++q) {
            double s = acc[q];
#pragma unroll
            for (int w = 0; w < kG2Waves - 1; ++w) s += part[w][q][lane];
            if (BB == 1 || b0 + q < batch) img[(int64_t)(b0 + q) * P.n_units + pix] = (float)s;
        }
    }
}

// 2D gather adjoint of a batch of up to 64 sinograms held interleaved ([ray][image]):
// one lane per pixel and 8 images per lane, as k_gather2d (same view split over the
// block's waves, same clip, same order of every sum), but a candidate's 8 values are
// contiguous: with VEC (batch a multiple of 4) two 16-byte loads of the group's images
// inside the batch (a group of 4 past it is not read), else 8 guarded loads.
template <int MODE, bool VEC>
__global__ __launch_bounds__(64 * kG2Waves) void k_gather2d_il(DevPlan P, const float* __restrict__ sino,
                                                                float* __restrict__ img, int32_t batch)
{
    constexpr int BB = 8;
    __shared__ double part[kG2Waves - 1][BB][64];
    const int32_t lane = threadIdx.x & 63;
    const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t pix = (int32_t)blockIdx.x * 64 + lane;
    const bool live = pix < P.nx * P.ny;
    const int32_t b0 = blockIdx.y * BB;
    const int32_t i = live ? pix % P.nx : 0, j = live ? pix / P.nx : 0;
    const double xa = fma((double)i, P.pdx, P.px0), xb = xa + P.pdx;
    const double yb = P.py0 - (double)j * P.pdy, ya = yb - P.pdy;
    const double idu = 1.0 / P.du;
    const bool hi4 = b0 + 4 < batch;   // the group's second 4 images lie in the batch
    double acc[BB];
#pragma unroll
    for (int q = 0; q < BB; ++q) acc[q] = 0.0;
    for (int32_t v = wv; v < P.n_views && live; v += kG2Waves) {
        const ViewGeom& V = P.views[v];
        const double Ax = V.A[0], Ay = V.A[1], Bx = V.B[0], By = V.B[1], Ex = V.E[0], Ey = V.E[1];
        const double a0 = xa - Ax, a1 = xb - Ax, c0y = ya - Ay, c1y = yb - Ay;
        int32_t cb, ce;
        candidate_bins<MODE>(P, a0, a1, c0y, c1y, Bx, By, Ex, Ey, idu, cb, ce);
        double jx = 0.0, jy = 0.0;
        if constexpr (MODE == MODE_PARALLEL) {
            jx = P.ray2d[2 * v];
            jy = P.ray2d[2 * v + 1];
        }
        for (int32_t c = cb; c <= ce; ++c) {
            double len;
            if constexpr (MODE == MODE_PARALLEL) {
                const double u = fma((double)c, P.du, P.ubase);
                const double ox = u * Bx, oy = u * By;
                len = clip2d(a0 - ox, a1 - ox, c0y - oy, c1y - oy, jx, jy);
            } else {
                const double2 J = *reinterpret_cast<const double2*>(P.ray2d + 2 * ((int64_t)v * P.n_cols + c));
                len = clip2d_src(a0, a1, c0y, c1y, J.x, J.y);
            }
            if (!(len > 0.0)) continue;
            const int64_t at = (int64_t)(v * P.n_cols + c) * batch + b0;
            float g[BB];
            if constexpr (VEC) {
                const float4 lo = *reinterpret_cast<const float4*>(sino + at);
                const float4 up = hi4 ? *reinterpret_cast<const float4*>(sino + at + 4) : make_float4(0, 0, 0, 0);
                g[0] = lo.x; g[1] = lo.y; g[2] = lo.z; g[3] = lo.w;
                g[4] = up.x; g[5] = up.y; g[6] = up.z; g[7] = up.w;
            } else {
#pragma unroll
                for (int q = 0; q < BB; ++q) g[q] = b0 + q < batch ? sino[at + q] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < BB; ++q) acc[q] = fma((double)g[q], len, acc[q]);
        }
    }
    if (wv > 0) {
#pragma unroll
        for (int q = 0; q < BB; ++q) part[wv - 1][q][lane] = acc[q];
    }
    __syncthreads();
    if (wv == 0 && live) {
#pragma unroll
        for (int q = 0; q < BB; ++q) {
            double s = acc[q];
#pragma unroll
            for (int w = 0; w < kG2Waves - 1; ++w) s += part[w][q][lane];
            if (b0 + q < batch) img[(int64_t)pix * batch + b0 + q] = (float)s;
        }
    }
}

template <int KB, int NR, bool CULL>
xrt_status launch_kb(const xrt_plan* p, const float* gT, float* img, hipStream_t s)
{
    const DevPlan& P = p->dp;
    const int32_t nzc = (P.nz + 64 * KB - 1) / (64 * KB);
    const int64_t cols = (int64_t)P.nx * P.ny * nzc;
    const int64_t nlog = (cols + kBlock / 64 - 1) / (kBlock / 64);
    if (nlog > INT32_MAX / 2) {
        set_error("volume too large for the gather adjoint");
        return XRT_E_SIZE;
    }
    const int64_t launched = (nlog + 7) / 8 * 8;
    const size_t lds = kWaves * sizeof(ColRecs) + (size_t)((P.n_rows + NR + 1) & ~1) * sizeof(double) +
                       (CULL && KB == 4 ? (size_t)kWaves * 64 * KB * sizeof(double) : 0);
    const double vlast = P.vbase + (P.n_rows - 1) * P.dv;
    const double vmin = std::fmin(P.vbase, vlast), vmax = std::fmax(P.vbase, vlast);
    const double vb = -P.vbase * (1.0 / P.dv);
    const double sz0 = p->sz0;
    if (p->zero_row >= 0)
        hipLaunchKernelGGL((k_cone_gather<KB, NR, true, CULL>), dim3((unsigned)launched), dim3(kBlock), lds, s, P,
                           gT, img, (const double*)p->d_invwz, p->zero_row, nzc, (int32_t)nlog, p->gather_lgs,
                           vmin, vmax, 1.0 / P.pdz, vb - kRangeSlack + 1.0, vb + kRangeSlack, sz0);
    else
        hipLaunchKernelGGL((k_cone_gather<KB, NR, false, CULL>), dim3((unsigned)launched), dim3(kBlock), lds, s, P,
                           gT, img, (const double*)p->d_invwz, p->zero_row, nzc, (int32_t)nlog, p->gather_lgs,
                           vmin, vmax, 1.0 / P.pdz, vb - kRangeSlack + 1.0, vb + kRangeSlack, sz0);
    return hip_fail(hipGetLastError(), "gather kernel launch");
}

template <int NR, bool CULL>
xrt_status launch_nr_c(const xrt_plan* p, const float* gT, float* img, hipStream_t s)
{
    const int32_t nz = p->dp.nz;
    if (nz <= 64) return launch_kb<1, NR, CULL>(p, gT, img, s);
    if (nz <= 128) return launch_kb<2, NR, CULL>(p, gT, img, s);
    return launch_kb<4, NR, CULL>(p, gT, img, s);   // deeper volumes: further z chunks
}

template <int NR>
xrt_status launch_nr(const xrt_plan* p, const float* gT, float* img, hipStream_t s)
{
    return p->helical ? launch_nr_c<NR, true>(p, gT, img, s) : launch_nr_c<NR, false>(p, gT, img, s);
}

}  // namespace

xrt_status launch_adjoint_gather2d(const xrt_plan* p, const float* sino, float* img, int batch, hipStream_t s,
                                   const float* wt, int64_t wt_stride)
{
    const DevPlan& P = p->dp;
    if (P.mode != MODE_PARALLEL && P.mode != MODE_DIVERGENT && P.mode != MODE_ARC) {
        set_error("no gather adjoint for ray lists");
        return XRT_E_UNSUPPORTED;
    }
    const unsigned blocks = (unsigned)((P.nx * P.ny + 63) / 64);
    auto go = [&](auto k1, auto k8, auto k1w, auto k8w) {
        const dim3 g1(blocks, 1u), g8(blocks, (unsigned)((batch + 7) / 8));
        if (wt == nullptr) {
            if (batch == 1) hipLaunchKernelGGL(k1, g1, dim3(64 * kG2Waves), 0, s, P, sino, img, batch, wt, wt_stride);
            else hipLaunchKernelGGL(k8, g8, dim3(64 * kG2Waves), 0, s, P, sino, img, batch, wt, wt_stride);
        } else {
            if (batch == 1) hipLaunchKernelGGL(k1w, g1, dim3(64 * kG2Waves), 0, s, P, sino, img, batch, wt, wt_stride);
            else hipLaunchKernelGGL(k8w, g8, dim3(64 * kG2Waves), 0, s, P, sino, img, batch, wt, wt_stride);
        }
    };
    switch (P.mode) {
        case MODE_PARALLEL:
            go(k_gather2d<MODE_PARALLEL, 1, false>, k_gather2d<MODE_PARALLEL, 8, false>,
               k_gather2d<MODE_PARALLEL, 1, true>, k_gather2d<MODE_PARALLEL, 8, true>);
            break;
        case MODE_DIVERGENT:
            go(k_gather2d<MODE_DIVERGENT, 1, false>, k_gather2d<MODE_DIVERGENT, 8, false>,
               k_gather2d<MODE_DIVERGENT, 1, true>, k_gather2d<MODE_DIVERGENT, 8, true>);
            break;
        default:
            go(k_gather2d<MODE_ARC, 1, false>, k_gather2d<MODE_ARC, 8, false>, k_gather2d<MODE_ARC, 1, true>,
               k_gather2d<MODE_ARC, 8, true>);
            break;
    }
    return hip_fail(hipGetLastError(), "2D gather launch");
}

xrt_status launch_adjoint_gather2d_il(const xrt_plan* p, const float* sino, float* img, int batch, hipStream_t s)
{
    const DevPlan& P = p->dp;
    const dim3 grid((unsigned)((P.nx * P.ny + 63) / 64), (unsigned)((batch + 7) / 8));
    const bool vec = (batch & 3) == 0 && ((uintptr_t)sino & 15) == 0;   // 16-byte aligned groups of 4
    auto go = [&](auto kv, auto ks) { hipLaunchKernelGGL(vec ? kv : ks, grid, dim3(64 * kG2Waves), 0, s, P, sino, img,
                                                         (int32_t)batch); };
    switch (P.mode) {
        case MODE_PARALLEL: go(k_gather2d_il<MODE_PARALLEL, true>, k_gather2d_il<MODE_PARALLEL, false>); break;
        case MODE_DIVERGENT: go(k_gather2d_il<MODE_DIVERGENT, true>, k_gather2d_il<MODE_DIVERGENT, false>); break;
        case MODE_ARC: go(k_gather2d_il<MODE_ARC, true>, k_gather2d_il<MODE_ARC, false>); break;
        default:
            set_error("no gather adjoint for ray lists");
            return XRT_E_UNSUPPORTED;
    }
    return hip_fail(hipGetLastError(), "interleaved 2D gather launch");
}

xrt_status launch_adjoint_cone_gather(const xrt_plan* p, const float* sino, float* img, int batch,
                                      hipStream_t s, const float* wt, int64_t wt_stride)
{
    const DevPlan& P = p->dp;
    const int32_t rblocks = (P.n_rows + kTile - 1) / kTile;
    const dim3 pgrid((unsigned)((P.n_cols + kTile - 1) / kTile), (unsigned)(rblocks * P.n_views));
    for (int b = 0; b < batch; ++b) {
        hipLaunchKernelGGL(k_cone_sino_prep, pgrid, dim3(kBlock), 0, s, P, sino + (int64_t)b * P.n_rays,
                           p->d_gT, rblocks, wt != nullptr ? wt + (int64_t)b * wt_stride : nullptr);
        xrt_status st = hip_fail(hipGetLastError(), "sinogram prep launch");
        if (st != XRT_OK) return st;
        float* out = img + (int64_t)b * P.n_units;
        if (p->gather_nr <= 2) st = launch_nr<2>(p, p->d_gT, out, s);
        else if (p->gather_nr == 3) st = launch_nr<3>(p, p->d_gT, out, s);
        else if (p->gather_nr == 4) st = launch_nr<4>(p, p->d_gT, out, s);
        else if (p->gather_nr <= 6) st = launch_nr<6>(p, p->d_gT, out, s);
        else st = launch_nr<8>(p, p->d_gT, out, s);
        if (st != XRT_OK) return st;
    }
    return XRT_OK;
}

}  // namespace xrt
