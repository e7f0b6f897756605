// Host side of libxrt: argument validation, FP64 geometry expansion into per-view
// tables, plan lifetime and the extern "C" entry points declared in include/xrt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "xrt_internal.h"

namespace xrt {
namespace {

thread_local char g_err[512] = "";

constexpr double kSnap = 1e-12;

bool finite(double x) { return std::isfinite(x); }

// Unit vector with components of magnitude <= kSnap set to exactly 0, so that a view
// at phi = pi/2 in floating point is the axis-parallel case of the paper (Case 2 of
// Sec. 2.2.1; Cases 2-4 of Sec. 3.2.1) and grid-aligned rays take the Sec. 4.1 rule.
void snap3(double v[3])
{
    for (int a = 0; a < 3; ++a)
        if (std::fabs(v[a]) <= kSnap) v[a] = 0.0;
}

void set3(double* dst, double x, double y, double z)
{
    dst[0] = x;
    dst[1] = y;
    dst[2] = z;
}

// 3D parallel-beam frame (Sec. 3.2.1, eqs. 3Dparallel_direction, theta_1, theta_2).
void frame3d(double phi1, double phi2, double th[3], double th1[3], double th2[3])
{
    const double c1 = std::cos(phi1), s1 = std::sin(phi1), c2 = std::cos(phi2), s2 = std::sin(phi2);
    set3(th, c2 * c1, c2 * s1, s2);
    set3(th1, -s1, c1, 0.0);
    set3(th2, -s2 * c1, -s2 * s1, c2);
    snap3(th);
    snap3(th1);
    snap3(th2);
}

bool is2d(int kind)
{
    return kind == XRT_PAR2D || kind == XRT_FAN2D_FLAT || kind == XRT_FAN2D_ARC || kind == XRT_RAYLIST2D;
}

// Is the point strictly outside the closed image box?
bool outside_box(const xrt_grid& g, const double S[3])
{
    const double hx = 0.5 * g.nx * g.dx, hy = 0.5 * g.ny * g.dy;
    if (std::fabs(S[0] - g.cx) > hx || std::fabs(S[1] - g.cy) > hy) return true;
    if (g.nz > 0) {
        const double hz = 0.5 * g.nz * g.dz;
        if (std::fabs(S[2] - g.cz) > hz) return true;
    }
    return false;
}

xrt_status validate(const xrt_grid* g, const xrt_scan* s)
{
    if (!g || !s) { set_error("null grid or scan"); return XRT_E_ARG; }
    if (s->kind < XRT_PAR2D || s->kind > XRT_RAYLIST3D) {
        set_error("unknown scan kind %d", s->kind);
        return XRT_E_ARG;
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 0) { set_error("grid sizes must be positive"); return XRT_E_GEOM; }
    if (!(g->dx > 0) || !(g->dy > 0) || !finite(g->dx) || !finite(g->dy) || !finite(g->cx) || !finite(g->cy)) {
        set_error("grid spacing must be positive and finite");
        return XRT_E_GEOM;
    }
    if (g->nz > 0 && (!(g->dz > 0) || !finite(g->dz) || !finite(g->cz))) {
        set_error("grid dz must be positive and finite");
        return XRT_E_GEOM;
    }
    const int64_t nu = (int64_t)g->nx * g->ny * (g->nz > 0 ? g->nz : 1);
    // image byte offsets are 32-bit (buffer loads with hardware bounds checks)
    if (nu > (int64_t)(INT32_MAX - 15) / 4) { set_error("more than 2^29 - 4 units"); return XRT_E_SIZE; }
    if (is2d(s->kind) != (g->nz == 0)) {
        set_error("scan kind %d does not match a %dD grid", s->kind, g->nz == 0 ? 2 : 3);
        return XRT_E_GEOM;
    }
    if (s->kind == XRT_RAYLIST2D || s->kind == XRT_RAYLIST3D) {
        if (!s->ray_params) { set_error("ray_params is NULL"); return XRT_E_ARG; }
        if (s->n_rays < 1) { set_error("n_rays must be >= 1"); return XRT_E_GEOM; }
        if (s->n_rays > INT32_MAX) { set_error("more than 2^31-1 rays"); return XRT_E_SIZE; }
        const int w = s->kind == XRT_RAYLIST2D ? 2 : 4;
        for (int64_t i = 0; i < s->n_rays * w; ++i)
            if (!finite(s->ray_params[i])) { set_error("non-finite ray parameter"); return XRT_E_GEOM; }
        return XRT_OK;
    }
    if (s->n_views < 1 || s->n_cols < 1 || s->n_rows < 1) {
        set_error("n_views, n_rows, n_cols must be >= 1");
        return XRT_E_GEOM;
    }
    if (is2d(s->kind) && s->n_rows != 1) { set_error("2D scans have n_rows = 1"); return XRT_E_GEOM; }
    if ((int64_t)s->n_views * s->n_rows * s->n_cols > INT32_MAX) {
        set_error("more than 2^31-1 rays");
        return XRT_E_SIZE;
    }
    if (!(s->du > 0) || !finite(s->du) || !finite(s->u0)) { set_error("du must be positive"); return XRT_E_GEOM; }
    if (!is2d(s->kind) && (!(s->dv > 0) || !finite(s->dv) || !finite(s->v0))) {
        set_error("dv must be positive");
        return XRT_E_GEOM;
    }
    if (!s->view_angle) { set_error("view_angle is NULL"); return XRT_E_ARG; }
    for (int i = 0; i < s->n_views; ++i) {
        if (!finite(s->view_angle[i])) { set_error("non-finite view angle"); return XRT_E_GEOM; }
        if (s->view_z && !finite(s->view_z[i])) { set_error("non-finite view_z"); return XRT_E_GEOM; }
    }
    if (s->kind == XRT_PAR3D) {
        if (!s->view_phi2) { set_error("view_phi2 is NULL"); return XRT_E_ARG; }
        for (int i = 0; i < s->n_views; ++i)
            if (!finite(s->view_phi2[i])) { set_error("non-finite view_phi2"); return XRT_E_GEOM; }
    }
    const bool divergent = s->kind == XRT_FAN2D_FLAT || s->kind == XRT_FAN2D_ARC ||
                           s->kind == XRT_CONE_FLAT || s->kind == XRT_CONE_ARC;
    if (divergent) {
        if (!(s->sod > 0) || !finite(s->sod)) { set_error("sod must be positive"); return XRT_E_GEOM; }
        const bool flat = s->kind == XRT_FAN2D_FLAT || s->kind == XRT_CONE_FLAT;
        if (flat && (!(s->sdd > 0) || !finite(s->sdd))) { set_error("sdd must be positive"); return XRT_E_GEOM; }
        if (s->kind == XRT_FAN2D_ARC || s->kind == XRT_CONE_ARC) {
            // equiangular bins must stay inside (-pi/2, pi/2)
            const double ue = 0.5 * (s->n_cols - 1) * s->du + std::fabs(s->u0);
            const double ve = 0.5 * (s->n_rows - 1) * s->dv + std::fabs(s->v0);
            if (ue >= M_PI / 2 || (s->kind == XRT_CONE_ARC && ve >= M_PI / 2)) {
                set_error("equiangular bins must lie in (-pi/2, pi/2)");
                return XRT_E_GEOM;
            }
        }
    }
    return XRT_OK;
}

// FP64 expansion of the scan into per-view vectors (see RayMode).  The rays are the
// paper's: eq. 2Dparalleltofan / 2Dparalleltofan_2 for fans, eqs. equiangular_cone_beam,
// equispaced_cone_beam and the helical variants for cones, written as the line from
// the source through the detector cell (the same line, cheaper per ray).
xrt_status expand(const xrt_grid& g, const xrt_scan& s, DevPlan& D, std::vector<ViewGeom>& views,
                  std::vector<double>& col, std::vector<double>& row, std::vector<double>& rays)
{
    const int kind = s.kind;
    if (kind == XRT_RAYLIST2D || kind == XRT_RAYLIST3D) {
        D.mode = MODE_LIST;
        D.n_views = 1;
        D.n_rows = 1;
        D.n_cols = (int32_t)s.n_rays;
        D.n_rays = s.n_rays;
        rays.resize((size_t)s.n_rays * 6);
        for (int64_t r = 0; r < s.n_rays; ++r) {
            double* t = &rays[(size_t)r * 6];
            if (kind == XRT_RAYLIST2D) {
                const double sv = s.ray_params[2 * r], phi = s.ray_params[2 * r + 1];
                double th[3] = {std::cos(phi), std::sin(phi), 0.0};
                double pe[3] = {-std::sin(phi), std::cos(phi), 0.0};
                snap3(th);
                snap3(pe);
                set3(t, sv * pe[0], sv * pe[1], 0.0);
                set3(t + 3, th[0], th[1], 0.0);
            } else {
                const double* q = s.ray_params + 4 * r;
                double th[3], t1[3], t2[3];
                frame3d(q[2], q[3], th, t1, t2);
                for (int a = 0; a < 3; ++a) {
                    t[a] = q[0] * t1[a] + q[1] * t2[a];
                    t[3 + a] = th[a];
                }
            }
        }
        return XRT_OK;
    }
    D.n_views = s.n_views;
    D.n_rows = s.n_rows;
    D.n_cols = s.n_cols;
    D.n_rays = (int64_t)s.n_views * s.n_rows * s.n_cols;
    D.du = s.du;
    D.ubase = s.u0 - 0.5 * (s.n_cols - 1) * s.du;
    D.dv = is2d(kind) ? 0.0 : s.dv;
    D.vbase = is2d(kind) ? 0.0 : s.v0 - 0.5 * (s.n_rows - 1) * s.dv;
    views.assign((size_t)s.n_views, ViewGeom{});
    for (int v = 0; v < s.n_views; ++v) {
        ViewGeom& V = views[(size_t)v];
        const double ang = s.view_angle[v];
        const double H = s.view_z ? s.view_z[v] : 0.0;
        switch (kind) {
            case XRT_PAR2D: {   // ray t theta + s theta_perp (Sec. 2.2.1)
                double th[3] = {std::cos(ang), std::sin(ang), 0.0};
                double pe[3] = {-std::sin(ang), std::cos(ang), 0.0};
                snap3(th);
                snap3(pe);
                set3(V.A, 0, 0, 0);
                std::memcpy(V.B, pe, sizeof pe);
                set3(V.C, 0, 0, 0);
                std::memcpy(V.E, th, sizeof th);
                D.mode = MODE_PARALLEL;
                break;
            }
            case XRT_PAR3D: {   // ray t theta + s1 theta_1 + s2 theta_2 (Sec. 3.2.1)
                double th[3], t1[3], t2[3];
                frame3d(ang, s.view_phi2[v], th, t1, t2);
                set3(V.A, 0, 0, 0);
                std::memcpy(V.B, t1, sizeof t1);
                std::memcpy(V.C, t2, sizeof t2);
                std::memcpy(V.E, th, sizeof th);
                D.mode = MODE_PARALLEL;
                break;
            }
            case XRT_FAN2D_FLAT:
            case XRT_FAN2D_ARC: {
                // source at D(-sin a, cos a); central ray e = (sin a, -cos a) through the
                // origin; positive bins rotate the ray counter-clockwise, b = (cos a, sin a)
                double e[3] = {std::sin(ang), -std::cos(ang), 0.0};
                double b[3] = {std::cos(ang), std::sin(ang), 0.0};
                snap3(e);
                snap3(b);
                set3(V.A, -s.sod * e[0], -s.sod * e[1], 0.0);
                if (kind == XRT_FAN2D_FLAT) {
                    set3(V.E, s.sdd * e[0], s.sdd * e[1], 0.0);
                    D.mode = MODE_DIVERGENT;
                } else {
                    std::memcpy(V.E, e, sizeof e);
                    D.mode = MODE_ARC;
                }
                std::memcpy(V.B, b, sizeof b);
                set3(V.C, 0, 0, 0);
                if (!outside_box(g, V.A)) {
                    set_error("view %d: source inside the image box", v);
                    return XRT_E_GEOM;
                }
                break;
            }
            default: {   // XRT_CONE_FLAT, XRT_CONE_ARC
                // source at -D (cos p, sin p, 0) + (0, 0, H); u along (-sin p, cos p, 0), v along z
                double e[3] = {std::cos(ang), std::sin(ang), 0.0};
                double b[3] = {-std::sin(ang), std::cos(ang), 0.0};
                snap3(e);
                snap3(b);
                set3(V.A, -s.sod * e[0], -s.sod * e[1], H);
                if (kind == XRT_CONE_FLAT) {
                    set3(V.E, s.sdd * e[0], s.sdd * e[1], 0.0);
                    D.mode = MODE_DIVERGENT;
                } else {
                    std::memcpy(V.E, e, sizeof e);
                    D.mode = MODE_ARC;
                }
                std::memcpy(V.B, b, sizeof b);
                set3(V.C, 0, 0, 1.0);
                if (!outside_box(g, V.A)) {
                    set_error("view %d: source inside the image box", v);
                    return XRT_E_GEOM;
                }
                break;
            }
        }
    }
    if (D.mode == MODE_ARC) {
        col.resize((size_t)s.n_cols * 2);
        row.resize((size_t)s.n_rows * 2);
        for (int c = 0; c < s.n_cols; ++c) {
            const double a = D.ubase + c * s.du;
            col[2 * c] = std::cos(a);
            col[2 * c + 1] = std::sin(a);
        }
        for (int r = 0; r < s.n_rows; ++r) {
            const double b = is2d(kind) ? 0.0 : D.vbase + r * s.dv;
            row[2 * r] = std::cos(b);
            row[2 * r + 1] = std::sin(b);
        }
    }
    return XRT_OK;
}

template <class T>
xrt_status upload(const std::vector<T>& h, void** d)
{
    *d = nullptr;
    if (h.empty()) return XRT_OK;
    hipError_t e = hipMalloc(d, h.size() * sizeof(T));
    if (e != hipSuccess) {
        *d = nullptr;
        (void)hipGetLastError();
        set_error("hipMalloc of %zu bytes failed: %s", h.size() * sizeof(T), hipGetErrorString(e));
        return XRT_E_NOMEM;
    }
    return hip_fail(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
}

void free_plan(xrt_plan* p)
{
    if (!p) return;
    for (void* q : {p->d_views, p->d_col, p->d_row, p->d_rays, p->d_ray2d, p->d_invwz, (void*)p->d_gT, (void*)p->d_imgT, (void*)p->d_imgZ,
                    (void*)p->d_att})
        if (q) (void)hipFree(q);
    delete p;
}

// Tables of the voxel-driven cone adjoint: 1/v of every detector row (v_r is the z
// component of the row's ray direction) and the transposed-sinogram workspace.
xrt_status cone_gather_setup(xrt_plan* p, const std::vector<ViewGeom>& views)
{
    const DevPlan& D = p->dp;
    p->zero_row = -1;
    p->gather_lgs = 2;
    p->helical = 0;
    for (const ViewGeom& V : views) p->helical |= V.A[2] != views[0].A[2] ? 1 : 0;
    p->sz0 = views.empty() ? 0.0 : views[0].A[2];
    // The detector columns that see a pixel are the interval between its corners' u
    // coordinates only when the pixel is in front of the source; require it of the
    // whole image box for every view, otherwise the plan uses the scatter adjoint.
    // sinogram byte offsets are 32-bit in the gather kernel
    p->gather_ok = D.n_rays + kGatherPad <= (int64_t)(INT32_MAX - 15) / 4 ? 1 : 0;
    for (const ViewGeom& V : views) {
        const double en = std::sqrt(V.E[0] * V.E[0] + V.E[1] * V.E[1] + V.E[2] * V.E[2]);
        for (int cnr = 0; cnr < 8; ++cnr) {
            const double P[3] = {D.px0 + ((cnr & 1) ? D.nx * D.pdx : 0.0), D.py0 - ((cnr & 2) ? D.ny * D.pdy : 0.0),
                                 D.pz0 - ((cnr & 4) ? D.nz * D.pdz : 0.0)};
            double depth = 0.0;
            for (int a = 0; a < 3; ++a) depth += (P[a] - V.A[a]) * V.E[a] / en;
            if (!(depth > 1e-6 * en)) p->gather_ok = 0;
        }
    }
    if (!p->gather_ok) return XRT_OK;
    // Bound on the rows whose rays can cross one voxel, for one detector column.  Along
    // a column the horizontal distance h from the source and the ray parameter satisfy
    // tau = h / rho with rho = |E + u B| <= sqrt(sdd^2 + u_max^2); a voxel's rows have
    // v = (z - Sz)/tau over its z range and the pixel's h interval [h_in, h_in + diag],
    // so their spread is at most rho (dz / h_min + |z - Sz|_max diag / h_min^2).
    // A voxel whose shadow reaches the detector has a point with |v| <= vabs (the rows'
    // largest |v|), so |z - Sz| <= vabs tau_max + dz over the whole voxel, tau = h / rho <=
    // hmax / sdd (h: horizontal distance from the source, hmax its largest value over the
    // image box); voxels whose shadows miss the detector add nothing whatever the bound,
    // which matters for helical scans, whose sources travel far beyond the detector's band.
    {
        const double umax = std::fmax(std::fabs(D.ubase), std::fabs(D.ubase + (D.n_cols - 1) * D.du));
        const double rho = std::sqrt(D.sdd * D.sdd + umax * umax);
        const double bx0 = D.px0, bx1 = D.px0 + D.nx * D.pdx, by1 = D.py0, by0 = D.py0 - D.ny * D.pdy;
        const double zhi = D.pz0, zlo = D.pz0 - D.nz * D.pdz;
        double hmin = INFINITY, hmax = 0.0, zrel = 0.0;
        for (const ViewGeom& V : views) {
            const double ddx = std::fmax(std::fmax(bx0 - V.A[0], V.A[0] - bx1), 0.0);
            const double ddy = std::fmax(std::fmax(by0 - V.A[1], V.A[1] - by1), 0.0);
            hmin = std::fmin(hmin, std::sqrt(ddx * ddx + ddy * ddy));
            const double fx = std::fmax(std::fabs(bx0 - V.A[0]), std::fabs(bx1 - V.A[0]));
            const double fy = std::fmax(std::fabs(by0 - V.A[1]), std::fabs(by1 - V.A[1]));
            hmax = std::fmax(hmax, std::sqrt(fx * fx + fy * fy));
            zrel = std::fmax(zrel, std::fmax(std::fabs(zhi - V.A[2]), std::fabs(zlo - V.A[2])));
        }
        const double vabs = std::fmax(std::fabs(D.vbase), std::fabs(D.vbase + (D.n_rows - 1) * D.dv));
        zrel = std::fmin(zrel, (vabs * hmax / D.sdd + D.pdz) * (1.0 + 1e-9));
        const double diag = std::sqrt(D.pdx * D.pdx + D.pdy * D.pdy);
        const double spread = rho * (D.pdz / hmin + zrel * diag / (hmin * hmin)) / D.dv;
        const double nr = std::floor(spread + 1e-6) + 1.0;
        // the 1/v table of the rows lives in LDS (at most 32 KiB)
        if (!(hmin > 0.0) || !(nr <= 8.0) || D.n_rows + 8 > 4096) {
            p->gather_ok = 0;
            return XRT_OK;
        }
        p->gather_nr = (int32_t)nr;
        // columns of one pixel's shadow: it subtends at most diag / hmin radians, and a
        // radian spans at most rho^2 / sdd along the flat detector; the gather fills its
        // per-view column records in slots of the next power of two of that bound + 2
        // (a wider shadow only costs a further pass)
        const double ncol = std::floor(diag / hmin * rho * rho / D.sdd / D.du) + 2.0;
        int lgs = 0;
        while (lgs < 6 && (double)(1 << lgs) < ncol) ++lgs;
        p->gather_lgs = lgs;
    }
    std::vector<double> inv((size_t)D.n_rows);
    for (int r = 0; r < D.n_rows; ++r) {
        const double v = D.vbase + r * D.dv;
        if (v == 0.0) {
            inv[(size_t)r] = 0.0;
            p->zero_row = r;
        } else {
            inv[(size_t)r] = 1.0 / v;
        }
    }
    xrt_status st = upload(inv, &p->d_invwz);
    if (st != XRT_OK) return st;
    void* ws = nullptr;
    hipError_t e = hipMalloc(&ws, (size_t)(D.n_rays + kGatherPad) * sizeof(float));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of the %lld-float adjoint workspace failed: %s", (long long)D.n_rays + kGatherPad,
                  hipGetErrorString(e));
        return XRT_E_NOMEM;
    }
    p->d_gT = (float*)ws;
    return XRT_OK;
}

}  // namespace

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

xrt_status hip_fail(hipError_t e, const char* what)
{
    if (e == hipSuccess) return XRT_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return XRT_E_HIP;
}

xrt_status build_tables(const xrt_grid* grid, const xrt_scan* scan, HostTables& T)
{
    xrt_status st = validate(grid, scan);
    if (st != XRT_OK) return st;
    const xrt_grid& g = *grid;
    T = HostTables{};
    T.kind = scan->kind;
    DevPlan& D = T.dp;
    D.dim = g.nz > 0 ? 3 : 2;
    D.nx = g.nx;
    D.ny = g.ny;
    D.nz = g.nz > 0 ? g.nz : 1;
    D.n_units = (int64_t)D.nx * D.ny * D.nz;
    D.ax = 1.0 / g.dx;
    D.bx = 0.5 * g.nx - g.cx * D.ax;
    D.ay = 1.0 / g.dy;
    D.by = 0.5 * g.ny + g.cy * D.ay;
    if (g.nz > 0) {
        D.az = 1.0 / g.dz;
        D.bz = 0.5 * g.nz + g.cz * D.az;
    } else {
        D.az = 0.0;
        D.bz = 0.5;
    }
    D.pdx = g.dx;
    D.pdy = g.dy;
    D.pdz = g.nz > 0 ? g.dz : 1.0;
    D.px0 = g.cx - 0.5 * g.nx * g.dx;
    D.py0 = g.cy + 0.5 * g.ny * g.dy;
    D.pz0 = g.nz > 0 ? g.cz + 0.5 * g.nz * g.dz : 0.5;
    D.sdd = scan->sdd;
    return expand(g, *scan, D, T.views, T.col, T.row, T.rays);
}

}  // namespace xrt

using namespace xrt;

extern "C" {

xrt_status xrt_plan_create(const xrt_grid* grid, const xrt_scan* scan, int device, xrt_plan** out)
{
    if (!out) { set_error("out is NULL"); return XRT_E_ARG; }
    *out = nullptr;
    HostTables T;
    xrt_status st = build_tables(grid, scan, T);
    if (st != XRT_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        set_error("device %d not available (%d devices)", device, ndev);
        return XRT_E_ARG;
    }
    xrt_plan* p = new (std::nothrow) xrt_plan{};
    if (!p) { set_error("host allocation failed"); return XRT_E_NOMEM; }
    p->device = device;
    p->kind = T.kind;
    p->dp = T.dp;
    DeviceGuard guard(device);
    if (!guard.ok) { delete p; set_error("hipSetDevice(%d) failed", device); return XRT_E_HIP; }
    if ((st = upload(T.views, &p->d_views)) != XRT_OK || (st = upload(T.col, &p->d_col)) != XRT_OK ||
        (st = upload(T.row, &p->d_row)) != XRT_OK || (st = upload(T.rays, &p->d_rays)) != XRT_OK) {
        free_plan(p);
        return st;
    }
    DevPlan& D = p->dp;
    // nested walk for the 3D forward where it measured faster: grids up to 256 units
    // across (the 256^3 cone 2 %, 128-class grids 4-8 %); on 512-wide grids the lanes'
    // z crossings spread over more slabs and the flat form is 11-15 % faster
    D.nest_z = D.dim == 3 && std::max(D.nx, D.ny) <= 256 ? 1 : 0;
    D.views = (const ViewGeom*)p->d_views;
    D.col_cs = (const double*)p->d_col;
    D.row_cs = (const double*)p->d_row;
    D.rays = (const double*)p->d_rays;
    p->zero_row = -1;
    p->gather_ok = 0;
    p->d_imgT = nullptr;
    // 2D gather: the detector coordinate of a pixel's corners bounds its bins when the
    // image lies in front of every source (divergent kinds) -- same test as the cone's
    p->gather2d_ok = 0;
    if (D.dim == 2 && D.mode != MODE_LIST) {
        p->gather2d_ok = 1;
        if (D.mode != MODE_PARALLEL) {
            for (const ViewGeom& V : T.views) {
                const double en = std::sqrt(V.E[0] * V.E[0] + V.E[1] * V.E[1]);
                for (int cnr = 0; cnr < 4; ++cnr) {
                    const double P[2] = {D.px0 + ((cnr & 1) ? D.nx * D.pdx : 0.0), D.py0 - ((cnr & 2) ? D.ny * D.pdy : 0.0)};
                    const double depth = ((P[0] - V.A[0]) * V.E[0] + (P[1] - V.A[1]) * V.E[1]) / en;
                    if (!(depth > 1e-6 * en)) p->gather2d_ok = 0;
                }
            }
        }
    }
    // candidate column ranges of the gathers: |u| / du up to the detector's edge times the
    // reciprocal's relative error bound, plus the exact ranges' own slack
    D.uslack = 1e-7 + std::ldexp(std::fmax(std::fabs(D.ubase), std::fabs(D.ubase + (D.n_cols - 1) * D.du)) / D.du + 1.0,
                                 -20);
    D.ray2d = nullptr;
    p->d_ray2d = nullptr;
    D.g2_umax2 = 0.0;
    D.g2_r = 0.0;
    if (p->gather2d_ok && D.mode == MODE_DIVERGENT) {
        // A pixel lies in the disc of radius rho (half its diagonal) around its centre; the
        // rays through the disc deviate from the centre's ray by at most
        // alpha = asin(rho / |centre - source|) <= A rho / depth (A = asin(x) / x at the
        // largest x = rho / depth of the image box, depth = distance along E); on the flat
        // detector u = sdd tan(theta) moves by at most sdd sec^2(theta) per radian, with
        // tan(theta) <= max(|u| on the detector (one bin beyond its edge), |u_c|) / sdd.
        const double rho = 0.5 * std::sqrt(D.pdx * D.pdx + D.pdy * D.pdy);
        double dmin = INFINITY;
        for (const ViewGeom& V : T.views) {
            const double en = std::sqrt(V.E[0] * V.E[0] + V.E[1] * V.E[1]);
            for (int cnr = 0; cnr < 4; ++cnr) {
                const double P[2] = {D.px0 + ((cnr & 1) ? D.nx * D.pdx : 0.0), D.py0 - ((cnr & 2) ? D.ny * D.pdy : 0.0)};
                dmin = std::fmin(dmin, ((P[0] - V.A[0]) * V.E[0] + (P[1] - V.A[1]) * V.E[1]) / en);
            }
        }
        const double x = rho / dmin;
        if (x < 0.5) {
            const double A = std::asin(x) / x * (1.0 + 1e-9);
            const double um = std::fmax(std::fabs(D.ubase), std::fabs(D.ubase + (D.n_cols - 1) * D.du)) + D.du;
            D.g2_umax2 = um * um;
            // hw (bins) = (sdd^2 + m) / sdd * alpha / du with alpha <= A rho sdd / D
            D.g2_r = A * rho / D.du;
        }
    }
    if (p->gather2d_ok) {
        // per (view, column) for rays that fan out, per view for parallel beams:
        // |d| / d_x and |d| / d_y of the ray direction d (as the forward builds it), so that
        // the gather's ray parameters are physical lengths
        const bool per_col = D.mode != MODE_PARALLEL;
        const int64_t nc = per_col ? D.n_cols : 1;
        std::vector<double> tab((size_t)(D.n_views * nc * 2));
        for (int32_t v = 0; v < D.n_views; ++v) {
            const ViewGeom& V = T.views[(size_t)v];
            for (int64_t c = 0; c < nc; ++c) {
                double dx = V.E[0], dy = V.E[1];
                if (D.mode == MODE_DIVERGENT) {
                    const double u = (double)c * D.du + D.ubase;
                    dx = V.E[0] + u * V.B[0];
                    dy = V.E[1] + u * V.B[1];
                } else if (D.mode == MODE_ARC) {
                    const double ca = T.col[(size_t)(2 * c)], sa = T.col[(size_t)(2 * c + 1)];
                    dx = ca * V.E[0] + sa * V.B[0];
                    dy = ca * V.E[1] + sa * V.B[1];
                }
                const double n = std::sqrt(dx * dx + dy * dy);
                // a zero component: 0 for parallel beams; for rays from a source, +1e300 (x)
                // and -1e300 (y), which turn the clip of a unit in front of the source into
                // the half-open membership test (x in [xa, xb), y in (ya, yb])
                const double zx = per_col ? 1e300 : 0.0, zy = per_col ? -1e300 : 0.0;
                tab[(size_t)((v * nc + c) * 2)] = dx != 0.0 ? n / dx : zx;
                tab[(size_t)((v * nc + c) * 2 + 1)] = dy != 0.0 ? n / dy : zy;
            }
        }
        if ((st = upload(tab, &p->d_ray2d)) != XRT_OK) {
            free_plan(p);
            return st;
        }
        D.ray2d = (const double*)p->d_ray2d;
    }
    bool any_y = false;   // a view whose u axis runs closer to y than to x
    for (const ViewGeom& V : T.views) any_y = any_y || std::fabs(V.B[1]) > std::fabs(V.B[0]);
    if (D.mode != MODE_LIST && any_y) {
        void* ws = nullptr;
        if (hipMalloc(&ws, (size_t)D.n_units * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            free_plan(p);
            set_error("hipMalloc of the %lld-float forward workspace failed", (long long)D.n_units);
            return XRT_E_NOMEM;
        }
        p->d_imgT = (float*)ws;
    }
    // Cone scans: the rays of one detector column share their xy path, so with at least 64
    // rows a wavefront takes 64 rows of one column by default (column packets, reading a
    // z-fastest copy of the image; the 256^3 cone forward 19.0 -> 11.3 ms)
    p->d_imgZ = nullptr;
    if ((p->kind == XRT_CONE_FLAT || p->kind == XRT_CONE_ARC) && D.n_rows >= 64) {
        void* ws = nullptr;
        if (hipMalloc(&ws, (size_t)D.n_units * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            free_plan(p);
            set_error("hipMalloc of the %lld-float column-packet workspace failed", (long long)D.n_units);
            return XRT_E_NOMEM;
        }
        p->d_imgZ = (float*)ws;
        D.packet_cols = 1;
    }
    if (p->kind == XRT_CONE_FLAT && (st = cone_gather_setup(p, T.views)) != XRT_OK) {
        free_plan(p);
        return st;
    }
    *out = p;
    return XRT_OK;
}

xrt_status xrt_plan_destroy(xrt_plan* plan)
{
    if (!plan) return XRT_OK;
    DeviceGuard guard(plan->device);
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return XRT_OK;
}

xrt_status xrt_plan_sizes(const xrt_plan* plan, int64_t* n_rays, int64_t* n_units)
{
    if (!plan) { set_error("plan is NULL"); return XRT_E_ARG; }
    if (n_rays) *n_rays = plan->dp.n_rays;
    if (n_units) *n_units = plan->dp.n_units;
    return XRT_OK;
}

xrt_status xrt_forward(xrt_plan* plan, const float* d_img, float* d_sino, int32_t batch, void* stream)
{
    if (!plan || !d_img || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 65535) { set_error("batch must be in [1, 65535]"); return XRT_E_ARG; }
    DeviceGuard guard(plan->device);
    return launch_forward(plan, d_img, d_sino, batch, (hipStream_t)stream);
}

namespace {

// The attenuated transform's plan workspace of 2 n_units floats, allocated on first use
// (never during stream capture: a captured call without it takes the path that needs
// none and allocates nothing).  XRT_OK with plan->d_att possibly still NULL.
xrt_status ensure_att_workspace(xrt_plan* plan, void* stream)
{
    if (plan->d_att != nullptr || plan->dp.n_units * 8 > (int64_t)INT32_MAX - 16) return XRT_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusActive;
    }
    if (cs != hipStreamCaptureStatusNone) return XRT_OK;
    void* ws = nullptr;
    if (hipMalloc(&ws, (size_t)plan->dp.n_units * 2 * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of the %lld-float attenuated-transform workspace failed", (long long)plan->dp.n_units * 2);
        return XRT_E_NOMEM;
    }
    plan->d_att = (float*)ws;
    return XRT_OK;
}

}  // namespace

xrt_status xrt_forward_attenuated(xrt_plan* plan, const float* d_img, const float* d_mu, int32_t mu_per_image,
                                  float* d_sino, int32_t batch, void* stream)
{
    if (!plan || !d_img || !d_mu || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 65535) { set_error("batch must be in [1, 65535]"); return XRT_E_ARG; }
    DeviceGuard guard(plan->device);
    const int64_t mu_stride = mu_per_image ? plan->dp.n_units : 0;
    // (f, mu) interleaved in the workspace, so that each candidate takes one 8-byte load
    const xrt_status st = ensure_att_workspace(plan, stream);
    if (st != XRT_OK) return st;
    if (plan->d_att != nullptr)
        return launch_forward_att_pairs(plan, d_img, d_mu, mu_stride, d_sino, batch, (hipStream_t)stream);
    return launch_forward_att(plan, d_img, d_mu, mu_stride, d_sino, batch, (hipStream_t)stream);
}

xrt_status xrt_adjoint_attenuated(xrt_plan* plan, const float* d_sino, const float* d_mu, int32_t mu_per_image,
                                  float* d_img, int32_t batch, void* stream)
{
    if (!plan || !d_img || !d_mu || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 65535) { set_error("batch must be in [1, 65535]"); return XRT_E_ARG; }
    DeviceGuard guard(plan->device);
    // the map's y-fastest copy for the views that scatter into the y-fastest layout
    // lives in the workspace's first half
    const xrt_status st = ensure_att_workspace(plan, stream);
    if (st != XRT_OK) return st;
    return launch_adjoint_att(plan, d_sino, d_mu, mu_per_image ? plan->dp.n_units : 0, d_img, batch,
                              (hipStream_t)stream, plan->d_att);
}

namespace {

xrt_status adjoint_impl(xrt_plan* plan, const float* d_sino, float* d_img, int32_t batch, int32_t mode,
                        void* stream, const float* wt, int64_t wt_stride)
{
    if (!plan || !d_img || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 65535) { set_error("batch must be in [1, 65535]"); return XRT_E_ARG; }
    if (mode != XRT_ADJ_AUTO && mode != XRT_ADJ_SCATTER && mode != XRT_ADJ_GATHER) {
        set_error("unknown adjoint mode %d", mode);
        return XRT_E_ARG;
    }
    const bool cone_gather = plan->kind == XRT_CONE_FLAT && plan->gather_ok;
    const bool gather2d = plan->gather2d_ok != 0;
    if (mode == XRT_ADJ_GATHER && !cone_gather && !gather2d) {
        set_error("the voxel-driven adjoint needs a 2D scan or a flat-detector cone scan with the image in "
                  "front of every source position");
        return XRT_E_UNSUPPORTED;
    }
    DeviceGuard guard(plan->device);
    const hipStream_t s = (hipStream_t)stream;
    if (mode != XRT_ADJ_SCATTER && cone_gather)
        return launch_adjoint_cone_gather(plan, d_sino, d_img, batch, s, wt, wt_stride);
    if (mode != XRT_ADJ_SCATTER && gather2d)
        return launch_adjoint_gather2d(plan, d_sino, d_img, batch, s, wt, wt_stride);
    return launch_adjoint_scatter(plan, d_sino, d_img, batch, s, wt, wt_stride);
}

}  // namespace

xrt_status xrt_plan_adjoint_info(const xrt_plan* plan, xrt_adjoint_info* out)
{
    if (!plan || !out) { set_error("null argument"); return XRT_E_ARG; }
    *out = xrt_adjoint_info{XRT_ADJ_SCATTER, 0, 0, 0, 0, -1};
    if (plan->kind == XRT_CONE_FLAT && plan->gather_ok) {
        const int32_t nz = plan->dp.nz, nr = plan->gather_nr;
        out->algorithm = XRT_ADJ_GATHER;
        out->voxels_per_lane = nz <= 64 ? 1 : nz <= 128 ? 2 : 4;
        // the kernel instantiations of launch_adjoint_cone_gather
        out->row_bound = nr <= 2 ? 2 : nr <= 4 ? nr : nr <= 6 ? 6 : 8;
        out->column_slots = 1 << plan->gather_lgs;
        out->helical = plan->helical;
        out->zero_row = plan->zero_row;
    } else if (plan->gather2d_ok) {
        out->algorithm = XRT_ADJ_GATHER;
    }
    return XRT_OK;
}

xrt_status xrt_adjoint(xrt_plan* plan, const float* d_sino, float* d_img, int32_t batch, int32_t mode,
                       void* stream)
{
    return adjoint_impl(plan, d_sino, d_img, batch, mode, stream, nullptr, 0);
}

xrt_status xrt_forward_simplex(xrt_plan* plan, const float* d_img, float* d_sino, int32_t batch, void* stream)
{
    if (!plan || !d_img || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 65535) { set_error("batch must be in [1, 65535]"); return XRT_E_ARG; }
    DeviceGuard guard(plan->device);
    return launch_forward_simplex(plan, d_img, d_sino, batch, (hipStream_t)stream);
}

xrt_status xrt_adjoint_simplex(xrt_plan* plan, const float* d_sino, float* d_img, int32_t batch, void* stream)
{
    if (!plan || !d_img || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 65535) { set_error("batch must be in [1, 65535]"); return XRT_E_ARG; }
    DeviceGuard guard(plan->device);
    return launch_adjoint_simplex(plan, d_sino, d_img, batch, (hipStream_t)stream);
}

xrt_status xrt_forward_weighted(xrt_plan* plan, const float* d_img, const float* d_w, int32_t w_per_image,
                                float* d_sino, int32_t batch, void* stream)
{
    if (!plan || !d_img || !d_w || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 65535) { set_error("batch must be in [1, 65535]"); return XRT_E_ARG; }
    DeviceGuard guard(plan->device);
    return launch_forward(plan, d_img, d_sino, batch, (hipStream_t)stream, d_w,
                          w_per_image ? plan->dp.n_rays : 0);
}

xrt_status xrt_adjoint_weighted(xrt_plan* plan, const float* d_sino, const float* d_w, int32_t w_per_image,
                                float* d_img, int32_t batch, int32_t mode, void* stream)
{
    if (!d_w) { set_error("null argument"); return XRT_E_ARG; }
    return adjoint_impl(plan, d_sino, d_img, batch, mode, stream, d_w,
                        plan != nullptr && w_per_image ? plan->dp.n_rays : 0);
}

xrt_status xrt_forward_interleaved(xrt_plan* plan, const float* d_img, float* d_sino, int32_t batch, void* stream)
{
    if (!plan || !d_img || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 64) { set_error("interleaved batch must be in [1, 64]"); return XRT_E_ARG; }
    if (plan->dp.n_units * batch * 4 > (int64_t)INT32_MAX - 16) {
        set_error("interleaved images too large for 32-bit offsets");
        return XRT_E_SIZE;
    }
    DeviceGuard guard(plan->device);
    return launch_forward_il(plan, d_img, d_sino, batch, (hipStream_t)stream);
}

xrt_status xrt_adjoint_interleaved(xrt_plan* plan, const float* d_sino, float* d_img, int32_t batch, void* stream)
{
    if (!plan || !d_img || !d_sino) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 64) { set_error("interleaved batch must be in [1, 64]"); return XRT_E_ARG; }
    if (!plan->gather2d_ok) {
        set_error("the interleaved adjoint needs a 2D scan with the image in front of every source position");
        return XRT_E_UNSUPPORTED;
    }
    if (plan->dp.n_rays * batch * 4 > (int64_t)INT32_MAX - 16) {
        set_error("interleaved sinograms too large for 32-bit offsets");
        return XRT_E_SIZE;
    }
    DeviceGuard guard(plan->device);
    return launch_adjoint_gather2d_il(plan, d_sino, d_img, batch, (hipStream_t)stream);
}

xrt_status xrt_ray_transmission(xrt_plan* plan, const float* d_mu, float* d_w, int32_t batch, void* stream)
{
    if (!plan || !d_mu || !d_w) { set_error("null argument"); return XRT_E_ARG; }
    if (batch < 1 || batch > 65535) { set_error("batch must be in [1, 65535]"); return XRT_E_ARG; }
    DeviceGuard guard(plan->device);
    const hipStream_t s = (hipStream_t)stream;
    xrt_status st = launch_forward(plan, d_mu, d_w, batch, s);
    if (st != XRT_OK) return st;
    return launch_transmission(d_w, d_w, plan->dp.n_rays * (int64_t)batch, s);
}

xrt_status xrt_ray_hit_counts(xrt_plan* plan, int64_t first, int64_t n, double eps, int32_t* d_counts,
                              void* stream)
{
    if (!plan || !d_counts) { set_error("null argument"); return XRT_E_ARG; }
    if (first < 0 || n < 0 || first + n > plan->dp.n_rays || !(eps >= 0)) {
        set_error("bad ray range or eps");
        return XRT_E_ARG;
    }
    DeviceGuard guard(plan->device);
    return launch_hit_counts(plan, first, n, eps, d_counts, (hipStream_t)stream);
}

xrt_status xrt_ray_hits(xrt_plan* plan, int64_t first, int64_t n, double eps, const int64_t* d_offsets,
                        int32_t* d_idx, float* d_len, void* stream)
{
    if (!plan || !d_offsets || !d_idx || !d_len) { set_error("null argument"); return XRT_E_ARG; }
    if (first < 0 || n < 0 || first + n > plan->dp.n_rays || !(eps >= 0)) {
        set_error("bad ray range or eps");
        return XRT_E_ARG;
    }
    DeviceGuard guard(plan->device);
    return launch_hits(plan, first, n, eps, d_offsets, d_idx, d_len, (hipStream_t)stream);
}

const char* xrt_status_str(int32_t status)
{
    switch (status) {
        case XRT_OK: return "XRT_OK";
        case XRT_E_ARG: return "XRT_E_ARG (invalid argument)";
        case XRT_E_GEOM: return "XRT_E_GEOM (invalid geometry)";
        case XRT_E_SIZE: return "XRT_E_SIZE (size limit exceeded)";
        case XRT_E_HIP: return "XRT_E_HIP (HIP runtime error)";
        case XRT_E_NOMEM: return "XRT_E_NOMEM (allocation failed)";
        case XRT_E_UNSUPPORTED: return "XRT_E_UNSUPPORTED";
        default: return "unknown xrt_status";
    }
}

const char* xrt_last_error(void) { return g_err; }

}  // extern "C"
