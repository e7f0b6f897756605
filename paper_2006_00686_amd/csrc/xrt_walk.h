// Ray construction and the slab walk of the discrete X-ray transform, shared by the
// gfx950 kernels and by a host build used to check bounds and results on the CPU.
//
// One ray at a time:
//   1. the ray is built in FP64 from the plan's per-view vectors and mapped to index
//      space q(t) = q0 + t w, in which unit (k,j,i) is [i,i+1) x [j,j+1) x [k,k+1)
//      (half-open: the bigger-index resolution of grid-aligned rays, Sec. 4.1);
//   2. the line is clipped to the image box;
//   3. the slabs of the driving axis are walked -- the axis along which the ray advances
//      fastest in index space, so that every other axis changes by at most one unit per
//      slab (|tan phi| <= 1 in eq. restriction_j; the "given i, j or k" choice of
//      Sec. 3.2.1 and Sec. 4.3).  Within a slab the candidate units are those whose
//      secondary indices satisfy the range conditions (eqs. restriction_j,
//      restriction_j_3D, restriction_k_3D_1): the index at slab entry and, if the ray
//      crosses a secondary grid plane before leaving the slab, its successor.  Each
//      candidate's C_low (largest entry parameter) and C_up (smallest exit parameter)
//      are formed from the slab bounds and the secondary crossing parameters; the unit
//      is hit iff C_low < C_up (eqs. conditions_2D_1, conditions_3D_1) and contributes
//      len = C_up - C_low (eqs. range_length, range_length_3D).
//
// The crossing parameters are FP64 (full-rate vector FP64 on CDNA): an FP32 parameter
// measured from a point ~200 units away carries ~1.5e-5 absolute error, which alone
// breaks a 1e-5 relative bound on the line integral of a grazing ray.
#pragma once

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "xrt_internal.h"

#define XRT_HD __host__ __device__ __forceinline__

namespace xrt {

constexpr double kInf = __builtin_huge_val();

struct Ray {
    double q[3];    // index-space point
    double w[3];    // index-space direction (per unit of the ray parameter)
    double scale;   // physical length per unit of the ray parameter (|d|)
    int32_t st[3];  // memory strides of the x, y, z unit indices in the image read
};

// Ray of linear index r (sinogram order [view][row][col]) in index space.
template <int DIM, int MODE>
XRT_HD void make_ray(const DevPlan& P, int32_t r, Ray& R)
{
    double p[3], d[3];
    if constexpr (MODE == MODE_LIST) {
        const double* t = P.rays + 6 * (int64_t)r;
#pragma unroll
        for (int a = 0; a < 3; ++a) { p[a] = t[a]; d[a] = t[3 + a]; }
    } else {
        const uint32_t per_view = (uint32_t)P.n_rows * (uint32_t)P.n_cols;
        const uint32_t view = (uint32_t)r / per_view;
        const uint32_t rem = (uint32_t)r - view * per_view;
        const uint32_t row = rem / (uint32_t)P.n_cols;
        const uint32_t col = rem - row * (uint32_t)P.n_cols;
        const ViewGeom& V = P.views[view];
        if constexpr (MODE == MODE_ARC) {
            const double ca = P.col_cs[2 * col], sa = P.col_cs[2 * col + 1];
            const double cb = P.row_cs[2 * row], sb = P.row_cs[2 * row + 1];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                p[a] = V.A[a];
                d[a] = cb * (ca * V.E[a] + sa * V.B[a]) + sb * V.C[a];
            }
        } else {
            const double u = fma((double)col, P.du, P.ubase);
            const double v = fma((double)row, P.dv, P.vbase);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if constexpr (MODE == MODE_PARALLEL) {
                    p[a] = V.A[a] + u * V.B[a] + v * V.C[a];
                    d[a] = V.E[a];
                } else {
                    p[a] = V.A[a];
                    d[a] = V.E[a] + u * V.B[a] + v * V.C[a];
                }
            }
        }
    }
    if constexpr (DIM == 2) { d[2] = 0.0; p[2] = 0.0; }
    R.q[0] = fma(p[0], P.ax, P.bx);
    R.q[1] = fma(-p[1], P.ay, P.by);
    R.q[2] = fma(-p[2], P.az, P.bz);
    R.w[0] = d[0] * P.ax;
    R.w[1] = -d[1] * P.ay;
    R.w[2] = -d[2] * P.az;
    R.scale = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    R.st[0] = 1;
    R.st[1] = P.nx;
    R.st[2] = P.nx * P.ny;
}

// State of one axis during the walk.
struct Axis {
    double q, w, inv;   // index-space origin and direction component, 1/w
    double tn;          // parameter of the next grid-plane crossing (inf: none)
    double m;           // index of that plane
    double sg;          // +1 / -1: direction of travel along the axis
    int32_t n, st;      // units along the axis, memory stride of the axis
    int32_t idx;        // unit index at the chord entry
    int32_t ncr;        // grid planes crossed inside the chord
};

XRT_HD int32_t clampi(int32_t v, int32_t lo, int32_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

XRT_HD void axis_swap(Axis& a, Axis& b)
{
    Axis t = a;
    a = b;
    b = t;
}

// Crossing parameters of plane m: the same expression is used for the box faces in the
// clip, so a face is never crossed before the chord ends (no out-of-range index).
XRT_HD double plane_t(double m, const Axis& A)
{
    return (m - A.q) * A.inv;
}

template <int DIM>
XRT_HD bool setup_axes(const DevPlan& P, const Ray& R, Axis* ax,
                                           double& tin, double& tout)
{
    const int32_t n[3] = {P.nx, P.ny, P.nz};
    const int32_t st[3] = {R.st[0], R.st[1], R.st[2]};
    tin = -kInf;
    tout = kInf;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        Axis& A = ax[a];
        A.q = R.q[a];
        A.w = R.w[a];
        A.n = n[a];
        A.st = st[a];
        if (A.w != 0.0) {
            A.inv = 1.0 / A.w;
            const double t0 = (0.0 - A.q) * A.inv;
            const double t1 = ((double)A.n - A.q) * A.inv;
            tin = fmax(tin, fmin(t0, t1));
            tout = fmin(tout, fmax(t0, t1));
        } else {
            A.inv = 0.0;
            inside = inside && (A.q >= 0.0) && (A.q < (double)A.n);
        }
    }
    if (!inside || !(tin < tout)) return false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        Axis& A = ax[a];
        if (A.w != 0.0) {
            const double ein = fma(tin, A.w, A.q);
            const double eout = fma(tout, A.w, A.q);
            int32_t iin, iout;
            if (A.w > 0.0) {
                iin = (int32_t)floor(ein);
                iout = (int32_t)ceil(eout) - 1;
                A.sg = 1.0;
            } else {
                iin = (int32_t)ceil(ein) - 1;
                iout = (int32_t)floor(eout);
                A.sg = -1.0;
            }
            iin = clampi(iin, 0, A.n - 1);
            iout = clampi(iout, 0, A.n - 1);
            A.idx = iin;
            A.ncr = iout > iin ? iout - iin : iin - iout;
            A.m = (double)(A.w > 0.0 ? iin + 1 : iin);
            A.tn = plane_t(A.m, A);
        } else {
            A.idx = (int32_t)floor(A.q);
            A.ncr = 0;
            A.sg = 0.0;
            A.m = 0.0;
            A.tn = kInf;
        }
    }
    // driving axis first
    if (fabs(ax[1].w) > fabs(ax[0].w)) axis_swap(ax[0], ax[1]);
    if constexpr (DIM == 3) {
        if (fabs(ax[2].w) > fabs(ax[0].w)) axis_swap(ax[0], ax[2]);
    }
    return true;
}

// A visitor with a member start(tin) is told the ray parameter at which the chord enters
// the image; the pieces it is then given follow each other without gaps from there.
template <class V, class = void>
struct wants_start : std::false_type {};
template <class V>
struct wants_start<V, std::void_t<decltype(&V::start)>> : std::true_type {};

// A visitor with members two_h / three_h is also told, per later candidate, whether it can
// have a positive length: the second of a slab's candidates iff some secondary crossing
// lies in the slab (its length is then >= 0, 0 only where two crossings coincide), the
// third iff both do (its length is then > 0).  The flags come from the crossing tests the
// walk makes anyway, so a visitor that only needs "may be hit" skips a compare per
// candidate; one that adds len * value gets the same sums (a flagged candidate of length
// 0 adds 0).
template <class V, class = void>
struct wants_flags : std::false_type {};
template <class V>
struct wants_flags<V, std::void_t<decltype(&V::three_h)>> : std::true_type {};

// Walk the chord slab by slab.  The visitor receives the candidate units of every slab
// with their C_up - C_low in ray-parameter units: vis.two(I1, l1, I2, l2) (2D) or
// vis.three(I1, l1, I2, l2, I3, l3) (3D), where I1 -- the unit the ray is in at slab
// entry -- is always a valid unit with l1 >= 0, and I2, I3 are valid units only when
// their length is positive (<= 0: not a hit; always finite).  Indices are in units of
// Visit::kIndexScale (1: element index, 4: byte offset).
//
// The first slab and the last two are walked with the exact per-slab expressions (every
// crossing parameter is (plane - q) / w, the expression of the box clip, so no face of
// the box is crossed before the chord ends).  The slabs in between keep, per secondary
// axis, the distance r from the slab start to the next crossing and step it by the slab
// width dt0 (a DDA in the ray parameter): two fewer exact evaluations per slab and no
// bounds logic, which the one-slab margin to the chord's end makes unnecessary.
//
// NEST (3D): the interior slabs in which the ray crosses no plane of the second secondary
// axis take a cheaper 2D form in an inner loop (same candidates, lengths and order of the
// visits).  Lanes of a wavefront then wait for each other at those crossings, which pays
// where the lanes' crossings fall in nearly the same slabs (coarse grids seen from far
// away); the flat form is the default.
template <int DIM, bool NEST = false, class Visit>
XRT_HD void walk(const DevPlan& P, const Ray& R, Visit& vis)
{
    constexpr double kNone = 1e300;   // "no further crossing" (finite: 0 * l stays 0)
    Axis ax[3];
    double tin, tout;
    if (!setup_axes<DIM>(P, R, ax, tin, tout)) return;
    if constexpr (wants_start<Visit>::value) vis.start(tin);
    constexpr int32_t SC = Visit::kIndexScale;
    auto emit2 = [&](int32_t I1, double l1, int32_t I2, double l2, bool h2) {
        if constexpr (wants_flags<Visit>::value)
            vis.two_h(I1, l1, I2, l2, h2);
        else
            vis.two(I1, l1, I2, l2);
    };
    auto emit3 = [&](int32_t I1, double l1, int32_t I2, double l2, bool h2, int32_t I3, double l3, bool h3) {
        if constexpr (wants_flags<Visit>::value)
            vis.three_h(I1, l1, I2, l2, h2, I3, l3, h3);
        else
            vis.three(I1, l1, I2, l2, I3, l3);
    };

    int32_t I = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) I += ax[a].idx * ax[a].st * SC;
    const int32_t sd0 = (int32_t)ax[0].sg * ax[0].st * SC;
    const int32_t sd1 = (int32_t)ax[1].sg * ax[1].st * SC;
    const double q0 = ax[0].q, inv0 = ax[0].inv, sg0 = ax[0].sg, dt0 = fabs(ax[0].inv);
    double m0 = ax[0].m;   // index of the driving plane that ends the current slab
    const double q1 = ax[1].q, inv1 = ax[1].inv, sg1 = ax[1].sg;
    double m1 = ax[1].m, tn1 = ax[1].w != 0.0 ? ax[1].tn : kNone;
    double q2 = 0.0, inv2 = 0.0, sg2 = 0.0, m2 = 0.0, tn2 = kNone;
    int32_t sd2 = 0;
    if constexpr (DIM == 3) {
        q2 = ax[2].q;
        inv2 = ax[2].inv;
        sg2 = ax[2].sg;
        m2 = ax[2].m;
        tn2 = ax[2].w != 0.0 ? ax[2].tn : kNone;
        sd2 = (int32_t)ax[2].sg * ax[2].st * SC;
    }
    double tx0 = tin;
    const int32_t nslab = ax[0].ncr + 1;

    // one slab with the exact expressions
    auto exact_slab = [&](bool last) {
        const double tx1 = last ? tout : fmin(plane_t(m0, ax[0]), tout);
        if constexpr (DIM == 2) {
            const double l1 = fmin(tx1, tn1) - tx0;
            const double l2 = tx1 - tn1;
            const bool c1 = tn1 < tx1;
            const int32_t Iend = c1 ? I + sd1 : I;
            emit2(I, fmax(l1, 0.0), Iend, l2, c1);
            if (c1) {
                m1 += sg1;
                tn1 = (m1 - q1) * inv1;
            }
            I = Iend + sd0;
        } else {
            const double a = fmin(tn1, tn2), b = fmax(tn1, tn2);
            const double l1 = fmin(tx1, a) - tx0;
            const double l2 = fmin(tx1, b) - a;
            const double l3 = tx1 - b;
            const bool c1 = tn1 < tx1, c2 = tn2 < tx1;
            const int32_t Imid = I + (tn1 < tn2 ? sd1 : sd2);
            const int32_t Iend = I + (c1 ? sd1 : 0) + (c2 ? sd2 : 0);
            emit3(I, fmax(l1, 0.0), Imid, l2, c1 || c2, Iend, l3, c1 && c2);
            if (c1) {
                m1 += sg1;
                tn1 = (m1 - q1) * inv1;
            }
            if (c2) {
                m2 += sg2;
                tn2 = (m2 - q2) * inv2;
            }
            I = Iend + sd0;
        }
        m0 += sg0;
        tx0 = tx1;
    };

    exact_slab(nslab == 1);
    int32_t left = nslab - 1;
    if (left > 2) {
        const int32_t nint = left - 2;
        const double dt1 = ax[1].w != 0.0 ? fabs(inv1) : kNone;
        const double e1 = dt1 - dt0;
        double r1 = fmax(tn1 - tx0, 0.0);
        const double r1s = r1;
        int32_t n1 = 0;
        if constexpr (DIM == 2) {
#pragma unroll 2
            for (int32_t s = nint; s > 0; --s) {
                const double l1 = fmin(r1, dt0);
                const double l2 = dt0 - r1;
                const bool c1 = r1 < dt0;
                const int32_t Iend = c1 ? I + sd1 : I;
                emit2(I, l1, Iend, l2, c1);
                r1 += c1 ? e1 : -dt0;
                I = Iend + sd0;
            }
        } else {
            const double dt2 = ax[2].w != 0.0 ? fabs(inv2) : kNone;
            const double e2 = dt2 - dt0;
            double r2 = fmax(tn2 - tx0, 0.0);
            const double r2s = r2;
            if constexpr (!NEST) {
#pragma unroll 2
                for (int32_t s = nint; s > 0; --s) {
                    const double a = fmin(r1, r2), b = fmax(r1, r2);
                    const double l1 = fmin(a, dt0);
                    const double l2 = fmin(b, dt0) - a;
                    const double l3 = dt0 - b;
                    const bool c1 = r1 < dt0, c2 = r2 < dt0;
                    const int32_t Imid = I + (r1 < r2 ? sd1 : sd2);
                    const int32_t Iend = I + (c1 ? sd1 : 0) + (c2 ? sd2 : 0);
                    emit3(I, l1, Imid, l2, c1 || c2, Iend, l3, c1 && c2);
                    r1 += c1 ? e1 : -dt0;
                    r2 += c2 ? e2 : -dt0;
                    I = Iend + sd0;
                }
            } else {
                int32_t s = nint;
                while (s > 0) {
                    // slabs in which the ray crosses no plane of the second secondary axis
                    // (r2 >= dt0): the candidates and lengths of the general slab below
                    // reduce to those of a 2D slab (its third length is dt0 - r2 <= 0)
#pragma unroll 2
                    for (; s > 0 && r2 >= dt0; --s) {
                        const double l1 = fmin(r1, dt0);
                        const double l2 = dt0 - r1;
                        const bool c1 = r1 < dt0;
                        const int32_t Iend = c1 ? I + sd1 : I;
                        emit2(I, l1, Iend, l2, c1);
                        r1 += c1 ? e1 : -dt0;
                        r2 -= dt0;
                        I = Iend + sd0;
                    }
                    if (s > 0) {
                        const double a = fmin(r1, r2), b = fmax(r1, r2);
                        const double l1 = fmin(a, dt0);
                        const double l2 = fmin(b, dt0) - a;
                        const double l3 = dt0 - b;
                        const bool c1 = r1 < dt0, c2 = r2 < dt0;
                        const int32_t Imid = I + (r1 < r2 ? sd1 : sd2);
                        const int32_t Iend = I + (c1 ? sd1 : 0) + (c2 ? sd2 : 0);
                        emit3(I, l1, Imid, l2, c1 || c2, Iend, l3, c1 && c2);
                        r1 += c1 ? e1 : -dt0;
                        r2 += c2 ? e2 : -dt0;
                        I = Iend + sd0;
                        --s;
                    }
                }
            }
            // crossings taken along the second secondary axis (see n1 below)
            const int32_t n2 = (int32_t)rint((r2 - r2s + (double)nint * dt0) / dt2);
            if (n2 > 0) {
                m2 += sg2 * (double)n2;
                tn2 = (m2 - q2) * inv2;
            }
        }
        // crossings taken along the first secondary axis: every slab moved r by -dt0 and
        // every crossing added dt1 (r - r_start + nint dt0 = n dt1, up to rounding far
        // below dt1 / 2; an axis without crossings keeps r = 1e300 and gives n = 0)
        n1 = (int32_t)rint((r1 - r1s + (double)nint * dt0) / dt1);
        if (n1 > 0) {
            m1 += sg1 * (double)n1;
            tn1 = (m1 - q1) * inv1;
        }
        // back to the exact parameters at the start of the next slab
        tx0 = (m0 + sg0 * (double)(nint - 1) - q0) * inv0;
        m0 += sg0 * (double)nint;
        left = 2;
    }
    for (; left > 0; --left) exact_slab(left == 1);
}

}  // namespace xrt
