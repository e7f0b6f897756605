// The transform on a simplex basis (the paper's polygonal / polyhedral extension,
// Introduction "Contributions" and Sec. 4.2), shared by the gfx950 kernels and the host
// build used to check them on the CPU.
//
// The image lives on the simplices of a structured triangulation: in index coordinates
// (unit (k,j,i) = [i,i+1) x [j,j+1) x [k,k+1)) every pixel is cut into 2 triangles by
// the plane x - y = const, every voxel into 6 tetrahedra by the planes x - y, y - z and
// x - z = const (Kuhn's triangulation).  Simplex s of a unit holds the points whose local
// coordinates, sorted largest first, come in the s-th axis order: 2D (x,y) = 0,
// (y,x) = 1; 3D (x,y,z) = 0, (x,z,y) = 1, (y,x,z) = 2, (y,z,x) = 3, (z,x,y) = 4,
// (z,y,x) = 5.  Equal coordinates (within kSimplexTie) rank the later axis first, so a
// point on a diagonal face belongs to the simplex with the bigger index (Sec. 4.1's
// resolution carried to the new faces).  Simplex index = I * S + s with S = 2 (2D) or 6 (3D): the values of a
// unit's simplices are contiguous.
//
// A simplex is hit iff the ray's interval inside it is non-empty (C_low < C_up of the
// simplex's facets, the paper's condition with the diagonal facets added), and its
// length is C_up - C_low.  The candidates are the simplices of the units the slab walk
// visits: the walk gives each hit unit's piece of the ray [t, t + l]; inside it the ray
// crosses each diagonal face at most once, so the piece splits into at most 2 (2D) or 4
// (3D) consecutive simplex pieces, whose owners follow from the order of the local
// coordinates at each sub-piece's midpoint.
#pragma once

#include "xrt_walk.h"

namespace xrt {

template <int DIM>
constexpr int32_t kSimplices = DIM == 3 ? 6 : 2;

// Local coordinates closer than this (index units) are equal: a ray placed in a diagonal
// face in exact arithmetic carries coordinates that differ by rounding only (far below
// this for rays from sources up to ~1e5 units away).  The faces' counterpart of snapping
// tiny direction components to zero.
constexpr double kSimplexTie = 1e-9;

// Simplex of a unit holding the point with local coordinates l (the ordering above).
template <int DIM>
XRT_HD int32_t simplex_rank(const double* l)
{
    if constexpr (DIM == 2) {
        return l[0] > l[1] + kSimplexTie ? 0 : 1;
    } else {
        // "a before b": larger coordinate, ties to the later axis
        const bool xy = l[0] > l[1] + kSimplexTie, yz = l[1] > l[2] + kSimplexTie, xz = l[0] > l[2] + kSimplexTie;
        if (xy && xz) return yz ? 0 : 1;
        if (!xy && yz) return xz ? 2 : 3;
        return xy ? 4 : 5;
    }
}

// The simplex pieces of the piece [t, t + len] (ray parameter) of ray q + t w (index
// space) inside unit (i, j, k): emit(s, piece_len) in order along the ray.
template <int DIM, class F>
XRT_HD void simplex_pieces(const double* q, const double* w, double t, double len, int32_t i, int32_t j,
                           int32_t k, F&& emit)
{
    const double base[3] = {(double)i, (double)j, (double)k};
    double a[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) a[d] = fma(t, w[d], q[d]) - base[d];
    // parameters (from t) at which the ray crosses a diagonal face inside the piece
    double c0 = kInf, c1 = kInf, c2 = kInf;
    auto cross = [&](int u, int v, double& c) {
        const double dw = w[u] - w[v];
        if (dw != 0.0) {
            const double tau = (a[v] - a[u]) / dw;
            if (tau > 0.0 && tau < len) c = tau;
        }
    };
    cross(0, 1, c0);
    if constexpr (DIM == 3) {
        cross(1, 2, c1);
        cross(0, 2, c2);
        // sort the three crossings
        double lo = fmin(c0, c1), hi = fmax(c0, c1);
        const double mid = fmin(hi, c2);
        c2 = fmax(hi, c2);
        c0 = fmin(lo, mid);
        c1 = fmax(lo, mid);
    }
    double prev = 0.0;
#pragma unroll
    for (int m = 0; m < (DIM == 3 ? 4 : 2); ++m) {
        const double next = fmin(m == 0 ? c0 : m == 1 ? (DIM == 3 ? c1 : kInf) : m == 2 ? c2 : kInf, len);
        if (next > prev) {
            const double h = 0.5 * (prev + next);
            double l[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int d = 0; d < DIM; ++d) l[d] = fma(h, w[d], a[d]);
            emit(simplex_rank<DIM>(l), next - prev);
        }
        prev = fmax(prev, next);
    }
}

// Visitor base: follows the walk's pieces along the ray (walk() calls start(tin) and then
// hands over the units in order, every positive length directly after the previous one)
// and hands each simplex piece to Derived::simplex(index, length).
template <int DIM, class Derived>
struct SimplexWalker {
    static constexpr int32_t kIndexScale = 1;
    double q[3], w[3];
    int32_t nx, nxy;
    double t = 0.0;
    XRT_HD void start(double tin) { t = tin; }
    XRT_HD void piece(int32_t I, double l)
    {
        if (!(l > 0.0)) return;
        const int32_t k = DIM == 3 ? I / nxy : 0;
        const int32_t r = I - k * nxy;
        const int32_t j = r / nx, i = r - j * nx;
        const int64_t base = (int64_t)I * kSimplices<DIM>;
        simplex_pieces<DIM>(q, w, t, l, i, j, k, [&](int32_t s, double ls) {
            static_cast<Derived*>(this)->simplex(base + s, ls);
        });
        t += l;
    }
    XRT_HD void two(int32_t I1, double l1, int32_t I2, double l2)
    {
        piece(I1, l1);
        piece(I2, l2);
    }
    XRT_HD void three(int32_t I1, double l1, int32_t I2, double l2, int32_t I3, double l3)
    {
        piece(I1, l1);
        piece(I2, l2);
        piece(I3, l3);
    }
};

template <int DIM, class Derived>
XRT_HD void simplex_walker_init(SimplexWalker<DIM, Derived>& v, const DevPlan& P, const Ray& R)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v.q[d] = R.q[d];
        v.w[d] = R.w[d];
    }
    v.nx = P.nx;
    v.nxy = P.nx * P.ny;
}

}  // namespace xrt
