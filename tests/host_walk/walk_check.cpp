// Host build of the GPU path's ray construction and slab walk (xrt_walk.h), run on the
// CPU over whole scans.  For every ray it records the hit list and checks that every
// image index the forward kernel would dereference lies inside the image, and (3D) that
// the walk's nested form gives the same hit list bit for bit.
//
// usage: walk_check <scan.txt> <hits.bin>
// scan.txt: "kind nx ny nz dx dy dz cx cy cz" / "n_views n_rows n_cols du dv u0 v0 sod sdd
//            has_z has_phi2 n_rays eps" / then the view angles, view_z, phi2 and ray
//            parameters as whitespace-separated numbers.
// hits.bin: per ray int32 count, then count x (int32 index, float64 length).
// With a third argument "simplex" the hit lists are those of the simplex basis
// (xrt_simplex.h: each hit unit's piece cut into its simplex pieces, index I * S + s),
// and every simplex index is checked to lie inside the simplex image.
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2006_00686_amd/csrc/xrt_simplex.h"

using namespace xrt;

namespace {

struct CheckVisit {
    static constexpr int32_t kIndexScale = 1;
    int64_t n_units;
    double thr, scale;
    std::vector<int32_t> idx;
    std::vector<double> len;
    long bad = 0;
    void check(int32_t I) { if (I < 0 || I >= n_units) ++bad; }
    void one(int32_t I, double l)
    {
        if (l > 0.0) check(I);
        if (l > thr) { idx.push_back(I); len.push_back(l * scale); }
    }
    // contract of walk(): I1 always valid with l1 >= 0; every length finite
    void first(int32_t I1, double l1)
    {
        check(I1);
        if (!(l1 >= 0.0)) ++bad;
    }
    void two(int32_t I1, double l1, int32_t I2, double l2)
    {
        first(I1, l1);
        if (!std::isfinite(l2)) ++bad;
        one(I1, l1);
        one(I2, l2);
    }
    void three(int32_t I1, double l1, int32_t I2, double l2, int32_t I3, double l3)
    {
        first(I1, l1);
        if (!std::isfinite(l2) || !std::isfinite(l3)) ++bad;
        one(I1, l1);
        one(I2, l2);
        one(I3, l3);
    }
};

template <int DIM>
struct SimplexCheck : SimplexWalker<DIM, SimplexCheck<DIM>> {
    int64_t n_simplices;
    double scale;
    std::vector<int32_t> idx;
    std::vector<double> len;
    long bad = 0;
    void simplex(int64_t T, double l)
    {
        if (T < 0 || T >= n_simplices || !(l > 0.0)) ++bad;
        idx.push_back((int32_t)T);
        len.push_back(l * scale);
    }
};

template <int DIM, int MODE>
long run_simplex(const DevPlan& P, FILE* out)
{
    long bad = 0;
    for (int32_t r = 0; r < (int32_t)P.n_rays; ++r) {
        Ray R;
        make_ray<DIM, MODE>(P, r, R);
        SimplexCheck<DIM> v;
        simplex_walker_init(v, P, R);
        v.n_simplices = P.n_units * kSimplices<DIM>;
        v.scale = R.scale;
        walk<DIM>(P, R, v);
        bad += v.bad;
        int32_t n = (int32_t)v.idx.size();
        fwrite(&n, 4, 1, out);
        for (int32_t k = 0; k < n; ++k) {
            fwrite(&v.idx[k], 4, 1, out);
            fwrite(&v.len[k], 8, 1, out);
        }
    }
    return bad;
}

template <int DIM, int MODE>
long run(const DevPlan& P, double eps, FILE* out, bool simplex)
{
    if (simplex) return run_simplex<DIM, MODE>(P, out);
    long bad = 0;
    for (int32_t r = 0; r < (int32_t)P.n_rays; ++r) {
        Ray R;
        make_ray<DIM, MODE>(P, r, R);
        CheckVisit v{P.n_units, eps / R.scale, R.scale, {}, {}, 0};
        walk<DIM>(P, R, v);
        bad += v.bad;
        if constexpr (DIM == 3) {
            // the nested form of the walk visits the same hits with the same lengths
            CheckVisit vn{P.n_units, eps / R.scale, R.scale, {}, {}, 0};
            walk<DIM, true>(P, R, vn);
            bad += vn.bad;
            if (vn.idx != v.idx || vn.len != v.len) ++bad;
        }
        int32_t n = (int32_t)v.idx.size();
        fwrite(&n, 4, 1, out);
        for (int32_t k = 0; k < n; ++k) {
            fwrite(&v.idx[k], 4, 1, out);
            fwrite(&v.len[k], 8, 1, out);
        }
    }
    return bad;
}

template <int DIM>
long run_dim(const DevPlan& P, double eps, FILE* out, bool simplex)
{
    switch (P.mode) {
        case MODE_PARALLEL: return run<DIM, MODE_PARALLEL>(P, eps, out, simplex);
        case MODE_DIVERGENT: return run<DIM, MODE_DIVERGENT>(P, eps, out, simplex);
        case MODE_ARC: return run<DIM, MODE_ARC>(P, eps, out, simplex);
        default: return run<DIM, MODE_LIST>(P, eps, out, simplex);
    }
}

std::vector<double> read_n(FILE* f, long n)
{
    std::vector<double> v((size_t)n);
    for (long i = 0; i < n; ++i)
        if (fscanf(f, "%lf", &v[(size_t)i]) != 1) { fprintf(stderr, "short input\n"); exit(2); }
    return v;
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 3 && !(argc == 4 && std::string(argv[3]) == "simplex")) {
        fprintf(stderr, "usage: walk_check scan.txt hits.bin [simplex]\n");
        return 2;
    }
    const bool simplex = argc == 4;
    FILE* f = fopen(argv[1], "r");
    if (!f) return 2;
    xrt_grid g{};
    xrt_scan s{};
    int has_z = 0, has_phi2 = 0;
    long long n_rays = 0;
    double eps = 0;
    if (fscanf(f, "%d %d %d %d %lf %lf %lf %lf %lf %lf", &s.kind, &g.nx, &g.ny, &g.nz, &g.dx, &g.dy, &g.dz,
               &g.cx, &g.cy, &g.cz) != 10)
        return 2;
    if (fscanf(f, "%d %d %d %lf %lf %lf %lf %lf %lf %d %d %lld %lf", &s.n_views, &s.n_rows, &s.n_cols, &s.du,
               &s.dv, &s.u0, &s.v0, &s.sod, &s.sdd, &has_z, &has_phi2, &n_rays, &eps) != 13)
        return 2;
    std::vector<double> ang = read_n(f, s.n_views), vz, p2, rays;
    if (has_z) vz = read_n(f, s.n_views);
    if (has_phi2) p2 = read_n(f, s.n_views);
    const int w = s.kind == XRT_RAYLIST2D ? 2 : 4;
    if (n_rays > 0) rays = read_n(f, n_rays * w);
    fclose(f);
    s.view_angle = ang.data();
    s.view_z = has_z ? vz.data() : nullptr;
    s.view_phi2 = has_phi2 ? p2.data() : nullptr;
    s.ray_params = rays.empty() ? nullptr : rays.data();
    s.n_rays = n_rays;
    HostTables T;
    xrt_status st = build_tables(&g, &s, T);
    if (st != XRT_OK) { fprintf(stderr, "build_tables: %d %s\n", st, xrt_last_error()); return 4; }
    T.dp.views = T.views.data();
    T.dp.col_cs = T.col.data();
    T.dp.row_cs = T.row.data();
    T.dp.rays = T.rays.data();
    FILE* out = fopen(argv[2], "wb");
    if (!out) return 2;
    long bad = T.dp.dim == 2 ? run_dim<2>(T.dp, eps, out, simplex) : run_dim<3>(T.dp, eps, out, simplex);
    fclose(out);
    if (bad) { fprintf(stderr, "%ld out-of-range image indices or contract violations\n", bad); return 3; }
    return 0;
}
