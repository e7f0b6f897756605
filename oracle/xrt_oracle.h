/*
 * Plain FP64 CPU reference ("oracle") of the discrete X-ray transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no code with the HIP path.
 *
 * What it computes is the plain definition of the paper's discrete transform
 * (Introduction, eq. Xray_transform_image; Sec. 2.2.1 eq. intersection_length;
 * Sec. 3.2.1 eq. intersection_length_3D):
 *
 *   a ray is the infinite line { p + t*th : t real }, |th| = 1, physical units;
 *   unit (k,j,i) occupies the box
 *       x in [cx + (i - nx/2)*dx, cx + (i - nx/2 + 1)*dx)
 *       y in (cy + (ny/2 - j - 1)*dy, cy + (ny/2 - j)*dy]
 *       z in (cz + (nz/2 - k - 1)*dz, cz + (nz/2 - k)*dz]
 *   (pixel/voxel supports of Sec. 2.1 and 3.2.1; the half-open sides realise the
 *   "take the bigger 1D index" resolution of grid-aligned rays, Sec. 4.1);
 *   len(ray, unit) = measure of { t : p + t*th in unit }  (physical length);
 *   forward  g_r = sum_I f_I len(r, I);  adjoint f_I = sum_r g_r len(r, I).
 *   The 1D index is I = (k*ny + j)*nx + i (the paper's I = k*Ny*Nx + j*Ny + i
 *   written for non-square grids).
 *
 * Method (chord partition): clip the line to the image box, collect every grid-plane
 * crossing strictly inside the chord, sort them, and give each piece between two
 * consecutive crossings to the unit that contains its midpoint.  No piece of the
 * GPU path's slab/range logic is used.
 *
 * nz == 0 selects a 2D image (components 0,1 of p and th are used).
 */
#ifndef XRT_ORACLE_H
#define XRT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny, nz;        /* nz == 0: 2D */
    double dx, dy, dz;     /* unit side lengths */
    double cx, cy, cz;     /* centre of the image box */
} ora_grid;

/* Forward: out[r] = sum_I img[I] len(r, I).  p, th: 3 doubles per ray. */
void ora_forward(const ora_grid* g, long nrays, const double* p, const double* th,
                 const double* img, double* out, int nthreads);

/* Adjoint: img[I] = sum_r sino[r] len(r, I) (overwrites img).  Deterministic:
 * per-thread FP64 partial images reduced in fixed thread order. */
void ora_adjoint(const ora_grid* g, long nrays, const double* p, const double* th,
                 const double* sino, double* img, int nthreads);

/* Hit list of one ray: units with len > eps, sorted by 1D index.
 * Returns the number of hits (writes at most cap entries). */
long ora_ray_hits(const ora_grid* g, const double* p, const double* th,
                  long* idx, double* len, long cap, double eps);

/* Number of hits (len > eps) of each ray. */
void ora_hit_counts(const ora_grid* g, long nrays, const double* p, const double* th,
                    double eps, long* counts, int nthreads);

/* Chord length of the line through the (half-open) image box. */
double ora_chord(const ora_grid* g, const double* p, const double* th);

/* Attenuated transform (Introduction, eq. generalizedRadontransform, SPECT case): the
 * weight of a point is exp(-integral of mu from it to the detector side, +th); mu is a
 * unit-wise constant attenuation map (1/length) on the same grid.
 *   out[r] = sum over the chord's pieces i of img_i exp(-A_i) (1 - exp(-mu_i len_i)) / mu_i,
 *   A_i = sum of mu_j len_j over the pieces after i (toward +th).
 * ora_adjoint_att is its transpose (fixed-order reduction). */
void ora_forward_att(const ora_grid* g, long nrays, const double* p, const double* th,
                     const double* img, const double* mu, double* out, int nthreads);
void ora_adjoint_att(const ora_grid* g, long nrays, const double* p, const double* th,
                     const double* sino, const double* mu, double* img, int nthreads);

/* Simplex basis (the paper's polygonal / polyhedral extension; Introduction
 * "Contributions", Sec. 4.2): every pixel cut into 2 triangles, every voxel into 6
 * tetrahedra (Kuhn's triangulation in index coordinates; the definition is stated in
 * xrt_oracle.c).  Images hold S = 2 (2D) or 6 (3D) values per unit, simplex index
 * I * S + s.  Forward, adjoint and hit lists as above, over simplices. */
void ora_forward_simplex(const ora_grid* g, long nrays, const double* p, const double* th,
                         const double* img, double* out, int nthreads);
void ora_adjoint_simplex(const ora_grid* g, long nrays, const double* p, const double* th,
                         const double* sino, double* img, int nthreads);
long ora_ray_hits_simplex(const ora_grid* g, const double* p, const double* th,
                          long* idx, double* len, long cap, double eps);

#ifdef __cplusplus
}
#endif
#endif
