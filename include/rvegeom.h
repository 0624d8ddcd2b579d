/*
 * rvegeom.h -- seeded input generator: random sequential adsorption (RSA) of
 * identical non-overlapping spheres (or aligned fibres) in the periodic unit
 * cell, and voxel-centre classification into the three phases (matrix,
 * inclusion, coating).
 *
 * This is setup, not the homogenization method: it holds none of the scheme's
 * arithmetic.  It serves both the GPU library (rve_create) and the tests that
 * feed the same phase image to the FP64 oracle.
 *
 * Paper: arXiv:1504.07499, Sec. 2 (RSA generation of up to 100 identical
 * spheres, up to 40 % volume fraction, sphere list as centre + radius;
 * voxelization with a coating of relative width l = coating width / sphere
 * radius, 0 < l < 1; the sphere volume fraction includes the coating).
 *
 * Conventions (the paper is silent on them):
 *  - unit cell [0,1)^3, periodic; sphere radius r = (3 f / (4 pi n))^(1/3)
 *    includes the coating; inclusion radius (1 - l) r;
 *  - centres are uniform in [0,1)^3 from std::mt19937_64(seed), each
 *    coordinate (u >> 11) * 2^-53;
 *  - two spheres overlap when their periodic minimum-image distance is
 *    below 2 r;
 *  - pure RSA is tried first; if the attempt budget runs out (RSA saturates
 *    near 38 % for equal spheres), placed spheres are shaken by hard-sphere
 *    Monte Carlo moves interleaved with further insertion attempts;
 *  - voxel (i, j, k) is classified by its centre ((i+.5)/N, (j+.5)/N,
 *    (k+.5)/N): d^2 < ((1-l) r)^2 -> inclusion (1), else d^2 < r^2 ->
 *    coating (2), else matrix (0); all in FP64, strict "<".
 *
 * Phase images are [z][y][x] with x fastest (index (k*N + j)*N + i for the
 * voxel at x = i, y = j, z = k).  All buffers are host memory owned by the
 * caller.  Functions return 0 on success, -1 on bad arguments, -2 when the
 * spheres could not be placed within the attempt budget.
 */
#ifndef RVEGEOM_H
#define RVEGEOM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Radius (unit-cell units, coating included) of n identical spheres that
 * fill volume fraction f: r = (3 f / (4 pi n))^(1/3).  Sec. 2, Sec. 5. */
double rvegeom_radius(int n_spheres, double volume_fraction);

/* RSA placement (Sec. 2).  centers: out, 3*n_spheres doubles (x,y,z).
 * method: out (may be NULL), 0 = pure RSA, 1 = RSA + Monte Carlo shaking.
 * n_spheres >= 1, 0 < f < 1, radius < 0.5. */
int rvegeom_place(int n_spheres, double volume_fraction, uint64_t seed,
                  double *centers, int *method);

/* Voxel-centre classification (Sec. 2) of spheres of one radius r with
 * coating layer l (0 <= l < 1) on an N^3 grid.  phases: out, N^3 bytes. */
int rvegeom_voxelize(int n, int n_spheres, const double *centers, double radius,
                     double layer, uint8_t *phases);

/* Both steps: placement, then voxelization.  centers may be NULL. */
int rvegeom_generate(int n, int n_spheres, double volume_fraction, double layer,
                     uint64_t seed, uint8_t *phases, double *centers, int *method);

/* Aligned coated fibres: the cylindrical inclusions Sec. 6 names as the next
 * geometry, as infinite circular cylinders along z (the image is invariant
 * along z).  Same conventions as the spheres in the xy cross-section: radius
 * r = (f / (pi n))^(1/2) (coating included; f is the area fraction of the
 * cross-section, hence the volume fraction), RSA of the axes in the periodic
 * unit square from std::mt19937_64(seed) (x then y per attempt), minimum
 * axis distance 2 r, Monte Carlo shaking if the budget runs out, voxel
 * classification by the centre ((i+.5)/N, (j+.5)/N) of each column.
 * centers: 2 doubles (x, y) per fibre. */
double rvegeom_fiber_radius(int n_fibers, double volume_fraction);
int rvegeom_place_fibers(int n_fibers, double volume_fraction, uint64_t seed,
                         double *centers, int *method);
int rvegeom_voxelize_fibers(int n, int n_fibers, const double *centers, double radius,
                            double layer, uint8_t *phases);
int rvegeom_generate_fibers(int n, int n_fibers, double volume_fraction, double layer,
                            uint64_t seed, uint8_t *phases, double *centers, int *method);

/* Mixed inclusions: coated fibres along z and coated spheres in one cell,
 * both with coating layer l.  Fibres are placed first (as above, seed), then
 * spheres by RSA (1e6 attempts, no shaking, a second stream derived from the
 * seed) against each other and against the fibres: a sphere's centre lies at
 * least rs + rf from every fibre axis in the cross-section.  The fractions
 * are those of each shape (coating included); f_spheres + f_fibers < 1.
 * sphere_centers: 3 n_spheres doubles, fiber_centers: 2 n_fibers. */
int rvegeom_place_mixed(int n_spheres, double f_spheres, int n_fibers, double f_fibers,
                        uint64_t seed, double *sphere_centers, double *fiber_centers,
                        int *method);
int rvegeom_generate_mixed(int n, int n_spheres, double f_spheres, int n_fibers,
                           double f_fibers, double layer, uint64_t seed, uint8_t *phases);

#ifdef __cplusplus
}
#endif

#endif /* RVEGEOM_H */
