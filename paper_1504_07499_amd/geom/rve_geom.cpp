// Seeded input generator: RSA sphere placement and voxelization into three
// phases (arXiv:1504.07499, Sec. 2), and the same for aligned coated fibres
// (the cylindrical inclusions Sec. 6 names as an extension).  Host-only C++;
// no homogenization arithmetic lives here.  Conventions are documented in
// include/rvegeom.h.
#include "../../include/rvegeom.h"

#include <cmath>
#include <cstdint>
#include <random>
#include <vector>

namespace {

struct Uniform {
    std::mt19937_64 eng;
    explicit Uniform(uint64_t seed) : eng(seed) {}
    // 53 random bits -> [0, 1); the mapping is fixed here rather than left to
    // std::uniform_real_distribution, whose algorithm is implementation-defined.
    double next() { return (double)(eng() >> 11) * (1.0 / 9007199254740992.0); }
};

inline double wrap01(double v) {
    v -= std::floor(v);
    return v >= 1.0 ? 0.0 : v;
}

// Squared periodic minimum-image distance of D-dimensional points.
template <int D> inline double min_image_d2n(const double *a, const double *b) {
    double s = 0.0;
    for (int d = 0; d < D; ++d) {
        double t = a[d] - b[d];
        t -= std::nearbyint(t);
        s += t * t;
    }
    return s;
}

template <int D>
bool fits_n(const std::vector<double> &c, int count, const double *p, double min_d2, int skip) {
    for (int i = 0; i < count; ++i) {
        if (i == skip) continue;
        if (min_image_d2n<D>(&c[D * i], p) < min_d2) return false;
    }
    return true;
}

// RSA of n identical D-balls of radius r in the periodic unit cell, then, if
// the attempt budget runs out, hard-ball Monte Carlo shaking interleaved with
// further insertions.  centers: D * n doubles.  Returns 0, or -2 when jammed.
template <int D> int place_balls(int n, double r, uint64_t seed, double *centers, int *method) {
    const double min_d2 = 4.0 * r * r;
    Uniform u(seed);
    std::vector<double> c((size_t)D * n);
    int placed = 0;
    const long rsa_budget = 1000000;
    for (long a = 0; a < rsa_budget && placed < n; ++a) {
        double p[D];
        for (int d = 0; d < D; ++d) p[d] = u.next();
        if (fits_n<D>(c, placed, p, min_d2, -1)) {
            for (int d = 0; d < D; ++d) c[(size_t)D * placed + d] = p[d];
            ++placed;
        }
    }
    int how = 0;
    if (placed < n) {
        how = 1;
        const double step = 0.5 * r;
        const int sweeps = 20000, inserts_per_sweep = 200;
        for (int s = 0; s < sweeps && placed < n; ++s) {
            for (int i = 0; i < placed; ++i) {
                double p[D];
                for (int d = 0; d < D; ++d) p[d] = wrap01(c[(size_t)D * i + d] + step * (2.0 * u.next() - 1.0));
                if (fits_n<D>(c, placed, p, min_d2, i))
                    for (int d = 0; d < D; ++d) c[(size_t)D * i + d] = p[d];
            }
            for (int a = 0; a < inserts_per_sweep && placed < n; ++a) {
                double p[D];
                for (int d = 0; d < D; ++d) p[d] = u.next();
                if (fits_n<D>(c, placed, p, min_d2, -1)) {
                    for (int d = 0; d < D; ++d) c[(size_t)D * placed + d] = p[d];
                    ++placed;
                }
            }
        }
    }
    if (placed < n) return -2;
    for (size_t i = 0; i < c.size(); ++i) centers[i] = c[i];
    if (method) *method = how;
    return 0;
}

}  // namespace

extern "C" double rvegeom_radius(int n_spheres, double f) {
    if (n_spheres < 1 || !(f > 0.0)) return 0.0;
    return std::cbrt(3.0 * f / (4.0 * M_PI * (double)n_spheres));
}

extern "C" int rvegeom_place(int n_spheres, double f, uint64_t seed, double *centers, int *method) {
    if (n_spheres < 1 || !(f > 0.0 && f < 1.0) || !centers) return -1;
    const double r = rvegeom_radius(n_spheres, f);
    if (!(r < 0.5)) return -1;
    return place_balls<3>(n_spheres, r, seed, centers, method);
}

extern "C" int rvegeom_voxelize(int n, int n_spheres, const double *centers, double radius,
                                double layer, uint8_t *phases) {
    if (n < 1 || n_spheres < 0 || !phases || (n_spheres > 0 && !centers)) return -1;
    if (!(radius >= 0.0 && radius < 0.5) || !(layer >= 0.0 && layer < 1.0)) return -1;
    const size_t M = (size_t)n * n * n;
    for (size_t v = 0; v < M; ++v) phases[v] = 0;
    const double r2 = radius * radius;
    const double ri = (1.0 - layer) * radius;
    const double ri2 = ri * ri;
    for (int s = 0; s < n_spheres; ++s) {
        const double *cc = centers + 3 * s;
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = (int)std::floor((cc[d] - radius) * n - 0.5) - 1;
            hi[d] = (int)std::ceil((cc[d] + radius) * n - 0.5) + 1;
        }
        for (int kz = lo[2]; kz <= hi[2]; ++kz) {
            double dz = ((double)kz + 0.5) / n - cc[2];
            int iz = ((kz % n) + n) % n;
            for (int ky = lo[1]; ky <= hi[1]; ++ky) {
                double dy = ((double)ky + 0.5) / n - cc[1];
                int iy = ((ky % n) + n) % n;
                for (int kx = lo[0]; kx <= hi[0]; ++kx) {
                    double dx = ((double)kx + 0.5) / n - cc[0];
                    int ix = ((kx % n) + n) % n;
                    double d2 = dx * dx + dy * dy + dz * dz;
                    size_t v = ((size_t)iz * n + iy) * n + ix;
                    if (d2 < ri2) phases[v] = 1;
                    else if (d2 < r2 && phases[v] != 1) phases[v] = 2;
                }
            }
        }
    }
    return 0;
}

extern "C" int rvegeom_generate(int n, int n_spheres, double f, double layer, uint64_t seed,
                                uint8_t *phases, double *centers, int *method) {
    if (n < 1 || n_spheres < 1 || !phases) return -1;
    if (!(layer > 0.0 && layer < 1.0)) return -1;
    std::vector<double> c(3 * (size_t)n_spheres);
    int rc = rvegeom_place(n_spheres, f, seed, c.data(), method);
    if (rc != 0) return rc;
    rc = rvegeom_voxelize(n, n_spheres, c.data(), rvegeom_radius(n_spheres, f), layer, phases);
    if (rc != 0) return rc;
    if (centers)
        for (size_t i = 0; i < c.size(); ++i) centers[i] = c[i];
    return 0;
}

// ------------------------------------------------------------- aligned fibres

extern "C" double rvegeom_fiber_radius(int n_fibers, double f) {
    if (n_fibers < 1 || !(f > 0.0)) return 0.0;
    return std::sqrt(f / (M_PI * (double)n_fibers));
}

extern "C" int rvegeom_place_fibers(int n_fibers, double f, uint64_t seed, double *centers, int *method) {
    if (n_fibers < 1 || !(f > 0.0 && f < 1.0) || !centers) return -1;
    const double r = rvegeom_fiber_radius(n_fibers, f);
    if (!(r < 0.5)) return -1;
    return place_balls<2>(n_fibers, r, seed, centers, method);
}

extern "C" int rvegeom_voxelize_fibers(int n, int n_fibers, const double *centers, double radius, double layer,
                                       uint8_t *phases) {
    if (n < 1 || n_fibers < 0 || !phases || (n_fibers > 0 && !centers)) return -1;
    if (!(radius >= 0.0 && radius < 0.5) || !(layer >= 0.0 && layer < 1.0)) return -1;
    const size_t NN = (size_t)n * n;
    std::vector<uint8_t> plane(NN, 0);
    const double r2 = radius * radius;
    const double ri = (1.0 - layer) * radius;
    const double ri2 = ri * ri;
    for (int s = 0; s < n_fibers; ++s) {
        const double *cc = centers + 2 * s;
        int lo[2], hi[2];
        for (int d = 0; d < 2; ++d) {
            lo[d] = (int)std::floor((cc[d] - radius) * n - 0.5) - 1;
            hi[d] = (int)std::ceil((cc[d] + radius) * n - 0.5) + 1;
        }
        for (int ky = lo[1]; ky <= hi[1]; ++ky) {
            double dy = ((double)ky + 0.5) / n - cc[1];
            int iy = ((ky % n) + n) % n;
            for (int kx = lo[0]; kx <= hi[0]; ++kx) {
                double dx = ((double)kx + 0.5) / n - cc[0];
                int ix = ((kx % n) + n) % n;
                double d2 = dx * dx + dy * dy;
                size_t v = (size_t)iy * n + ix;
                if (d2 < ri2) plane[v] = 1;
                else if (d2 < r2 && plane[v] != 1) plane[v] = 2;
            }
        }
    }
    for (int z = 0; z < n; ++z)
        for (size_t v = 0; v < NN; ++v) phases[(size_t)z * NN + v] = plane[v];
    return 0;
}

extern "C" int rvegeom_generate_fibers(int n, int n_fibers, double f, double layer, uint64_t seed,
                                       uint8_t *phases, double *centers, int *method) {
    if (n < 1 || n_fibers < 1 || !phases) return -1;
    if (!(layer > 0.0 && layer < 1.0)) return -1;
    std::vector<double> c(2 * (size_t)n_fibers);
    int rc = rvegeom_place_fibers(n_fibers, f, seed, c.data(), method);
    if (rc != 0) return rc;
    rc = rvegeom_voxelize_fibers(n, n_fibers, c.data(), rvegeom_fiber_radius(n_fibers, f), layer, phases);
    if (rc != 0) return rc;
    if (centers)
        for (size_t i = 0; i < c.size(); ++i) centers[i] = c[i];
    return 0;
}

// ------------------------------------------------------ spheres and fibres

extern "C" int rvegeom_place_mixed(int n_spheres, double f_spheres, int n_fibers, double f_fibers, uint64_t seed,
                                   double *sphere_centers, double *fiber_centers, int *method) {
    if (n_spheres < 1 || n_fibers < 1 || !(f_spheres > 0.0) || !(f_fibers > 0.0) ||
        !(f_spheres + f_fibers < 1.0) || !sphere_centers || !fiber_centers)
        return -1;
    const double rs = rvegeom_radius(n_spheres, f_spheres), rf = rvegeom_fiber_radius(n_fibers, f_fibers);
    if (!(rs < 0.5) || !(rf < 0.5)) return -1;
    // fibres first (RSA of their axes, own seed stream), then spheres by RSA
    // against the fibres (axis distance in the cross-section >= rs + rf) and
    // each other; no shaking for the spheres
    int rc = place_balls<2>(n_fibers, rf, seed, fiber_centers, method);
    if (rc != 0) return rc;
    Uniform u(seed ^ 0x9e3779b97f4a7c15ull);
    std::vector<double> c(3 * (size_t)n_spheres);
    const double ss2 = 4.0 * rs * rs, sf2 = (rs + rf) * (rs + rf);
    int placed = 0;
    const long budget = 1000000;
    for (long a = 0; a < budget && placed < n_spheres; ++a) {
        double p[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < 3; ++d) p[d] = u.next();
        bool ok = fits_n<3>(c, placed, p, ss2, -1);
        for (int i = 0; ok && i < n_fibers; ++i)
            if (min_image_d2n<2>(fiber_centers + 2 * i, p) < sf2) ok = false;
        if (ok) {
            for (int d = 0; d < 3; ++d) c[3 * (size_t)placed + d] = p[d];
            ++placed;
        }
    }
    if (placed < n_spheres) return -2;
    for (size_t i = 0; i < c.size(); ++i) sphere_centers[i] = c[i];
    return 0;
}

extern "C" int rvegeom_generate_mixed(int n, int n_spheres, double f_spheres, int n_fibers, double f_fibers,
                                      double layer, uint64_t seed, uint8_t *phases) {
    if (n < 1 || !phases || !(layer > 0.0 && layer < 1.0)) return -1;
    if (n_spheres < 1 || n_fibers < 1) return -1;
    std::vector<double> cs(3 * (size_t)n_spheres), cf(2 * (size_t)n_fibers);
    int rc = rvegeom_place_mixed(n_spheres, f_spheres, n_fibers, f_fibers, seed, cs.data(), cf.data(), nullptr);
    if (rc != 0) return rc;
    const size_t M = (size_t)n * n * n;
    std::vector<uint8_t> sph(M);
    rc = rvegeom_voxelize_fibers(n, n_fibers, cf.data(), rvegeom_fiber_radius(n_fibers, f_fibers), layer, phases);
    if (rc != 0) return rc;
    rc = rvegeom_voxelize(n, n_spheres, cs.data(), rvegeom_radius(n_spheres, f_spheres), layer, sph.data());
    if (rc != 0) return rc;
    // inclusions do not overlap, so a voxel is claimed by at most one shape up
    // to voxel-centre rounding; an inclusion (core) id wins over a coating id
    for (size_t v = 0; v < M; ++v)
        if (sph[v] == 1 || (sph[v] == 2 && phases[v] == 0)) phases[v] = sph[v];
    return 0;
}
