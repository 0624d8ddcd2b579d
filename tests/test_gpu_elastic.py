"""GPU parity of the elastic case (linear elasticity with isotropic phases,
the extension Sec. 6 names) against the FP64 elastic oracle and closed forms.

The GPU works in the orthonormal basis B_0..B_5 of symmetric tensors with the
load cases E = B_j; the oracle takes any imposed strain in plain tensor
components, so it is called with E = B_j and its results are projected on
the basis here.  Bars as for conductivity: FP64 1e-9 (fields after fixed
iterations 1e-11), FP32 1e-4 (fields 3e-5).
"""
import numpy as np
import pytest

import oracle
import paper_1504_07499_amd as rh
from paper_1504_07499_amd import geom

pytestmark = pytest.mark.gpu

B = rh.ELASTIC_BASIS
# bulk, shear modulus: matrix (epoxy-like), inclusion (glass-like), coating (stiff)
MOD = np.array([[4.0, 1.5], [40.0, 30.0], [150.0, 100.0]])
COMPS = oracle.EL_COMPS
MULT = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])  # off-diagonal components appear twice


def basis_strains():
    """B_j as the oracle's tensor components (11, 22, 33, 23, 13, 12)."""
    return np.array([[B[j][a, b] for (a, b) in COMPS] for j in range(6)])


def to_basis(t):
    """Tensor components (..., 6) -> basis components (..., 6)."""
    P = np.array([[MULT[q] * B[k][COMPS[q]] for q in range(6)] for k in range(6)])
    return np.tensordot(t, P.T, axes=([-1], [0]))


def tensor_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("n", [8, 12, 16, 24])
def test_elastic_fixed_iterations_vs_oracle(n, precision):
    """Three iterations from E = B_j on an i.i.d. phase image: every voxel of
    every component, the stiffness and the residual histories."""
    print(f"\n[case] elastic field n={n} precision={precision}", flush=True)
    ph = geom.random_phases(n, seed=500 + n)
    ref = oracle.homogenize_elastic(ph, MOD, basis_strains(), tol=0.0, max_iter=3, want_field=True)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize_elastic(r, MOD, 0.0, max_iter=3, precision=precision, want_field=True, hist_cap=8)
    bar = 1e-11 if precision == 1 else 3e-5
    ref_field = to_basis(np.moveaxis(ref.field, 1, -1))  # (lc, z, y, x, k)
    assert tensor_err(np.moveaxis(g.field, 1, -1), ref_field) <= bar
    Cb = to_basis(ref.S).T  # column j: stress of load case j in the basis
    assert tensor_err(g.C_basis, Cb) <= bar
    assert list(g.iters) == [3] * 6
    for j in range(6):
        np.testing.assert_allclose(g.history[j], ref.history[j], rtol=bar * 10)


def test_elastic_converged_fp64_vs_oracle():
    """16^3 RSA coated spheres, tol 1e-8, FP64: C_hom (Voigt) within 1e-9 of
    the oracle's, built from the same six load cases."""
    print("\n[case] elastic converged fp64", flush=True)
    ph, _, _ = geom.generate(16, 4, 0.25, 0.2, 5)
    ref = oracle.homogenize_elastic(ph, MOD, basis_strains(), tol=1e-8)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize_elastic(r, MOD, 1e-8, precision=1)
    assert g.status == rh.RVE_OK
    assert list(g.iters) == list(ref.iters)
    assert tensor_err(g.C_basis, to_basis(ref.S).T) <= 1e-9
    assert np.abs(g.C - g.C.T).max() <= 1e-9 * np.abs(g.C).max()


@pytest.mark.parametrize("n,precision", [(64, 1), (64, 0), (96, 0)])
def test_elastic_equal_shear_hill(n, precision):
    """Phases of equal shear modulus on an RSA RVE (64^3; 96^3 in FP32, a
    radix-3 grid on the separate passes): the hydrostatic load case gives
    Hill's exact bulk modulus (closed form, any geometry)."""
    print(f"\n[case] elastic hill {n} precision={precision}", flush=True)
    mod = np.array([[4.0, 2.0], [40.0, 2.0], [150.0, 2.0]])
    ph, _, _ = geom.generate(n, 12, 0.3, 0.2, 6)
    kv = mod[ph, 0]
    khill = 1.0 / np.mean(1.0 / (kv + 4.0 * 2.0 / 3.0)) - 4.0 * 2.0 / 3.0
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize_elastic(r, mod, 1e-11 if precision else 1e-6, precision=precision)
    # load case B_0 = I / sqrt3: mean stress 3 kappa* B_0 -> C_basis[0, 0] = 3 kappa*
    # (exact at the fixed point; the stopping tolerance sets the bar)
    assert abs(g.C_basis[0, 0] / 3.0 - khill) <= (1e-9 if precision else 1e-5) * khill


@pytest.mark.parametrize("flags", [0, 2])
def test_elastic_equal_shear_hill_256_fp32(flags):
    """The same closed form on the 256^3 RVE of 100 RSA spheres at f = 0.40
    (FP32; split planes, by default with the fused pass writing the parity
    layout that the z pass combines, with flags 2 in separate passes;
    8-column z tiles in 1024-thread workgroups): the random geometry feeds
    every z tile and every plane of all six load cases, and the hydrostatic
    load case must give Hill's bulk modulus."""
    print(f"\n[case] elastic hill 256 fp32 flags={flags}", flush=True)
    mod = np.array([[4.0, 2.0], [40.0, 2.0], [150.0, 2.0]])
    ph, _, _ = geom.generate(256, 100, 0.40, 0.1, 3)
    kv = mod[ph, 0]
    khill = 1.0 / np.mean(1.0 / (kv + 4.0 * 2.0 / 3.0)) - 4.0 * 2.0 / 3.0
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize_elastic(r, mod, 1e-6, precision=0, path_flags=flags)
    C = np.asarray(g.C_basis)
    assert abs(C[0, 0] / 3.0 - khill) <= 1e-5 * khill
    # with one shear modulus a uniform deviatoric strain is the exact
    # solution (its stress 2 mu E is uniform, hence in equilibrium), so the
    # deviatoric block is 2 mu I and, by the major symmetry of the discrete
    # problem, the hydrostatic load case carries no deviatoric mean stress
    assert np.allclose(np.diag(C)[1:], 4.0, rtol=1e-6, atol=0)
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() <= 1e-5 * C[0, 0]


def test_elastic_five_pass_256_fp64_vs_oracle():
    """FP64 at 256^3 runs the five-pass form with six components per load
    case (the xy-plane does not fit in LDS): two iterations on an RSA RVE,
    load case B_3 (a shear) voxel by voxel and its stiffness column against
    the oracle."""
    print("\n[case] elastic five-pass 256 fp64", flush=True)
    ph, _, _ = geom.generate(256, 100, 0.3, 0.2, 3)
    j = 3
    ref = oracle.homogenize_elastic(ph, MOD, basis_strains()[[j]], tol=0.0, max_iter=2, want_field=True)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize_elastic(r, MOD, 0.0, max_iter=2, precision=1, want_field=True)
    ref_field = to_basis(np.moveaxis(ref.field[0], 0, -1))  # (z, y, x, k)
    assert tensor_err(np.moveaxis(g.field[j], 0, -1), ref_field) <= 1e-11
    assert tensor_err(np.asarray(g.C_basis)[:, j], to_basis(ref.S)[0]) <= 1e-11
    assert list(g.iters) == [2] * 6


@pytest.mark.parametrize("precision", [0, 1])
def test_elastic_equal_shear_hill_512(precision):
    """512^3 (five-pass form in both precisions) on an RSA RVE of equal shear
    moduli: Hill's bulk modulus, the exact deviatoric block 2 mu I and no
    coupling, as at 256^3."""
    print(f"\n[case] elastic hill 512 precision={precision}", flush=True)
    mod = np.array([[4.0, 2.0], [40.0, 2.0], [150.0, 2.0]])
    ph, _, _ = geom.generate(512, 100, 0.30, 0.2, 7)
    kv = mod[ph, 0]
    khill = 1.0 / np.mean(1.0 / (kv + 4.0 * 2.0 / 3.0)) - 4.0 * 2.0 / 3.0
    del kv
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize_elastic(r, mod, 1e-11 if precision else 1e-6, precision=precision)
    C = np.asarray(g.C_basis)
    bar = 1e-9 if precision else 1e-5
    assert abs(C[0, 0] / 3.0 - khill) <= bar * khill
    assert np.allclose(np.diag(C)[1:], 4.0, rtol=bar, atol=0)
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() <= bar * C[0, 0]


@pytest.mark.parametrize("n,precision,axis", [(48, 1, 0), (48, 0, 0), (256, 0, 0), (256, 0, 2)])
def test_elastic_laminate_backus(n, precision, axis):
    """Layers normal to x (or z) on an n^3 grid: the Backus stiffness (closed
    form); 256^3 runs the split-plane passes and the one-per-CU z tiles."""
    print(f"\n[case] elastic laminate n={n} precision={precision} axis={axis}", flush=True)
    w0, w1 = round(n * 17 / 48) | 1, round(n * 9 / 48) | 1
    prof = np.array([0] * w0 + [1] * w1 + [2] * (n - w0 - w1), np.uint8)
    shape = [1, 1, 1]
    shape[2 - axis] = n  # the phase image is [z][y][x]
    ph = np.broadcast_to(prof.reshape(shape), (n, n, n)).copy()
    kap, mu = MOD[prof, 0], MOD[prof, 1]
    lam = kap - 2 * mu / 3
    a = lam + 2 * mu
    h = np.mean
    b, c = [d for d in range(3) if d != axis]
    C = np.zeros((6, 6))
    C11 = 1.0 / h(1 / a)
    C12 = h(lam / a) * C11
    C[axis, axis] = C11
    C[axis, b] = C[b, axis] = C[axis, c] = C[c, axis] = C12
    C[b, b] = C[c, c] = h(a - lam ** 2 / a) + h(lam / a) ** 2 * C11
    C[b, c] = C[c, b] = h(lam - lam ** 2 / a) + h(lam / a) ** 2 * C11
    # Voigt shear index of the plane of two axes: 3 + the third axis
    C[3 + axis, 3 + axis] = h(mu)
    C[3 + b, 3 + b] = C[3 + c, 3 + c] = 1.0 / h(1 / mu)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize_elastic(r, MOD, 1e-10 if precision else 1e-6, precision=precision, max_iter=20000)
    assert tensor_err(g.C, C) <= (1e-9 if precision else 1e-4)


def test_elastic_128_fp32_against_fp64():
    """128^3 RSA coated spheres (50 spheres, f = 0.3, l = 0.2): FP32 stiffness
    within 1e-4 of FP64, both major-symmetric and near-isotropic."""
    print("\n[case] elastic 128", flush=True)
    with rh.rve_create(128, 50, 0.30, 0.2, 2) as r:
        g32 = rh.homogenize_elastic(r, MOD, 1e-6, precision=0)
        g64 = rh.homogenize_elastic(r, MOD, 1e-6, precision=1)
    assert g64.status == rh.RVE_OK and g32.status in (rh.RVE_OK, rh.RVE_STALLED)
    assert tensor_err(g32.C, g64.C) <= 1e-4
    for g in (g32, g64):
        assert np.abs(g.C - g.C.T).max() <= 1e-5 * np.abs(g.C).max()


def test_elastic_rejections():
    print("\n[case] elastic rejections", flush=True)
    with rh.rve_create_from_phases(geom.random_phases(16, 5)) as r:
        with pytest.raises(rh.RveError):
            rh.homogenize_elastic(r, [[1.0, 1.0], [2.0, -1.0], [3.0, 1.0]], 1e-6)
    for prec in (0, 1):
        sizes = rh.rve_supported_n_elastic(prec)
        assert 128 in sizes and 256 in sizes and 512 in sizes and 36 not in sizes
    # a grid the elastic case does not instantiate is refused before any GPU work
    with rh.rve_create_from_phases(geom.random_phases(36, 5)) as r:
        with pytest.raises(rh.RveError) as ei:
            rh.homogenize_elastic(r, MOD, 1e-6)
        assert ei.value.status == rh.RVE_ERR_ARG


def test_elastic_start_field_continues_the_iteration():
    """The accelerated iteration's state is the strain field alone: one
    iteration from the field of two equals three iterations from E (FP64)."""
    print("\n[case] elastic start field", flush=True)
    ph = geom.random_phases(16, 77)
    with rh.rve_create_from_phases(ph) as r:
        g2 = rh.homogenize_elastic(r, MOD, 0.0, max_iter=2, precision=1, want_field=True)
        g1 = rh.homogenize_elastic(r, MOD, 0.0, max_iter=1, precision=1, want_field=True, init_field=g2.field)
        g3 = rh.homogenize_elastic(r, MOD, 0.0, max_iter=3, precision=1, want_field=True)
    assert tensor_err(g1.field, g3.field) <= 1e-12
    assert tensor_err(g1.C_basis, g3.C_basis) <= 1e-12


def test_elastic_homogeneous_and_iteration_cap():
    """One phase everywhere: C_hom = C after one iteration; an unreachable
    tolerance with a cap reports NOT_CONVERGED after exactly the cap."""
    print("\n[case] elastic homogeneous and cap", flush=True)
    ph = np.full((16, 16, 16), 1, np.uint8)
    kap, mu = MOD[1]
    lam = kap - 2 * mu / 3
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] = lam + 2 * mu
    C[np.arange(3, 6), np.arange(3, 6)] = mu
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize_elastic(r, MOD, 1e-10, precision=1)
        assert list(g.iters) == [1] * 6
        np.testing.assert_allclose(g.C, C, atol=1e-10 * np.abs(C).max())
    with rh.rve_create_from_phases(geom.random_phases(16, 3)) as r:
        c = rh.homogenize_elastic(r, MOD, 1e-30, precision=1, max_iter=7)
        assert c.status == rh.RVE_NOT_CONVERGED and list(c.iters) == [7] * 6
