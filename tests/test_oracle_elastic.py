"""Pins of the FP64 elastic oracle (the elastic case Sec. 6 names as the
extension of the method): closed forms and an independent formulation.

Nothing here retypes the oracle's formulas: Hill's exact bulk modulus for
phases of equal shear modulus, the layered-laminate (Backus) stiffness, a
dense Galerkin solve in displacements on an odd grid, the homogeneous
medium, symmetry and the Voigt / Reuss bounds, and the contraction rate.
"""
import numpy as np
import pytest

import oracle
from paper_1504_07499_amd import geom

# bulk, shear modulus per phase: matrix, inclusion, coating
MOD = np.array([[10.0, 3.0], [2.0, 1.0], [50.0, 30.0]])

# Voigt load cases: unit normal strains, unit engineering shear strains
EV = np.diag([1.0, 1.0, 1.0, 0.5, 0.5, 0.5])


def voigt_matrix(S):
    """Column j = Voigt stress (11, 22, 33, 23, 13, 12) for Voigt strain j."""
    return np.asarray(S).T.copy()


def iso_voigt(kappa, mu):
    lam = kappa - 2.0 * mu / 3.0
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] = lam + 2 * mu
    C[np.arange(3, 6), np.arange(3, 6)] = mu
    return C


def freqs(n):
    return np.array([k if k < (n + 1) // 2 else k - n for k in range(n)], dtype=float)


@pytest.mark.parametrize("n", [5, 8])
def test_homogeneous_medium_exact(n):
    """One phase everywhere: C_hom = C after one iteration."""
    ph = np.full((n, n, n), 2, np.uint8)
    r = oracle.homogenize_elastic(ph, MOD, EV, tol=1e-12)
    assert list(r.iters) == [1] * 6
    np.testing.assert_allclose(voigt_matrix(r.S), iso_voigt(*MOD[2]), atol=1e-12 * 110)


@pytest.mark.parametrize("n,seed", [(5, 3), (6, 4), (9, 5)])
def test_equal_shear_hill_bulk_modulus(n, seed):
    """Phases of equal shear modulus mu: under a hydrostatic mean strain the
    mean stress is kappa* tr(E) I with Hill's exact
    1 / (kappa* + 4 mu / 3) = <1 / (kappa + 4 mu / 3)>, for any geometry."""
    mod = np.array([[10.0, 3.0], [2.0, 3.0], [50.0, 3.0]])
    ph = geom.random_phases(n, seed)
    E = np.array([[1.0, 1.0, 1.0, 0.0, 0.0, 0.0]]) / 3.0
    r = oracle.homogenize_elastic(ph, mod, E, tol=1e-13, max_iter=20000)
    assert r.status[0] == 0
    kv = mod[ph, 0]
    khill = 1.0 / np.mean(1.0 / (kv + 4.0)) - 4.0
    np.testing.assert_allclose(r.S[0, :3], khill, rtol=1e-11)
    assert np.abs(r.S[0, 3:]).max() <= 1e-11 * khill


def _laminate(n, widths, phases):
    prof = np.concatenate([np.full(w, p, np.uint8) for w, p in zip(widths, phases)])
    return np.broadcast_to(prof.reshape(1, 1, n), (n, n, n)).copy()  # layers normal to x


def _backus(ph, mod):
    """Stiffness of layers normal to x (series for the normal and the two
    normal-shear components, parallel for the in-plane ones)."""
    kap, mu = mod[ph[0, 0], 0], mod[ph[0, 0], 1]
    lam = kap - 2 * mu / 3
    a = lam + 2 * mu
    h = lambda v: np.mean(v)
    C = np.zeros((6, 6))
    C11 = 1.0 / h(1 / a)
    C12 = h(lam / a) * C11
    C[0, 0] = C11
    C[0, 1] = C[1, 0] = C[0, 2] = C[2, 0] = C12
    C[1, 1] = C[2, 2] = h(a - lam ** 2 / a) + h(lam / a) ** 2 * C11
    C[1, 2] = C[2, 1] = h(lam - lam ** 2 / a) + h(lam / a) ** 2 * C11
    C[3, 3] = h(mu)                          # 23: in-plane shear
    C[4, 4] = C[5, 5] = 1.0 / h(1 / mu)      # 13, 12: shear across the layers
    return C


@pytest.mark.parametrize("n,widths,phases", [(9, [2, 4, 3], [0, 1, 2]), (8, [3, 5], [0, 2])])
def test_laminate_exact(n, widths, phases):
    """Layered laminate: the Backus stiffness (the strain components in the
    layer plane and the tractions on it are uniform)."""
    ph = _laminate(n, widths, phases)
    r = oracle.homogenize_elastic(ph, MOD, EV, tol=1e-13, max_iter=20000)
    assert np.all(r.status == 0)
    np.testing.assert_allclose(voigt_matrix(r.S), _backus(ph, MOD), atol=1e-10 * 60)


def _dense_displacement_solve(ph, mod):
    """Independent formulation for odd N: u periodic, e = E + sym(grad u)
    with spectral derivatives, div(C : e) = 0, dense linear solve."""
    n = ph.shape[0]
    j = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(j, j) / n)
    D1 = np.real(np.conj(F) / n @ np.diag(1j * freqs(n)) @ F)
    I = np.eye(n)
    D = [np.kron(I, np.kron(I, D1)), np.kron(I, np.kron(D1, I)), np.kron(D1, np.kron(I, I))]
    M = n ** 3
    kap = mod[ph.ravel(), 0]
    mu = mod[ph.ravel(), 1]
    lam = kap - 2 * mu / 3
    # strain (i, j) from u: (D_j u_i + D_i u_j) / 2 ; stress = lam tr e I + 2 mu e
    def strain_op(i, jj):
        Z = np.zeros((M, 3 * M))
        Z[:, i * M:(i + 1) * M] += 0.5 * D[jj]
        Z[:, jj * M:(jj + 1) * M] += 0.5 * D[i]
        return Z
    Eop = {(i, jj): strain_op(i, jj) for i in range(3) for jj in range(3)}
    tr = Eop[(0, 0)] + Eop[(1, 1)] + Eop[(2, 2)]
    Sop = {}
    for i in range(3):
        for jj in range(3):
            Sop[(i, jj)] = 2 * mu[:, None] * Eop[(i, jj)] + ((lam[:, None] * tr) if i == jj else 0)
    A = np.zeros((3 * M, 3 * M))
    for i in range(3):
        for jj in range(3):
            A[i * M:(i + 1) * M] += D[jj] @ Sop[(i, jj)]
    S = np.zeros((6, 6))
    for lc in range(6):
        Et = np.zeros((3, 3))
        for q, (a, b) in enumerate(oracle.EL_COMPS):
            Et[a, b] = Et[b, a] = EV[lc, q]
        s0 = {(i, jj): 2 * mu * Et[i, jj] + (lam * np.trace(Et) if i == jj else 0) for i in range(3) for jj in range(3)}
        b = np.zeros(3 * M)
        for i in range(3):
            for jj in range(3):
                b[i * M:(i + 1) * M] -= D[jj] @ s0[(i, jj)]
        u = np.linalg.lstsq(A, b, rcond=None)[0]
        for q, (a, bb) in enumerate(oracle.EL_COMPS):
            S[lc, q] = np.mean(s0[(a, bb)] + Sop[(a, bb)] @ u)
    return S


def test_odd_grid_matches_dense_displacement_solve():
    """N = 5: the fixed point is the Galerkin solution of the displacement
    problem (independent of the reference medium)."""
    ph = geom.random_phases(5, 7)
    ref = _dense_displacement_solve(ph, MOD)
    r = oracle.homogenize_elastic(ph, MOD, EV, tol=1e-13, max_iter=20000)
    assert np.all(r.status == 0)
    np.testing.assert_allclose(r.S, ref, atol=1e-10 * np.abs(ref).max())


def test_symmetry_bounds_and_rate():
    """Major symmetry, Reuss <= C_hom <= Voigt (as quadratic forms), and an
    asymptotic rate at most max over the two moduli of
    (sqrt c - 1) / (sqrt c + 1) on an odd grid."""
    ph = geom.random_phases(9, 12)
    r = oracle.homogenize_elastic(ph, MOD, EV, tol=1e-12, max_iter=20000)
    C = voigt_matrix(r.S)
    assert np.abs(C - C.T).max() <= 1e-9 * np.abs(C).max()
    # compare in Mandel form (orthonormal) so that the quadratic forms are tensor norms
    w = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    Cm = C * np.outer(w, w)
    cv = [iso_voigt(*MOD[p]) * np.outer(w, w) for p in range(3)]
    f = np.bincount(ph.ravel(), minlength=3) / ph.size
    voigt = sum(f[p] * cv[p] for p in range(3))
    reuss = np.linalg.inv(sum(f[p] * np.linalg.inv(cv[p]) for p in range(3)))
    assert np.linalg.eigvalsh(voigt - 0.5 * (Cm + Cm.T)).min() >= -1e-9
    assert np.linalg.eigvalsh(0.5 * (Cm + Cm.T) - reuss).min() >= -1e-9
    ck = MOD[:, 0].max() / MOD[:, 0].min()
    cm = MOD[:, 1].max() / MOD[:, 1].min()
    rho = max((np.sqrt(ck) - 1) / (np.sqrt(ck) + 1), (np.sqrt(cm) - 1) / (np.sqrt(cm) + 1))
    for h in r.history:
        assert (h[-1] / h[-21]) ** (1 / 20) <= rho * 1.02
