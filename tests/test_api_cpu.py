"""Host-side definitions of the binding that need no GPU: the orthonormal
basis of the elastic case and the modulus conversion."""
import numpy as np

import paper_1504_07499_amd as rh


def _iso(kappa, mu):
    d = np.eye(3)
    lam = kappa - 2.0 * mu / 3.0
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def test_elastic_basis_is_orthonormal_and_symmetric():
    B = rh.ELASTIC_BASIS
    assert B.shape == (6, 3, 3)
    assert np.allclose(B, np.transpose(B, (0, 2, 1)))
    np.testing.assert_allclose(np.einsum("kij,lij->kl", B, B), np.eye(6), atol=1e-15)


def test_isotropic_stiffness_is_diagonal_in_the_basis():
    """B_k : C : B_l = diag(3 kappa, 2 mu, 2 mu, 2 mu, 2 mu, 2 mu): the update
    of each basis component is independent of the others."""
    B = rh.ELASTIC_BASIS
    C = _iso(7.0, 2.5)
    Cb = np.einsum("kij,ijmn,lmn->kl", B, C, B)
    np.testing.assert_allclose(Cb, np.diag([21.0, 5.0, 5.0, 5.0, 5.0, 5.0]), atol=1e-13)


def test_moduli_from_young_poisson():
    m = rh.moduli_from_young_poisson([1.0, 200.0], [0.25, 0.3])
    np.testing.assert_allclose(m[0], [2.0 / 3.0, 0.4])
    np.testing.assert_allclose(m[1], [200.0 / 1.2, 200.0 / 2.6])
