"""Pins of the oracle's covariance functions against independent definitions."""
import math

import numpy as np
import pytest
from scipy.special import gamma, kv

from oracle import matern


def general_matern(nu, d, ell, s2):
    """Matern(nu) through the modified Bessel function of the second kind."""
    z = np.sqrt(2.0 * nu) * np.asarray(d) / ell
    return s2 * (2.0 ** (1.0 - nu) / gamma(nu)) * z ** nu * kv(nu, z)


@pytest.mark.parametrize("nu2", [1, 3, 5])
def test_closed_forms_match_bessel_definition(nu2):
    d = np.array([1e-3, 0.05, 0.2, 0.5, 1.0, 2.5, 7.0])
    for ell, s2 in [(0.2, 1.0), (0.3, 2.5), (1.7, 0.4)]:
        ref = general_matern(nu2 / 2.0, d, ell, s2)
        np.testing.assert_allclose(matern.matern(nu2, d, ell, s2), ref, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("nu2", [1, 3, 5])
def test_value_at_zero_is_variance(nu2):
    assert matern.matern(nu2, np.array([0.0]), 0.3, 1.7)[0] == pytest.approx(1.7, rel=0, abs=1e-15)


@pytest.mark.parametrize("nu2", [1, 3, 5])
def test_lengthscale_derivative_matches_finite_differences(nu2):
    d = np.linspace(0.01, 3.0, 25)
    ell, s2, h = 0.37, 1.3, 1e-6
    fd = (matern.matern(nu2, d, ell + h, s2) - matern.matern(nu2, d, ell - h, s2)) / (2 * h)
    np.testing.assert_allclose(matern.matern_dell(nu2, d, ell, s2), fd, rtol=1e-7, atol=1e-10)


def test_geodesic_is_arccos_for_unit_vectors_and_zero_on_the_diagonal():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((7, 3))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    geo = matern.distances(A, A, matern.GEODESIC)
    np.testing.assert_allclose(geo, np.arccos(np.clip(A @ A.T, -1, 1)), atol=1e-7)
    # rounding of the length (e.g. FP32 inputs) must not move a point away from itself
    A32 = A.astype(np.float32).astype(np.float64)
    assert np.abs(np.diag(matern.distances(A32, A32, matern.GEODESIC))).max() < 1e-12


def test_geodesic_is_twice_arcsine_of_half_chord():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((9, 3))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    chord = matern.distances(A, A, matern.EUCLID)
    geo = matern.distances(A, A, matern.GEODESIC)
    np.testing.assert_allclose(geo, 2.0 * np.arcsin(np.clip(chord / 2.0, 0, 1)), atol=1e-7)


@pytest.mark.parametrize("nu2", [1, 3, 5])
def test_gram_is_psd_in_the_plane_and_chordal_on_sphere(nu2):
    rng = np.random.default_rng(2)
    X = rng.random((60, 2))
    lam = np.linalg.eigvalsh(matern.gram(X, X, nu2, 0.3))
    assert lam.min() > -1e-10
    S = rng.standard_normal((60, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    lam = np.linalg.eigvalsh(matern.gram(S, S, nu2, 0.3))
    assert lam.min() > -1e-10


def test_chunked_matmul_equals_dense_product():
    rng = np.random.default_rng(3)
    A, B = rng.random((37, 2)), rng.random((23, 2))
    V = rng.standard_normal((23, 4))
    ref = matern.gram(A, B, 5, 0.4, 1.1) @ V
    got = matern.gram_matmul(A, B, V, 5, 0.4, 1.1, rows_per_chunk=5)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)
