"""Pins for oracle.rbf: kernel derivatives (Sec. 3 closed forms and the Hermite form)."""
import numpy as np
import numpy.polynomial.hermite as nph
import pytest

from oracle import rbf


@pytest.mark.parametrize("k", range(8))
def test_hermite_matches_numpy_physicists_series(k):
    z = np.linspace(-4, 4, 41)
    coef = np.zeros(k + 1)
    coef[k] = 1.0
    np.testing.assert_allclose(rbf.hermite(k, z), nph.hermval(z, coef), rtol=1e-12, atol=1e-9)


def test_first_and_second_derivative_match_paper_closed_forms():
    # Sec. 3: d/du K = -2(u-v)/sigma^2 K ; d2/du2 K = (4(u-v)^2/sigma^4 - 2/sigma^2) K
    sig = 0.37
    u = np.linspace(-1, 1, 23)[:, None]
    v = np.array([0.1, -0.4, 0.77])[None, :]
    k = np.exp(-((u - v) ** 2) / sig ** 2)
    np.testing.assert_allclose(rbf.kernel_du(1, u, v, sig), -2 * (u - v) / sig ** 2 * k, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(rbf.kernel_du(2, u, v, sig),
                               (4 * (u - v) ** 2 / sig ** 4 - 2 / sig ** 2) * k, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_derivative_matches_central_difference(d):
    sig, h = 0.5, 1e-5
    u = np.linspace(-1.5, 1.5, 31)
    fd = (rbf.kernel_du(d - 1, u + h, 0.2, sig) - rbf.kernel_du(d - 1, u - h, 0.2, sig)) / (2 * h)
    scale = np.max(np.abs(rbf.kernel_du(d, u, 0.2, sig)))
    np.testing.assert_allclose(rbf.kernel_du(d, u, 0.2, sig), fd, atol=1e-7 * scale)


def test_mixed_partial_matches_difference_in_second_argument():
    sig, h = 0.6, 1e-5
    u = np.linspace(-1, 1, 17)
    for a in range(3):
        for c in range(1, 3):
            fd = (rbf.kernel_mixed(a, c - 1, u, 0.3 + h, sig) - rbf.kernel_mixed(a, c - 1, u, 0.3 - h, sig)) / (2 * h)
            scale = np.max(np.abs(fd)) + 1
            np.testing.assert_allclose(rbf.kernel_mixed(a, c, u, 0.3, sig), fd, atol=1e-7 * scale)


@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_sigma_derivative_matches_central_difference(d):
    sig, h = 0.45, 1e-6
    u = np.linspace(-1, 1, 21)
    fd = (rbf.kernel_du(d, u, 0.1, sig + h) - rbf.kernel_du(d, u, 0.1, sig - h)) / (2 * h)
    scale = np.max(np.abs(fd))
    np.testing.assert_allclose(rbf.kernel_du_dsigma(d, u, 0.1, sig), fd, atol=1e-7 * scale)


def test_kernel_is_symmetric_and_unit_on_diagonal():
    u = np.linspace(0, 1, 9)
    k = rbf.kernel(u[:, None], u[None, :], 0.3)
    np.testing.assert_array_equal(k, k.T)
    np.testing.assert_array_equal(np.diag(k), 1.0)
