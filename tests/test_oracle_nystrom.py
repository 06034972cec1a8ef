"""Pins for oracle.nystrom: landmarks, eigendecomposition, feature map (App. A.2, Sec. 3, Sec. 4.1)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import nystrom, rbf


def test_equidistant_landmarks_end_points_and_all_points():
    for n, m in [(200, 20), (10000, 50), (2000, 50), (7, 7), (5, 2), (10001, 101)]:
        idx = nystrom.equidistant_landmarks(n, m)
        assert idx[0] == 0 and idx[-1] == n - 1
        assert np.all(np.diff(idx) > 0)
        exact = np.floor(np.arange(m) * (n - 1) / (m - 1) + 0.5).astype(np.int64)
        np.testing.assert_array_equal(idx, exact)
    np.testing.assert_array_equal(nystrom.equidistant_landmarks(9, 9), np.arange(9))


def test_equidistant_landmarks_on_exact_spacing():
    # when (n-1) is a multiple of (m-1) the landmarks sit exactly every (n-1)/(m-1) points
    np.testing.assert_array_equal(nystrom.equidistant_landmarks(201, 21), np.arange(0, 201, 10))


def test_eigendecomposition_matches_lapack_and_reconstructs():
    t = np.linspace(0, 1, 20)
    kmm = nystrom.landmark_gram(t, 0.1)
    lam, u = nystrom.eig_desc(kmm)
    ref = scipy.linalg.eigh(kmm, eigvals_only=True)[::-1]
    np.testing.assert_allclose(lam, ref, atol=1e-13 * ref[0])
    assert np.all(np.diff(lam) <= 0)
    np.testing.assert_allclose(kmm @ u, u * lam[None, :], atol=1e-13 * lam[0])
    np.testing.assert_allclose(u.T @ u, np.eye(20), atol=1e-13)


def test_sign_convention_largest_entry_positive():
    kmm = nystrom.landmark_gram(np.linspace(0, 10, 50), 0.5)
    _, u = nystrom.eig_desc(kmm)
    for k in range(u.shape[1]):
        j = np.argmax(np.abs(u[:, k]))
        assert u[j, k] > 0


def test_full_landmark_set_reproduces_kernel_matrix():
    # m = n and full rank: Phi Phi^T = K on the grid (App. A.2 Nystrom identity)
    t = np.linspace(0, 1, 30)
    lam, u, r, w = nystrom.basis(t, 0.05, 1e-14)
    assert r == 30
    phi = nystrom.features(0, t, t, 0.05, w)
    k = rbf.kernel(t[:, None], t[None, :], 0.05)
    np.testing.assert_allclose(phi @ phi.T, k, atol=1e-13)


def test_landmark_reproduction_and_projection_bound():
    t = np.linspace(0, 2, 2000)
    idx = nystrom.equidistant_landmarks(2000, 50)
    tl = t[idx]
    lam, u, r, w = nystrom.basis(tl, 0.1, 1e-12)
    assert r == 50
    phil = nystrom.features(0, tl, tl, 0.1, w)
    np.testing.assert_allclose(phil @ phil.T, nystrom.landmark_gram(tl, 0.1), atol=1e-10)
    # phi(t)^T phi(t) is the Nystrom approximation of K(t,t) = 1 and can not exceed it
    phi = nystrom.features(0, t, tl, 0.1, w)
    nrm = np.sum(phi * phi, axis=1)
    assert np.all(nrm <= 1 + 1e-9)
    # the derivative bound ||phi'(t)||^2 <= d/du d/dv K (t, t) = 2 / sigma^2
    dphi = nystrom.features(1, t, tl, 0.1, w)
    assert np.max(np.sum(dphi * dphi, axis=1)) <= 2 / 0.1 ** 2 * (1 + 1e-9)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_feature_derivatives_match_central_difference(d):
    t = np.linspace(0, 1, 200)
    tl = t[nystrom.equidistant_landmarks(200, 20)]
    _, _, _, w = nystrom.basis(tl, 0.1, 1e-12)
    tq = np.linspace(0.03, 0.97, 15)
    h = 1e-6
    fd = (nystrom.features(d - 1, tq + h, tl, 0.1, w) - nystrom.features(d - 1, tq - h, tl, 0.1, w)) / (2 * h)
    ex = nystrom.features(d, tq, tl, 0.1, w)
    np.testing.assert_allclose(ex, fd, atol=2e-6 * np.max(np.abs(ex)))


def test_truncation_drops_eigenvalues_below_cutoff():
    t = np.linspace(0, 10, 10000)
    tl = t[nystrom.equidistant_landmarks(10000, 50)]
    lam, u, r, w = nystrom.basis(tl, 1.0, 1e-8)
    assert r < 50
    assert lam[r - 1] > 1e-8 * lam[0] >= lam[r]
    # retained features are orthonormal in the landmark inner product: W^T K_mm W = I_r
    np.testing.assert_allclose(w.T @ nystrom.landmark_gram(tl, 1.0) @ w, np.eye(r), atol=1e-7)


def test_random_landmarks_contract():
    """The seeded random landmark sets are m distinct, ascending, in-range grid indices,
    hold both end points when asked to, and repeat for the same seed."""
    from paper_2510_04094_amd import workloads
    for n, m, ends in [(200, 20, True), (237, 40, False), (100, 100, True), (50, 2, True)]:
        idx = workloads.random_landmarks(7, n, m, ends=ends)
        assert idx.size == m and np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < n
        if ends:
            assert idx[0] == 0 and idx[-1] == n - 1
        np.testing.assert_array_equal(idx, workloads.random_landmarks(7, n, m, ends=ends))
    assert not np.array_equal(workloads.random_landmarks(1, 500, 30), workloads.random_landmarks(2, 500, 30))
