"""Explicit Nystrom feature map of the RBF kernel (oracle).

Paper: App. A.2 (Mercer expansion, the m-sample eigenproblem of the landmark
kernel matrix Omega_(m,m), and the explicit feature eq. labelled eq32), Sec. 3
(the p-th derivative of the feature map) and Sec. 4.1 (equidistant landmark
sampling is the recommended strategy).

Readings taken where the paper is silent or inconsistent:
  * scaling: phi(t) = Lambda^{-1/2} U^T k_m(t).  The paper's eq32 carries an
    extra sqrt(m); that is the same model with gamma replaced by m*gamma.
  * the sum in eq32 runs over the landmarks s, and the derivative is taken in
    the evaluation time t.
  * K_mm is numerically singular for smooth kernels, so eigenpairs with
    lambda_k <= tau * lambda_1 are dropped (a spectral cut-off, tau an input).
  * eigenvalues in descending order; each eigenvector signed so that its
    largest-magnitude entry is positive (ties: lowest index).
  * landmark s (0-based) sits on grid index floor(s (n-1)/(m-1) + 1/2).
"""
import numpy as np

from . import rbf


def equidistant_landmarks(n, m):
    """Grid indices of m equidistant landmarks on an n-point grid (0-based).

    i_s = floor(s (n-1)/(m-1) + 1/2), computed in integers; includes both
    end points, and every grid point when m == n.
    """
    if m < 2 or m > n:
        raise ValueError("need 2 <= m <= n")
    s = np.arange(m, dtype=np.int64)
    return (2 * s * (n - 1) + (m - 1)) // (2 * (m - 1))


def landmark_indices(prob):
    """The instance's landmark grid indices: given ones, else the equidistant rule."""
    if prob.get("lidx") is not None:
        return np.asarray(prob["lidx"], dtype=np.int64)
    return equidistant_landmarks(int(np.asarray(prob["t"]).size), int(prob["m"]))


def landmark_gram(t_land, sigma):
    """K_mm[s, z] = K(t_s, t_z)."""
    t_land = np.asarray(t_land, dtype=np.float64)
    return rbf.kernel(t_land[:, None], t_land[None, :], sigma)


def eig_desc(kmm):
    """Eigenpairs of the symmetric K_mm, descending, with the sign convention."""
    lam, u = np.linalg.eigh(kmm)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    u = u[:, order].copy()
    for k in range(u.shape[1]):
        j = int(np.argmax(np.abs(u[:, k])))  # first index of the maximum
        if u[j, k] < 0:
            u[:, k] = -u[:, k]
    return lam, u


def basis(t_land, sigma, tau):
    """Nystrom basis: returns (lam[m], U[m, m], r, W[m, r]) with W = U_r Lambda_r^{-1/2}.

    r counts eigenvalues lambda_k > tau * lambda_1 (the retained rank).
    """
    lam, u = eig_desc(landmark_gram(t_land, sigma))
    r = int(np.sum(lam > tau * lam[0]))
    w = u[:, :r] / np.sqrt(lam[:r])[None, :]
    return lam, u, r, w


def kvec(d, t, t_land, sigma):
    """d-th time derivative of k_m(t) = [K(t, t_s)]_s; shape (len(t), m)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return rbf.kernel_du(d, t[:, None], np.asarray(t_land)[None, :], sigma)


def features(d, t, t_land, sigma, w):
    """phi^(d)(t) = W^T d^d/dt^d k_m(t) for every t; shape (len(t), r)."""
    return kvec(d, t, t_land, sigma) @ w
