"""Leverage-score landmark sampling for the Nystrom basis (oracle).

Test infrastructure only (like the rest of oracle/): never imported by the library or its
binding.

Paper: Sec. 4.1, "Sampling strategy analysis for Nystrom landmarks" (equidistant, random and
leverage-score sampling compared; Table 1 and the per-problem Table 5).  The paper names
leverage-score sampling but gives no formula; the readings taken here:

  * scores: ridge leverage scores of the grid points in the feature space of a pilot
    Nystrom basis (the instance's own landmarks, sigma and cut-off),
        l_i = phi(t_i)^T (Phi^T Phi + (1/gamma) I)^{-1} phi(t_i),   Phi = [phi(t_i)]_i (all n),
    with the ridge 1/gamma of the LS-SVM objective (1/2 |omega|^2 + gamma/2 sum e_i^2);
  * sampling: m distinct grid indices with probabilities proportional to l_i, without
    replacement, by exponential keys (Efraimidis and Spirakis, "Weighted random sampling with
    a reservoir", 2006): key_i = ln(u_i) / l_i with uniforms u_i in (0, 1) handed in by the
    caller, and the m largest keys are taken.  With `ends` the first and last grid points are
    always landmarks and the other m - 2 are drawn from the interior.
"""
import numpy as np

from . import nystrom


def scores(prob, ridge=None):
    """Ridge leverage scores l_i of every grid point (n,) for the instance's pilot basis."""
    t = np.asarray(prob["t"], dtype=np.float64)
    t_land = t[nystrom.landmark_indices(prob)]
    _, _, r, w = nystrom.basis(t_land, prob["sigma"], prob["tau"])
    phi = nystrom.features(0, t, t_land, prob["sigma"], w)          # n x r
    lam = 1.0 / float(prob["gamma"]) if ridge is None else float(ridge)
    g = phi.T @ phi + lam * np.eye(r)
    return np.einsum("ij,ji->i", phi, np.linalg.solve(g, phi.T))


def exact_ridge_scores(kfull, ridge):
    """The definition the scores reduce to when the features reproduce K exactly (m = n):
    diag(K (K + ridge I)^{-1})."""
    n = kfull.shape[0]
    return np.diag(kfull @ np.linalg.inv(kfull + ridge * np.eye(n)))


def sample(score, m, u, ends=True):
    """m ascending distinct grid indices: the m largest keys ln(u_i) / score_i (with `ends`:
    indices 0 and n-1 plus the m - 2 largest keys among the interior)."""
    score = np.asarray(score, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n = score.size
    key = np.log(u) / score
    if ends:
        inner = np.arange(1, n - 1)
        order = inner[np.argsort(-key[1:n - 1], kind="stable")][:m - 2]
        idx = np.concatenate([[0], order, [n - 1]])
    else:
        idx = np.argsort(-key, kind="stable")[:m]
    return np.sort(idx).astype(np.int64)
