"""Dual LS-SVM for p-th order linear ODEs with an arbitrary kernel (oracle cross-check).

Paper: Sec. 2 and App. A.1 describe the classical LS-SVM ODE solver, whose
dual for the linear IVP is an (n+p)-sized system built from the kernel and
its mixed partials nabla^a_c K (Sec. 3, the Omega^a_c matrices).  It is
written out here from the Lagrangian of the same primal problem as Lemma 1,
with one multiplier a_i per residual constraint and one beta_j per condition:
    omega = sum_i a_i g_i + sum_j beta_j h_j,   e_i = -a_i / gamma,
    [ Omega_gg + I/gamma  Omega_gh  c ] [a   ]   [r]
    [ Omega_gh^T          Omega_hh  d ] [beta] = [v]
    [ c^T                 d^T       0 ] [b   ]   [0]
    y_hat^(d)(t) = sum_i a_i <g_i, phi^(d)(t)> + sum_j beta_j <h_j, phi^(d)(t)> + [d=0] b
where every inner product of features is a mixed partial of the kernel:
<phi^(a)(u), phi^(c)(v)> = d^a/du^a d^c/dv^c K(u, v), and g_i applies the ODE
operator L = d^p - sum_k f_k d^(p-k) in the first argument.

Two kernels are used: the Nystrom kernel K~(u, v) = k_m(u)^T W W^T k_m(v),
for which this dual and the primal Lemma 1 solve the same problem (strong
duality, equal up to rounding), and the true RBF kernel, which gives the
classical LS-SVM solution (a different function space; close, not equal).
"""
import numpy as np

from . import nystrom, rbf
from .linear import residual_set


def nystrom_kernel(t_land, sigma, w):
    """Mixed partials of K~(u, v) = k_m(u)^T W W^T k_m(v)."""
    q = w @ w.T

    def kmix(a, c, u, v):
        ku = nystrom.kvec(a, u, t_land, sigma)
        kv = nystrom.kvec(c, v, t_land, sigma)
        return ku @ q @ kv.T
    return kmix


def rbf_kernel(sigma):
    """Mixed partials of the true RBF kernel."""
    def kmix(a, c, u, v):
        u = np.atleast_1d(np.asarray(u, dtype=np.float64))
        v = np.atleast_1d(np.asarray(v, dtype=np.float64))
        return rbf.kernel_mixed(a, c, u[:, None], v[None, :], sigma)
    return kmix


def solve(prob, kmix):
    """Solve the dual system; returns a predictor y_hat^(d)(t) and the dual variables."""
    p = int(prob["p"])
    t = np.asarray(prob["t"], dtype=np.float64)
    f = np.asarray(prob["f"], dtype=np.float64).reshape(p, -1)
    idx = residual_set(t.size, prob["cond_i"])
    ti = t[idx]
    wts = {p: np.ones(idx.size)}                     # operator weights w_d(t_i)
    for k in range(1, p + 1):
        wts[p - k] = -f[k - 1, idx]
    c = -f[p - 1, idx]
    rr = np.asarray(prob["r"], dtype=np.float64)[idx]
    cd = [int(d) for d in prob["cond_d"]]
    ct = np.array([t[int(i)] for i in prob["cond_i"]])
    ni = idx.size
    ogg = np.zeros((ni, ni))
    for a in range(p + 1):
        for cc in range(p + 1):
            ogg += wts[a][:, None] * wts[cc][None, :] * kmix(a, cc, ti, ti)
    ogh = np.zeros((ni, p))
    for j in range(p):
        for a in range(p + 1):
            ogh[:, j] += wts[a] * kmix(a, cd[j], ti, ct[j:j + 1])[:, 0]
    ohh = np.zeros((p, p))
    for j in range(p):
        for l in range(p):
            ohh[j, l] = kmix(cd[j], cd[l], ct[j:j + 1], ct[l:l + 1])[0, 0]
    delta = np.array([1.0 if d == 0 else 0.0 for d in cd])
    nsys = ni + p + 1
    a_mat = np.zeros((nsys, nsys))
    a_mat[:ni, :ni] = ogg + np.eye(ni) / float(prob["gamma"])
    a_mat[:ni, ni:ni + p] = ogh
    a_mat[ni:ni + p, :ni] = ogh.T
    a_mat[ni:ni + p, ni:ni + p] = ohh
    a_mat[:ni, -1] = c
    a_mat[-1, :ni] = c
    a_mat[ni:ni + p, -1] = delta
    a_mat[-1, ni:ni + p] = delta
    rhs = np.concatenate([rr, np.asarray(prob["v"], dtype=np.float64), [0.0]])
    sol = np.linalg.solve(a_mat, rhs)
    av, beta, b = sol[:ni], sol[ni:ni + p], sol[-1]

    def predict(tq, d=0):
        tq = np.atleast_1d(np.asarray(tq, dtype=np.float64))
        out = np.zeros(tq.size)
        for a in range(p + 1):
            out += (wts[a] * av) @ kmix(a, d, ti, tq)
        for j in range(p):
            out += beta[j] * kmix(cd[j], d, ct[j:j + 1], tq)[0]
        return out + (b if d == 0 else 0.0)

    return dict(a=av, beta=beta, b=b, predict=predict)
