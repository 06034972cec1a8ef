"""Lemma 1: the primal KKT system for p-th order linear ODEs (oracle).

Paper: Sec. 3.1 (problem statement, optimisation problem, Lemma 1 and its
matrix), App. A.3 (Lagrangian and KKT conditions; first-order IVP), App. A.4
(second-order IVP and BVP).

ODE (Sec. 3.1):  y^(p)(t) - sum_{k=1..p} f_k(t) y^(p-k)(t) = r(t)
conditions:      y^(d_j)(t_{i_j}) = v_j,  j = 1..p
model:           y_hat(t) = omega^T phi(t) + b

For every grid point i in the residual set I (all grid indices that carry no
condition; for an IVP i = 2..n, for a two-point BVP i = 2..n-1) the residual is
    e_i = omega^T g_i + c_i b - r_i,
    g_i = phi^(p)(t_i) - sum_k f_k(t_i) phi^(p-k)(t_i) = W^T p_i,
    p_i = k_m^(p)(t_i) - sum_k f_k(t_i) k_m^(p-k)(t_i),   c_i = -f_p(t_i).
Minimising 1/2 |omega|^2 + gamma/2 sum e_i^2 subject to
omega^T h_j + delta_j b = v_j (h_j = phi^(d_j)(t_{i_j}), delta_j = [d_j = 0])
gives the symmetric (r+1+p) system of Lemma 1:
    [ I + gamma G^T G   gamma G^T c   H ] [omega]   [gamma G^T r]
    [ gamma c^T G       gamma c^T c   d ] [  b  ] = [gamma c^T r]
    [ H^T               d^T           0 ] [ lam ]   [     v     ]
Term by term this is the paper's matrix with A = gamma G^T, V = gamma c^T,
E = I and -A (f_p 1) = gamma G^T c.  (The paper's "(m+p)" size counts the
bias and multipliers loosely; the system has r + 1 + p unknowns.)  The sign of
lam differs between Sec. 3.1 and App. A.3; omega, b and y_hat do not depend on it.
"""
import numpy as np

from . import nystrom


def _data(x):
    """Float64 array, or complex128 when the caller perturbs data by a complex step."""
    x = np.asarray(x)
    return x.astype(np.complex128 if np.iscomplexobj(x) else np.float64)


def residual_set(n, cond_i):
    """Grid indices that carry an ODE residual: all points minus the condition points."""
    mask = np.ones(n, dtype=bool)
    mask[np.asarray(cond_i, dtype=np.int64)] = False
    return np.nonzero(mask)[0]


def operator_rows(prob, w, t_land):
    """p_i (|I| x m, kernel space), g_i = W^T p_i, c_i and r_i over the residual set."""
    p = int(prob["p"])
    t = np.asarray(prob["t"], dtype=np.float64)
    f = _data(prob["f"]).reshape(p, -1)
    idx = residual_set(t.size, prob["cond_i"])
    ti = t[idx]
    pk = nystrom.kvec(p, ti, t_land, prob["sigma"])
    for k in range(1, p + 1):
        pk = pk - f[k - 1, idx][:, None] * nystrom.kvec(p - k, ti, t_land, prob["sigma"])
    c = -f[p - 1, idx]
    r = _data(prob["r"])[idx]
    return idx, pk, pk @ w, c, r


def condition_rows(prob, w, t_land):
    """H (r x p) with columns h_j = phi^(d_j)(t_{i_j}), and delta_j = [d_j == 0]."""
    t = np.asarray(prob["t"], dtype=np.float64)
    cols = []
    for d, i in zip(prob["cond_d"], prob["cond_i"]):
        cols.append(nystrom.features(int(d), t[int(i)], t_land, prob["sigma"], w)[0])
    h = np.stack(cols, axis=1)
    delta = np.array([1.0 if int(d) == 0 else 0.0 for d in prob["cond_d"]])
    return h, delta


def assemble(prob):
    """Build the Lemma 1 system.  Returns a dict with A (r+1+p square), rhs and the pieces."""
    p = int(prob["p"])
    t = np.asarray(prob["t"], dtype=np.float64)
    t_land = t[nystrom.landmark_indices(prob)]
    lam, u, r, w = nystrom.basis(t_land, prob["sigma"], prob["tau"])
    idx, pk, g, c, rr = operator_rows(prob, w, t_land)
    h, delta = condition_rows(prob, w, t_land)
    gam = prob["gamma"]
    vv = _data(prob["v"])
    nsys = r + 1 + p
    dt = np.result_type(g, rr, vv, gam)
    a = np.zeros((nsys, nsys), dtype=dt)
    a[:r, :r] = np.eye(r) + gam * g.T @ g
    a[:r, r] = gam * g.T @ c
    a[r, :r] = gam * c @ g
    a[r, r] = gam * c @ c
    a[:r, r + 1:] = h
    a[r + 1:, :r] = h.T
    a[r, r + 1:] = delta
    a[r + 1:, r] = delta
    rhs = np.zeros(nsys, dtype=dt)
    rhs[:r] = gam * g.T @ rr
    rhs[r] = gam * c @ rr
    rhs[r + 1:] = vv
    return dict(A=a, rhs=rhs, lam=lam, U=u, r=r, W=w, t_land=t_land, idx=idx,
                P=pk, G=g, c=c, rvec=rr, H=h, delta=delta)


def solve(prob):
    """Solve Lemma 1 with LAPACK LU and evaluate y_hat on the grid.

    Returns the assembly dict extended with omega, b, lam_kkt, alpha = W omega
    and yhat (y_hat at every grid point).
    """
    out = assemble(prob)
    x = np.linalg.solve(out["A"], out["rhs"])
    r = out["r"]
    omega, b, lk = x[:r], x[r], x[r + 1:]
    alpha = out["W"] @ omega
    t = np.asarray(prob["t"], dtype=np.float64)
    yhat = nystrom.kvec(0, t, out["t_land"], prob["sigma"]) @ alpha + b
    out.update(x=x, omega=omega, b=b, lam_kkt=lk, alpha=alpha, yhat=yhat)
    return out


def predict(sol, t, sigma, d=0):
    """d-th derivative of y_hat(t) = alpha^T k_m(t) + b at arbitrary times."""
    val = nystrom.kvec(d, t, sol["t_land"], sigma) @ sol["alpha"]
    return val + (sol["b"] if d == 0 else 0.0)
