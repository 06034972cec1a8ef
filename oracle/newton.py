"""Lemma 2: Newton's method on the primal KKT system of a first-order nonlinear ODE (oracle).

Paper: Sec. 2 (the nonlinear primal problem with extra unknowns y_i, eq. 2.2),
Sec. 3.2 (Lemma 2, Newton iteration and its convergence theorem), App. A.5
(Lagrangian and KKT functions Y1..Y4 for the first-order IVP y' = F(t, y)).

Unknowns x = (omega[r], b, lam, y[|I|]) over the residual set I = 2..n.  With
phi_i = phi(t_i), phi'_i = phi'(t_i), rho_i = phi'_i^T omega - F(t_i, y_i) and
eta_i = y_i - phi_i^T omega - b, the Lagrangian of App. A.5 is
    L = 1/2 |omega|^2 + gamma/2 sum rho_i^2 + gamma/2 sum eta_i^2
        + lam (phi_1^T omega + b - v)
and its gradient Y = (Y1, Y2, Y3, Y4) is
    Y1 = omega + gamma sum rho_i phi'_i - gamma sum eta_i phi_i + lam phi_1
    Y2 = -gamma sum eta_i + lam
    Y3 = phi_1^T omega + b - v
    Y4_i = -gamma rho_i F_y(t_i, y_i) + gamma eta_i.
The Jacobian J is the Hessian of L (symmetric).  Its y-block is diagonal:
    dY4_i/dy_i = gamma (1 + F_y^2 - rho_i F_yy).
Newton: x <- x - J^{-1} Y.  Two ways of solving J dx = Y are given: the dense
system (what the paper states, size r+2+|I|) and the Schur complement that
eliminates the diagonal y-block first (same result, exactly up to rounding).
"""
import numpy as np

from . import nystrom
from .linear import residual_set


def setup(prob):
    """Basis and the feature rows needed by every Newton step."""
    t = np.asarray(prob["t"], dtype=np.float64)
    t_land = t[nystrom.landmark_indices(prob)]
    lam, u, r, w = nystrom.basis(t_land, prob["sigma"], prob["tau"])
    idx = residual_set(t.size, prob["cond_i"])
    phi = nystrom.features(0, t[idx], t_land, prob["sigma"], w)
    dphi = nystrom.features(1, t[idx], t_land, prob["sigma"], w)
    i0 = int(prob["cond_i"][0])
    phi1 = nystrom.features(0, t[i0], t_land, prob["sigma"], w)[0]
    return dict(t=t, t_land=t_land, lam=lam, U=u, r=r, W=w, idx=idx,
                phi=phi, dphi=dphi, phi1=phi1)


def unpack(x, r):
    return x[:r], x[r], x[r + 1], x[r + 2:]


def lagrangian(x, st, prob, fun):
    """The App. A.5 Lagrangian at x (used to pin Y by differentiation)."""
    r = st["r"]
    om, b, lm, y = unpack(x, r)
    fv, _, _ = fun(st["idx"], y)
    rho = st["dphi"] @ om - fv
    eta = y - st["phi"] @ om - b
    g = float(prob["gamma"])
    v = float(np.asarray(prob["v"]).ravel()[0])
    return (0.5 * om @ om + 0.5 * g * rho @ rho + 0.5 * g * eta @ eta
            + lm * (st["phi1"] @ om + b - v))


def residual(x, st, prob, fun):
    """Y(x) = grad L(x), written out as in App. A.5."""
    r = st["r"]
    om, b, lm, y = unpack(x, r)
    fv, fy, _ = fun(st["idx"], y)
    rho = st["dphi"] @ om - fv
    eta = y - st["phi"] @ om - b
    g = float(prob["gamma"])
    v = float(np.asarray(prob["v"]).ravel()[0])
    y1 = om + g * st["dphi"].T @ rho - g * st["phi"].T @ eta + lm * st["phi1"]
    y2 = -g * np.sum(eta) + lm
    y3 = st["phi1"] @ om + b - v
    y4 = -g * rho * fy + g * eta
    return np.concatenate([y1, [y2, y3], y4])


def jacobian(x, st, prob, fun):
    """Dense symmetric Jacobian dY/dx of size r + 2 + |I|."""
    r = st["r"]
    om, b, lm, y = unpack(x, r)
    fv, fy, fyy = fun(st["idx"], y)
    rho = st["dphi"] @ om - fv
    g = float(prob["gamma"])
    ni = y.size
    nn = r + 2 + ni
    jac = np.zeros((nn, nn))
    phi, dphi = st["phi"], st["dphi"]
    jac[:r, :r] = np.eye(r) + g * dphi.T @ dphi + g * phi.T @ phi
    jac[:r, r] = g * phi.sum(axis=0)
    jac[:r, r + 1] = st["phi1"]
    qy = -g * (fy[:, None] * dphi + phi)           # dY1/dy_i as rows
    jac[:r, r + 2:] = qy.T
    jac[r, r] = g * ni
    jac[r, r + 1] = 1.0
    jac[r, r + 2:] = -g
    jac[r + 1, :r] = st["phi1"]
    jac[r + 1, r] = 1.0
    jac[r + 2:, :r] = qy
    jac[r:r + 1, :r] = jac[:r, r][None, :]
    jac[r + 2:, r] = -g
    jac[r + 2:, r + 2:] = np.diag(g * (1.0 + fy * fy - rho * fyy))
    return jac


def step_dense(x, st, prob, fun):
    """One Newton step solving the full dense system (the paper's formulation)."""
    dx = np.linalg.solve(jacobian(x, st, prob, fun), residual(x, st, prob, fun))
    return x - dx, dx


def step_schur(x, st, prob, fun):
    """One Newton step with the diagonal y-block eliminated first.

    J = [[A, B], [B^T, D]] with D diagonal: (A - B D^-1 B^T) dz = Y_z - B D^-1 Y_y,
    dy = D^-1 (Y_y - B^T dz).
    """
    r = st["r"]
    jac = jacobian(x, st, prob, fun)
    yv = residual(x, st, prob, fun)
    nz = r + 2
    a = jac[:nz, :nz]
    bm = jac[:nz, nz:]
    dg = np.diag(jac[nz:, nz:])
    schur = a - (bm / dg[None, :]) @ bm.T
    dz = np.linalg.solve(schur, yv[:nz] - bm @ (yv[nz:] / dg))
    dy = (yv[nz:] - bm.T @ dz) / dg
    dx = np.concatenate([dz, dy])
    return x - dx, dx


def initial_state(st, prob):
    """Start of the iteration: omega = 0, b = v, lam = 0, y_i = v."""
    v = float(np.asarray(prob["v"]).ravel()[0])
    x = np.zeros(st["r"] + 2 + st["idx"].size)
    x[st["r"]] = v
    x[st["r"] + 2:] = v
    return x


def solve(prob, fun, tol=1e-12, max_iter=15, schur=False):
    """Newton iteration to |dx|_inf < tol or max_iter steps.

    Returns dict(x, iters, steps=[|dx|_inf per step], yhat on the grid, alpha, b, ...).
    """
    st = setup(prob)
    x = initial_state(st, prob)
    steps = []
    xs = [x.copy()]
    for _ in range(max_iter):
        x, dx = (step_schur if schur else step_dense)(x, st, prob, fun)
        xs.append(x.copy())
        steps.append(float(np.max(np.abs(dx))))
        if steps[-1] < tol:
            break
    r = st["r"]
    om, b, lm, y = unpack(x, r)
    alpha = st["W"] @ om
    yhat = nystrom.kvec(0, st["t"], st["t_land"], prob["sigma"]) @ alpha + b
    st.update(x=x, iterates=xs, steps=steps, iters=len(steps), omega=om, b=b,
              lam_kkt=lm, y=y, alpha=alpha, yhat=yhat)
    return st
