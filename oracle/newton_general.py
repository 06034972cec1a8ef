"""Lemma 2 for p-th order nonlinear ODEs y^(p) = F(t, y, y', ..., y^(p-1)) (oracle).

Test infrastructure only (like the rest of oracle/): never imported by the library or its
binding.

Paper: Sec. 2 (the nonlinear primal problem with the extra unknowns y_i, eq. 2.2), Sec. 3.2
(Lemma 2: Newton's method on the gradient of the Lagrangian), App. A.4 "Nystrom method for
Lemma 2" (the general Lagrangian and its KKT functions), and the appendix section on
Problem 15 (a second-order boundary problem whose right-hand side contains y').

Readings (as in the paper's Problem 15 Lagrangian): y itself enters F through the auxiliary
unknown y_i, the derivatives y^(d), d = 1..p-1, through the model, u_{d,i} = omega^T
phi^(d)(t_i); the ODE residual and the y_i run over the residual set I (grid points without
a condition); the conditions are those of the linear path, h_j^T omega + delta_j b = v_j.

With phi^(d)_i = phi^(d)(t_i), rho_i = omega^T phi^(p)_i - F_i, eta_i = y_i - omega^T phi_i - b,
F_i = F(t_i, y_i, u_{1,i}, ..., u_{p-1,i}), F_a its partial derivative in its a-th state
argument (a = 0: y, a >= 1: u_a) and F_ab the second ones, the Lagrangian is
    L = 1/2 |omega|^2 + gamma/2 sum rho_i^2 + gamma/2 sum eta_i^2
        + sum_j lam_j (h_j^T omega + delta_j b - v_j)
and its gradient Y = (Y_omega, Y_b, Y_lam, Y_y):
    q_i     = phi^(p)_i - sum_{a>=1} F_a,i phi^(a)_i            (d rho_i / d omega)
    Y_omega = omega + gamma sum rho_i q_i - gamma sum eta_i phi_i + sum_j lam_j h_j
    Y_b     = -gamma sum eta_i + sum_j delta_j lam_j
    Y_lam_j = h_j^T omega + delta_j b - v_j
    Y_y,i   = -gamma rho_i F_0,i + gamma eta_i.
The Jacobian J is the Hessian of L (symmetric):
    J_omega,omega = I + gamma sum (q_i q_i^T - rho_i sum_{a,b>=1} F_ab,i phi^(a)_i phi^(b)_i^T
                                   + phi_i phi_i^T)
    J_omega,b = gamma sum phi_i,  J_omega,lam_j = h_j,  J_b,b = gamma |I|,  J_b,lam_j = delta_j
    J_omega,y_i = -gamma (F_0,i q_i + rho_i sum_{a>=1} F_0a,i phi^(a)_i + phi_i),  J_b,y_i = -gamma
    J_y_i,y_i = gamma (1 + F_0,i^2 - rho_i F_00,i)      (diagonal y-block).
The Gauss-Newton variant drops the terms carrying rho_i times a second derivative of F.
Newton: x <- x - J^{-1} Y, by the dense system (the paper's formulation) or by the Schur
complement that eliminates the diagonal y-block first (same step up to rounding).
"""
import numpy as np

from . import linear, nystrom


def setup(prob):
    """Basis, residual set, feature rows phi^(d)_i (d = 0..p) and condition rows."""
    p = int(prob["p"])
    t = np.asarray(prob["t"], dtype=np.float64)
    t_land = t[nystrom.landmark_indices(prob)]
    lam, u, r, w = nystrom.basis(t_land, prob["sigma"], prob["tau"])
    idx = linear.residual_set(t.size, prob["cond_i"])
    phis = [nystrom.features(d, t[idx], t_land, prob["sigma"], w) for d in range(p + 1)]
    h, delta = linear.condition_rows(prob, w, t_land)
    return dict(p=p, t=t, t_land=t_land, lam=lam, U=u, r=r, W=w, idx=idx, phis=phis,
                H=h, delta=delta)


def unpack(x, st):
    r, p = st["r"], st["p"]
    return x[:r], x[r], x[r + 1:r + 1 + p], x[r + 1 + p:]


def _state(x, st, fun):
    """rho, eta, F and its derivatives at x; fun(idx, y, u) returns (F, dF[p], d2F[p][p])
    with the state arguments ordered (y, u_1, ..., u_{p-1})."""
    om, b, _, y = unpack(x, st)
    p = st["p"]
    u = [st["phis"][d] @ om for d in range(1, p)]
    fv, df, d2f = fun(st["idx"], y, u)
    rho = st["phis"][p] @ om - fv
    eta = y - st["phis"][0] @ om - b
    q = st["phis"][p] - sum(df[a][:, None] * st["phis"][a] for a in range(1, p))
    return rho, eta, fv, np.asarray(df), np.asarray(d2f), q


def lagrangian(x, st, prob, fun):
    om, b, lm, y = unpack(x, st)
    rho, eta, _, _, _, _ = _state(x, st, fun)
    g = float(prob["gamma"])
    v = np.asarray(prob["v"], dtype=np.float64)
    cons = st["H"].T @ om + st["delta"] * b - v
    return 0.5 * om @ om + 0.5 * g * rho @ rho + 0.5 * g * eta @ eta + lm @ cons


def residual(x, st, prob, fun):
    """Y(x) = grad L(x), written out."""
    om, b, lm, y = unpack(x, st)
    rho, eta, _, df, _, q = _state(x, st, fun)
    g = float(prob["gamma"])
    v = np.asarray(prob["v"], dtype=np.float64)
    y_om = om + g * q.T @ rho - g * st["phis"][0].T @ eta + st["H"] @ lm
    y_b = -g * np.sum(eta) + st["delta"] @ lm
    y_lm = st["H"].T @ om + st["delta"] * b - v
    y_y = -g * rho * df[0] + g * eta
    return np.concatenate([y_om, [y_b], y_lm, y_y])


def jacobian(x, st, prob, fun, gauss_newton=False):
    """Dense symmetric Jacobian dY/dx of size r + 1 + p + |I|."""
    om, b, lm, y = unpack(x, st)
    rho, eta, _, df, d2f, q = _state(x, st, fun)
    g = float(prob["gamma"])
    r, p = st["r"], st["p"]
    phis = st["phis"]
    ni = y.size
    nz = r + 1 + p
    jac = np.zeros((nz + ni, nz + ni))
    rw = np.zeros_like(rho) if gauss_newton else rho
    a_om = np.eye(r) + g * q.T @ q + g * phis[0].T @ phis[0]
    for a in range(1, p):
        for c in range(1, p):
            a_om -= g * phis[a].T @ ((rw * d2f[a][c])[:, None] * phis[c])
    jac[:r, :r] = a_om
    jac[:r, r] = g * phis[0].sum(axis=0)
    jac[:r, r + 1:nz] = st["H"]
    jac[r, r] = g * ni
    jac[r, r + 1:nz] = st["delta"]
    cy = df[0][:, None] * q + phis[0]
    for a in range(1, p):
        cy = cy + (rw * d2f[0][a])[:, None] * phis[a]
    jac[:r, nz:] = -g * cy.T
    jac[r, nz:] = -g
    jac[nz:, nz:] = np.diag(g * (1.0 + df[0] ** 2 - rw * d2f[0][0]))
    jac[nz:, :nz] = jac[:nz, nz:].T
    jac[r + 1:nz, :r + 1] = jac[:r + 1, r + 1:nz].T
    jac[r, :r] = jac[:r, r]
    return jac


def step_dense(x, st, prob, fun, gauss_newton=False):
    dx = np.linalg.solve(jacobian(x, st, prob, fun, gauss_newton), residual(x, st, prob, fun))
    return x - dx, dx


def step_schur(x, st, prob, fun, gauss_newton=False):
    """J = [[A, B], [B^T, D]], D diagonal: (A - B D^-1 B^T) dz = Y_z - B D^-1 Y_y,
    dy = D^-1 (Y_y - B^T dz)."""
    nz = st["r"] + 1 + st["p"]
    jac = jacobian(x, st, prob, fun, gauss_newton)
    yv = residual(x, st, prob, fun)
    a, bm, dg = jac[:nz, :nz], jac[:nz, nz:], np.diag(jac[nz:, nz:])
    dz = np.linalg.solve(a - (bm / dg[None, :]) @ bm.T, yv[:nz] - bm @ (yv[nz:] / dg))
    dy = (yv[nz:] - bm.T @ dz) / dg
    dx = np.concatenate([dz, dy])
    return x - dx, dx


def initial_state(st, prob):
    """omega = 0, lam = 0, b = y_i = the first value condition (d = 0), or 0 without one."""
    vals = [float(v) for d, v in zip(prob["cond_d"], np.asarray(prob["v"]).ravel()) if int(d) == 0]
    b = vals[0] if vals else 0.0
    x = np.zeros(st["r"] + 1 + st["p"] + st["idx"].size)
    x[st["r"]] = b
    x[st["r"] + 1 + st["p"]:] = b
    return x


def solve(prob, fun, tol=1e-12, max_iter=30, schur=False, gauss_newton_steps=0):
    """Newton iteration to |dx|_inf <= tol max(1, |x|_inf) or max_iter steps; the first
    `gauss_newton_steps` steps use the Gauss-Newton Jacobian.  Returns the setup dict with
    x, steps (|dx|_inf per step), iterates, omega, b, alpha and y_hat on the grid."""
    st = setup(prob)
    x = initial_state(st, prob)
    steps, xs = [], [x.copy()]
    for k in range(max_iter):
        step = step_schur if schur else step_dense
        x, dx = step(x, st, prob, fun, gauss_newton=k < gauss_newton_steps)
        xs.append(x.copy())
        steps.append(float(np.max(np.abs(dx))))
        if steps[-1] <= tol * max(1.0, float(np.max(np.abs(x)))):
            break
    om, b, lm, y = unpack(x, st)
    alpha = st["W"] @ om
    yhat = nystrom.kvec(0, st["t"], st["t_land"], prob["sigma"]) @ alpha + b
    st.update(x=x, iterates=xs, steps=steps, iters=len(steps), omega=om, b=b, lam_kkt=lm,
              y=y, alpha=alpha, yhat=yhat)
    return st
