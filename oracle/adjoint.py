"""Gradient of a loss on y_hat through the Lemma 1 solve (oracle).

The paper has no adjoint; this is the derivative of the Lemma 1 solution
(Sec. 3.1, App. A.3/A.4) taken by the adjoint method, written from the KKT
conditions.  Notation as in oracle.linear: x = (omega, b, lam) solves A x = rhs,
A symmetric; alpha = W omega; e_i = p_i^T alpha + c_i b - r_i (the ODE residual
of y_hat at t_i).

For l = loss(y_hat(s_1..s_J)) with g_j = dl/dy_hat(s_j):
  1. x_bar = (W^T kbar, sum_j g_j, 0) with kbar = sum_j g_j k_m(s_j);  mu = A^{-1} x_bar.
  2. beta = W mu_omega;  nu_i = beta^T p_i + mu_b c_i;
     yh^(d)_i = alpha^T k^(d)_i + [d=0] b;  zh^(d)_i = beta^T k^(d)_i + [d=0] mu_b.
  3. dl/df_{k,i} = gamma (e_i zh^(p-k)_i + nu_i yh^(p-k)_i)      (i in I, zero elsewhere)
     dl/dr_i     = gamma nu_i
     dl/dv_j     = mu_lam_j
     dl/dgamma   = -sum_i nu_i e_i = mu_omega^T omega / gamma.
     The second form follows from the KKT conditions: the first two block rows of
     A x = rhs say gamma G^T e = -(omega + H lam) and gamma c^T e = -delta^T lam, and the
     last block row of A mu = x_bar says H^T mu_omega + delta mu_b = 0, so
     sum_i nu_i e_i = mu_omega^T G^T e + mu_b c^T e = -mu_omega^T omega / gamma.  At large
     gamma the residuals e_i are tiny and the sum over the points cancels by orders of
     magnitude, so the product of the two small vectors is the one evaluated (the sum is
     kept as dl_dgamma_direct).
  4. sigma enters through k^(d)(.) at fixed W (closed form d/dsigma of the
     kernel derivatives) and through W.  The problem depends on W only via
     Q = W W^T = f(K_mm), f(lam) = 1/lam above the cut-off and 0 below, so the
     K_mm part is the Daleckii-Krein formula dQ = U (F o (U^T dK U)) U^T with
     F_kl = (f(l_k) - f(l_l)) / (l_k - l_l), F_kk = f'(l_k).
The signs of lam and mu_lam follow the Lagrangian with +lam (Sec. 3.1).
"""
import numpy as np

from . import linear, nystrom, rbf


def grad(prob, t_obs, g_obs):
    """Return dict of dl/df [p, n], dl/dr [n], dl/dv [p], dl/dsigma, dl/dgamma and the solution."""
    p = int(prob["p"])
    sig = float(prob["sigma"])
    gam = float(prob["gamma"])
    t = np.asarray(prob["t"], dtype=np.float64)
    f = np.asarray(prob["f"], dtype=np.float64).reshape(p, -1)
    n = t.size
    sol = linear.solve(prob)
    r, w, u, lam = sol["r"], sol["W"], sol["U"], sol["lam"]
    t_land, idx = sol["t_land"], sol["idx"]
    t_obs = np.asarray(t_obs, dtype=np.float64)
    g_obs = np.asarray(g_obs, dtype=np.float64)

    # 1. adjoint solve with the same (symmetric) matrix
    k_obs = nystrom.kvec(0, t_obs, t_land, sig)            # J x m
    kbar = k_obs.T @ g_obs
    xbar = np.zeros(r + 1 + p)
    xbar[:r] = w.T @ kbar
    xbar[r] = np.sum(g_obs)
    mu = np.linalg.solve(sol["A"], xbar)
    mu_w, mu_b, mu_l = mu[:r], mu[r], mu[r + 1:]
    alpha, b = sol["alpha"], sol["b"]
    beta = w @ mu_w

    # 2. per-point quantities over the residual set
    ti = t[idx]
    kd = [nystrom.kvec(d, ti, t_land, sig) for d in range(p + 1)]
    pk = sol["P"]
    c, rr = sol["c"], sol["rvec"]
    e = pk @ alpha + c * b - rr
    nu = pk @ beta + c * mu_b
    yh = [kd[d] @ alpha + (b if d == 0 else 0.0) for d in range(p + 1)]
    zh = [kd[d] @ beta + (mu_b if d == 0 else 0.0) for d in range(p + 1)]

    # 3. coefficient, forcing, condition and gamma gradients
    dl_df = np.zeros((p, n))
    for k in range(1, p + 1):
        dl_df[k - 1, idx] = gam * (e * zh[p - k] + nu * yh[p - k])
    dl_dr = np.zeros(n)
    dl_dr[idx] = gam * nu
    dl_dv = mu_l.copy()
    dl_dgamma_direct = -float(np.sum(nu * e))
    dl_dgamma = float(mu_w @ sol["omega"]) / gam

    # 4a. sigma at fixed W: observation kernel, operator rows, condition rows
    dks = [nystrom_dsigma(d, ti, t_land, sig) for d in range(p + 1)]
    dpk = dks[p].copy()
    for k in range(1, p + 1):
        dpk = dpk - f[k - 1, idx][:, None] * dks[p - k]
    term_obs = float(g_obs @ (nystrom_dsigma(0, t_obs, t_land, sig) @ alpha))
    term_pts = -gam * float(np.sum((e[:, None] * beta[None, :] + nu[:, None] * alpha[None, :]) * dpk))
    term_cond = 0.0
    lam_kkt = sol["lam_kkt"]
    hk = []
    for j, (d, i) in enumerate(zip(prob["cond_d"], prob["cond_i"])):
        dh = nystrom_dsigma(int(d), t[int(i)], t_land, sig)[0]
        term_cond -= float((lam_kkt[j] * beta + mu_l[j] * alpha) @ dh)
        hk.append(nystrom.kvec(int(d), t[int(i)], t_land, sig)[0])
    direct = term_obs + term_pts + term_cond
    hk = np.stack(hk, axis=1)                               # m x p, kernel space

    # 4b. sigma through K_mm: dl/dW, then Q_bar, then Daleckii-Krein
    om = sol["omega"]
    a_e = pk.T @ e
    a_nu = pk.T @ nu
    g_w = (np.outer(kbar, om) - gam * np.outer(a_e, mu_w) - gam * np.outer(a_nu, om)
           - hk @ (np.outer(lam_kkt, mu_w) + np.outer(mu_l, om)))
    m = lam.size
    qbar_u = np.zeros((m, m))
    qbar_u[:, :r] = 0.5 * (u.T @ g_w) * np.sqrt(lam[:r])[None, :]
    qbar_u[:r, r:] = qbar_u[r:, :r].T
    fval = np.zeros(m)
    fval[:r] = 1.0 / lam[:r]
    fmat = np.zeros((m, m))
    for k in range(m):
        for l in range(m):
            if k < r or l < r:
                if k == l:
                    fmat[k, l] = -1.0 / lam[k] ** 2
                elif lam[k] != lam[l]:
                    fmat[k, l] = (fval[k] - fval[l]) / (lam[k] - lam[l])
                else:
                    fmat[k, l] = -1.0 / lam[min(k, l)] ** 2
    kbar_mm = u @ (fmat * qbar_u) @ u.T
    dkmm = rbf.kernel_du_dsigma(0, t_land[:, None], t_land[None, :], sig)
    via_kmm = float(np.sum(kbar_mm * dkmm))
    dl_dsigma = direct + via_kmm

    return dict(dl_df=dl_df, dl_dr=dl_dr, dl_dv=dl_dv, dl_dsigma=dl_dsigma,
                dl_dgamma=dl_dgamma, dl_dgamma_direct=dl_dgamma_direct, sol=sol, mu=mu, e=e, nu=nu,
                sigma_direct=direct, sigma_kmm=via_kmm,
                sigma_terms=np.array([term_obs, term_pts, term_cond, via_kmm]))


def nystrom_dsigma(d, t, t_land, sigma):
    """d/dsigma of d^d/dt^d k_m(t); shape (len(t), m)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return rbf.kernel_du_dsigma(d, t[:, None], np.asarray(t_land)[None, :], sigma)
