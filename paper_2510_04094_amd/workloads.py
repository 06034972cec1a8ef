"""Seeded synthetic ODE workloads (manufactured solutions).

This module only draws problem instances: a grid, coefficient functions, a
manufactured solution y* and the forcing / conditions that make y* exact.
It contains none of the solver's arithmetic and imports nothing else from the
package, so the HIP binding and the CPU oracle can both consume its output.

Every instance is a plain dict:
  p, n, m            ODE order, grid size, number of landmarks
  t0, dt, t          uniform grid t_i = t0 + i*dt (t is the float64 array)
  f                  [p, n] coefficients f_k(t_i) of y^(p) = sum_k f_k y^(p-k) + r
  r                  [n] forcing r(t_i)
  cond_d, cond_i, v  conditions y^(d_j)(t_{i_j}) = v_j
  sigma, gamma, tau  RBF bandwidth (K = exp(-(u-v)^2/sigma^2)), ridge, eigen cut-off
  ystar              [n] manufactured solution on the grid (for accuracy reports)
  lidx               None: landmarks follow the solver's default equidistant rule
Nonlinear (Riccati) instances carry `q` [n] with y' = q(t) - y^2 instead of f/r.

Seeds: numpy.random.default_rng(251004094 + 100000*config + instance); draws
in the order bandwidth, coefficients, solution parameters, noise.
"""
import numpy as np

SEED_BASE = 251004094


def _rng(config, instance):
    return np.random.default_rng(SEED_BASE + 100000 * config + instance)


def _grid(t_end, n):
    dt = t_end / (n - 1)
    return 0.0, dt, 0.0 + np.arange(n, dtype=np.float64) * dt


def _sines(rng, k, t, damp=0.0):
    """y*, y*', y*'' of exp(-damp t) sum_k c_k sin(w_k t + ph_k)."""
    c = rng.uniform(-1.0, 1.0, k)
    w = rng.uniform(1.0, 6.0, k)
    ph = rng.uniform(0.0, 2.0 * np.pi, k)
    arg = w[None, :] * t[:, None] + ph[None, :]
    s = np.sin(arg) @ c
    ds = (np.cos(arg) * w[None, :]) @ c
    dds = (-np.sin(arg) * (w * w)[None, :]) @ c
    e = np.exp(-damp * t)
    y = e * s
    dy = e * (ds - damp * s)
    ddy = e * (dds - 2.0 * damp * ds + damp * damp * s)
    return y, dy, ddy, dict(c=c, w=w, ph=ph, damp=damp)


def ystar_at(prob, s):
    """Manufactured solution of a linear instance at arbitrary times s."""
    sp = prob["sol"]
    s = np.asarray(s, dtype=np.float64)
    arg = sp["w"][None, :] * s[:, None] + sp["ph"][None, :]
    return np.exp(-sp["damp"] * s) * (np.sin(arg) @ sp["c"])


def random_landmarks(instance, n, m, ends=True, config=6):
    """m strictly ascending grid indices drawn uniformly without replacement (the random
    landmark variant of the Nystrom basis, Sec. 3); with `ends` the first and last grid
    points are always landmarks."""
    rng = _rng(config, instance)
    if ends:
        inner = rng.choice(np.arange(1, n - 1), size=m - 2, replace=False)
        idx = np.concatenate([[0], np.sort(inner), [n - 1]])
    else:
        idx = np.sort(rng.choice(n, size=m, replace=False))
    return idx.astype(np.int64)


def leverage_uniforms(instance, n, config=9):
    """n uniforms in (0, 1] for the exponential keys of leverage-score landmark sampling (the
    random numbers that sampling draws, handed to both the library and the oracle)."""
    return 1.0 - _rng(config, instance).random(n)


def linear_first_order(instance, n=200, m=20, t_end=1.0, sigma=0.1, gamma=1e8,
                       tau=1e-12, config=1):
    """y' + a(t) y = g(t), y(0) = y*(0); a = a0 + a1 cos t, a ~ U(.5, 2); y* = 3 sinusoids."""
    rng = _rng(config, instance)
    t0, dt, t = _grid(t_end, n)
    a01 = rng.uniform(0.5, 2.0, 2)
    a = a01[0] + a01[1] * np.cos(t)
    y, dy, _, sp = _sines(rng, 3, t)
    g = dy + a * y
    return dict(p=1, n=n, m=m, t0=t0, dt=dt, t=t, f=(-a)[None, :].copy(), r=g,
                cond_d=[0], cond_i=[0], v=np.array([y[0]]), sigma=float(sigma),
                gamma=float(gamma), tau=float(tau), ystar=y, lidx=None,
                coef=dict(alpha=a01), sol=sp)


def linear_second_order(instance, n=10000, m=50, t_end=10.0, gamma=1e7, tau=1e-8,
                        sigma=None, config=2, obs=0, noise=1e-3):
    """y'' + b(t) y' + a(t) y = g(t) with y(0), y'(0) from y*.

    sigma ~ U(0.2, 1); a = a0 + a1 cos t, a ~ U(.5, 2); b = b0 + b1 sin t,
    b ~ U(0, .5); y* = exp(-lam t) * (5 sinusoids), lam ~ U(0, .3).
    With obs > 0 the same stream then draws `obs` sorted observation times
    s_j ~ U(t0, t_end) and y_obs = y*(s_j) + noise * N(0, 1) (keys t_obs, y_obs).
    """
    rng = _rng(config, instance)
    s_draw = rng.uniform(0.2, 1.0)
    sig = s_draw if sigma is None else sigma
    t0, dt, t = _grid(t_end, n)
    a01 = rng.uniform(0.5, 2.0, 2)
    b01 = rng.uniform(0.0, 0.5, 2)
    a = a01[0] + a01[1] * np.cos(t)
    bb = b01[0] + b01[1] * np.sin(t)
    lam = rng.uniform(0.0, 0.3)
    y, dy, ddy, sp = _sines(rng, 5, t, damp=lam)
    g = ddy + bb * dy + a * y
    f = np.stack([-bb, -a])
    prob = dict(p=2, n=n, m=m, t0=t0, dt=dt, t=t, f=f, r=g, cond_d=[0, 1],
                cond_i=[0, 0], v=np.array([y[0], dy[0]]), sigma=float(sig),
                gamma=float(gamma), tau=float(tau), ystar=y, lidx=None,
                coef=dict(alpha=a01, beta=b01, damp=lam), sol=sp)
    if obs > 0:
        s = np.sort(rng.uniform(t0, t0 + (n - 1) * dt, obs))
        prob["t_obs"] = s
        prob["y_obs"] = ystar_at(prob, s) + noise * rng.standard_normal(obs)
    return prob


def linear_order_p(instance, p, n=2000, m=30, t_end=2.0, sigma=0.3, gamma=1e7, tau=1e-8,
                   bvp=False, config=7):
    """y^(p) = sum_k f_k(t) y^(p-k) + g(t) of any order p = 1..4 with a manufactured y*.

    f_k = c_k0 + c_k1 cos t with c ~ U(-0.5, 0.5); y* = sum of 3 sinusoids (amplitude U(-1, 1),
    frequency U(1, 3), phase U(0, 2 pi)).  IVP: y^(d)(t_0) = y*^(d)(t_0) for d < p.  With
    `bvp` the conditions are split over both ends: y^(d)(t_0) for d < ceil(p/2) and
    y^(d)(t_end) for d < floor(p/2) (for p = 4 the clamped-beam form of the paper's
    fourth-order boundary problem)."""
    rng = _rng(config, instance)
    t0, dt, t = _grid(t_end, n)
    cf = rng.uniform(-0.5, 0.5, (p, 2))
    f = cf[:, :1] + cf[:, 1:] * np.cos(t)[None, :]
    amp = rng.uniform(-1.0, 1.0, 3)
    w = rng.uniform(1.0, 3.0, 3)
    ph = rng.uniform(0.0, 2.0 * np.pi, 3)

    def deriv(k, tt):
        arg = w[None, :] * tt[:, None] + ph[None, :] + 0.5 * np.pi * k
        return np.sin(arg) @ (amp * w ** k)

    ys = [deriv(k, t) for k in range(p + 1)]
    g = ys[p] - sum(f[k - 1] * ys[p - k] for k in range(1, p + 1))
    if bvp:
        conds = [(d, 0) for d in range((p + 1) // 2)] + [(d, n - 1) for d in range(p // 2)]
    else:
        conds = [(d, 0) for d in range(p)]
    v = np.array([ys[d][i] for d, i in conds])
    return dict(p=p, n=n, m=m, t0=t0, dt=dt, t=t, f=f, r=g, cond_d=[c[0] for c in conds],
                cond_i=[c[1] for c in conds], v=v, sigma=float(sigma), gamma=float(gamma),
                tau=float(tau), ystar=ys[0], lidx=None, coef=dict(c=cf),
                sol=dict(c=amp, w=w, ph=ph, damp=0.0))


def riccati(instance, n=2000, m=50, t_end=2.0, sigma=0.1, gamma=1e6, tau=1e-12,
            config=3):
    """y' = q(t) - y^2 with y* = 0.5 + 0.3 tanh(kappa (t - 1)), kappa ~ U(1, 4)."""
    rng = _rng(config, instance)
    t0, dt, t = _grid(t_end, n)
    kappa = rng.uniform(1.0, 4.0)
    th = np.tanh(kappa * (t - 1.0))
    y = 0.5 + 0.3 * th
    dy = 0.3 * kappa * (1.0 - th * th)
    q = dy + y * y
    return dict(p=1, n=n, m=m, t0=t0, dt=dt, t=t, q=q, cond_d=[0], cond_i=[0],
                v=np.array([y[0]]), sigma=float(sigma), gamma=float(gamma),
                tau=float(tau), ystar=y, lidx=None, coef=dict(kappa=kappa))


def nonlinear_second_order(instance, n=1000, m=20, t_end=2.0, sigma=0.6, gamma=1e7, tau=1e-12,
                           bvp=False, config=8):
    """y'' = q(t) - c1 y - c2 y^3 - c3 (y')^2 with c ~ U(0.2, 1) and the manufactured
    y* = 0.5 + 0.3 sin(w t + ph), w ~ U(1, 3), ph ~ U(0, 2 pi) (q makes y* exact).  The
    conditions are y(t_0), y'(t_0); with `bvp`, y(t_0), y(t_end) (a two-point problem like
    the paper's nonlinear problems 14 and 15; such problems can have several solutions, and
    Newton from a constant start may find another one than y*).  The instance carries `q` and the
    coefficients `c` instead of f / r; F and its partial derivatives in (y, y') are
    nonlinear_second_order_rhs(prob, y, yp)."""
    rng = _rng(config, instance)
    t0, dt, t = _grid(t_end, n)
    c = rng.uniform(0.2, 1.0, 3)
    w = rng.uniform(1.0, 3.0)
    ph = rng.uniform(0.0, 2.0 * np.pi)
    y = 0.5 + 0.3 * np.sin(w * t + ph)
    dy = 0.3 * w * np.cos(w * t + ph)
    ddy = -0.3 * w * w * np.sin(w * t + ph)
    q = ddy + c[0] * y + c[1] * y ** 3 + c[2] * dy * dy
    if bvp:
        cond_d, cond_i, v = [0, 0], [0, n - 1], np.array([y[0], y[-1]])
    else:
        cond_d, cond_i, v = [0, 1], [0, 0], np.array([y[0], dy[0]])
    return dict(p=2, n=n, m=m, t0=t0, dt=dt, t=t, q=q, c=c, cond_d=cond_d, cond_i=cond_i, v=v,
                sigma=float(sigma), gamma=float(gamma), tau=float(tau), ystar=y, lidx=None,
                coef=dict(c=c, w=w, ph=ph))


def nonlinear_second_order_rhs(prob, y, yp, idx=None):
    """F(t_i, y, y') of a nonlinear_second_order instance and its partial derivatives in
    (y, y'): returns (F, [F_y, F_y'], [[F_yy, F_yy'], [F_y'y, F_y'y']]) (array module of y:
    numpy or torch)."""
    c = prob["c"]
    q = prob["q"] if idx is None else prob["q"][idx]
    zero = 0 * y
    return (q - c[0] * y - c[1] * y ** 3 - c[2] * yp * yp,
            [-c[0] - 3 * c[1] * y * y, -2 * c[2] * yp],
            [[-6 * c[1] * y, zero], [zero, zero - 2 * c[2]]])


def _mixed_params(count, n_lo, n_hi, ms, config):
    rng = _rng(config, 0)
    orders = np.array([1] * (count // 2) + [2] * (count - count // 2))
    rng.shuffle(orders)
    ns = rng.integers(n_lo, n_hi + 1, count)
    mm = rng.choice(np.array(ms), count)
    return orders, ns, mm


def mixed_batch_instance(i, count=4096, n_lo=500, n_hi=10000, ms=(20, 50, 100), tau=1e-8,
                         config=4):
    """Instance i of mixed_batch(count, ...) alone."""
    orders, ns, mm = _mixed_params(count, n_lo, n_hi, ms, config)
    if orders[i] == 1:
        return linear_first_order(i + 1, n=int(ns[i]), m=int(mm[i]), tau=tau, config=config)
    return linear_second_order(i + 1, n=int(ns[i]), m=int(mm[i]), tau=tau, config=config)


def mixed_batch(count=4096, n_lo=500, n_hi=10000, ms=(20, 50, 100), tau=1e-8, config=4):
    """Uneven batch: p in {1, 2} (exactly half each, shuffled), n ~ U{n_lo..n_hi}, m from ms."""
    orders, ns, mm = _mixed_params(count, n_lo, n_hi, ms, config)
    out = []
    for i in range(count):
        if orders[i] == 1:
            prob = linear_first_order(i + 1, n=int(ns[i]), m=int(mm[i]), tau=tau,
                                      config=config)
        else:
            prob = linear_second_order(i + 1, n=int(ns[i]), m=int(mm[i]), tau=tau,
                                       config=config)
        out.append(prob)
    return out


def adjoint_batch(count=1024, n=5000, m=50, obs=100, config=5):
    """Second-order instances with observations for the parameter-estimation loss."""
    return [linear_second_order(i, n=n, m=m, config=config, obs=obs) for i in range(count)]
