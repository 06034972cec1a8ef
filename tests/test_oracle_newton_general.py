"""Pins for oracle.newton_general (Lemma 2 for y^(p) = F(t, y, ..., y^(p-1)), Sec. 3.2 and the
Problem 15 appendix) against derivatives taken independently of its formulas, the
first-order oracle, and the closed-form solutions of the paper's nonlinear second-order
boundary problems 14 and 15."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import newton_general as ng
from paper_2510_04094_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_problems.json")
GN_STEPS = 5  # Gauss-Newton steps before Newton from the constant start


def p14(idx, y, u):
    """Problem 14: y'' = -(y')^2 + 2 exp(-y)."""
    e = np.exp(-y)
    yp = u[0]
    return (-yp * yp + 2 * e, [-2 * e, -2 * yp],
            [[2 * e, 0 * y], [0 * y, -2 + 0 * y]])


def p15(idx, y, u):
    """Problem 15: y'' = -y + 2 (y')^2 / y."""
    yp = u[0]
    return (-y + 2 * yp * yp / y, [-1 - 2 * yp * yp / (y * y), 4 * yp / y],
            [[4 * yp * yp / y ** 3, -4 * yp / (y * y)], [-4 * yp / (y * y), 4 / y]])


CLOSED = {14: (p14, [(0, 0, 0.0), (0, -1, 0.0)], lambda t: np.log(t * t - t + 1)),
          15: (p15, [(0, 0, 0.324027137), (0, -1, 0.324027137)], lambda t: 0.5 / np.cosh(t))}


def paper_nonlinear(entry, tau=1e-12):
    fun, conds, exact = CLOSED[entry["id"]]
    n = entry["n"]
    t = np.linspace(entry["domain"][0], entry["domain"][1], n)
    prob = dict(p=2, n=n, m=entry["m"], t=t, cond_d=[c[0] for c in conds],
                cond_i=[c[1] % n for c in conds], v=np.array([c[2] for c in conds]),
                sigma=np.sqrt(entry["sigma2"]), gamma=entry["gamma"], tau=tau, lidx=None)
    return prob, fun, exact(t)


def entries():
    return json.load(open(GOLDEN))["nonlinear"]


def small_problem(which=15, n=40, m=8):
    entry = dict([e for e in entries() if e["id"] == which][0])
    entry.update(n=n, m=m)
    return paper_nonlinear(entry)


def perturbed_state(st, prob, seed=0):
    x = ng.initial_state(st, prob)
    rng = np.random.default_rng(seed)
    x = x + 0.05 * rng.standard_normal(x.size)
    return x


@pytest.mark.parametrize("which", [14, 15])
def test_residual_is_the_gradient_of_the_lagrangian(which):
    """Y = grad L, by complex-step differentiation of the Lagrangian (exact to rounding)."""
    prob, fun, _ = small_problem(which)
    st = ng.setup(prob)
    x = perturbed_state(st, prob)
    if which == 15:
        x[st["r"] + 1 + st["p"]:] = 0.4  # keep y away from 0 (F has 1/y)
    y = ng.residual(x, st, prob, fun)
    h = 1e-30
    g = np.array([np.imag(ng.lagrangian(x + 1j * h * e, st, prob, fun)) / h for e in np.eye(x.size)])
    np.testing.assert_allclose(y, g, rtol=1e-10, atol=1e-10 * np.max(np.abs(g)))


@pytest.mark.parametrize("which", [14, 15])
def test_jacobian_is_the_derivative_of_the_residual(which):
    prob, fun, _ = small_problem(which)
    st = ng.setup(prob)
    x = perturbed_state(st, prob, seed=1)
    x[st["r"] + 1 + st["p"]:] = np.abs(x[st["r"] + 1 + st["p"]:]) + 0.3
    jac = ng.jacobian(x, st, prob, fun)
    h = 1e-30
    cols = [np.imag(ng.residual(x + 1j * h * e, st, prob, fun)) / h for e in np.eye(x.size)]
    jcs = np.stack(cols, axis=1)
    np.testing.assert_allclose(jac, jcs, rtol=1e-9, atol=1e-9 * np.max(np.abs(jcs)))
    np.testing.assert_allclose(jac, jac.T, rtol=0, atol=1e-13 * np.max(np.abs(jac)))


def test_dense_and_schur_steps_agree():
    """Same step through the dense system and through the Schur complement, compared where
    it is determined well: the change of y_hat on the grid (phi_i^T d omega + d b) and the
    y-block (omega itself is ill-determined: the Jacobian's condition number is ~1e18)."""
    prob, fun, _ = small_problem(15, n=60, m=10)
    st = ng.setup(prob)
    x = ng.initial_state(st, prob)
    r, p = st["r"], st["p"]
    for gn in (True, False):
        _, dd = ng.step_dense(x, st, prob, fun, gauss_newton=gn)
        _, ds = ng.step_schur(x, st, prob, fun, gauss_newton=gn)
        yd = st["phis"][0] @ dd[:r] + dd[r]
        ys = st["phis"][0] @ ds[:r] + ds[r]
        np.testing.assert_allclose(ys, yd, rtol=0, atol=1e-10 * np.max(np.abs(yd)))
        np.testing.assert_allclose(ds[r + 1 + p:], dd[r + 1 + p:], rtol=0,
                                   atol=1e-10 * np.max(np.abs(dd[r + 1 + p:])))


def test_first_order_case_matches_the_first_order_oracle():
    """p = 1 with F(t, y): the same iterates as oracle.newton (App. A.5)."""
    q = workloads.riccati(0, n=300, m=20)
    qq = q["q"]

    def f_first(idx, y):
        return qq[idx] - y * y, -2 * y, -2 + 0 * y

    def f_gen(idx, y, u):
        return qq[idx] - y * y, [-2 * y], [[-2 + 0 * y]]

    a = oracle.newton.solve(q, f_first, max_iter=3, tol=0.0)
    b = ng.solve(q, f_gen, max_iter=3, tol=0.0)
    for xa, xb in zip(a["iterates"], b["iterates"]):
        np.testing.assert_allclose(xb, xa, rtol=0, atol=1e-9 * max(1.0, np.max(np.abs(xa))))


def test_affine_right_hand_side_converges_in_one_step():
    """F affine in (y, y'): L is quadratic, so one Newton step lands on the minimiser."""
    q = workloads.linear_second_order(0, n=400, m=20, t_end=4.0, tau=1e-10)
    f1, f2, rr = q["f"][0], q["f"][1], q["r"]

    def fun(idx, y, u):
        return (f1[idx] * u[0] + f2[idx] * y + rr[idx], [f2[idx], f1[idx]],
                [[0 * y, 0 * y], [0 * y, 0 * y]])

    out = ng.solve(q, fun, max_iter=3, tol=0.0)
    assert out["steps"][1] <= 1e-9 * max(1.0, out["steps"][0])


def test_plain_newton_from_a_constant_start_diverges():
    """Why the iteration starts with Gauss-Newton steps: from y = const, Newton's own
    Jacobian (with the rho_i F'' terms) sends problem 15 far away and never recovers."""
    prob, fun, _ = paper_nonlinear([e for e in entries() if e["id"] == 15][0])
    out = ng.solve(prob, fun, tol=1e-12, max_iter=15, gauss_newton_steps=0)
    assert not out["steps"][-1] <= 1e-6


def test_quadratic_convergence_on_problem_15():
    """After the Gauss-Newton steps, Newton converges quadratically (Sec. 3.2 theorem)."""
    prob, fun, _ = paper_nonlinear([e for e in entries() if e["id"] == 15][0])
    out = ng.solve(prob, fun, tol=1e-12, max_iter=30, gauss_newton_steps=GN_STEPS)
    st, r, p = out, out["r"], out["p"]
    # restart pure Newton from the solution with its y-block perturbed by 1e-2
    x = out["x"].copy()
    x[r + 1 + p:] += 1e-2 * np.sin(np.arange(x.size - r - 1 - p))
    s = []
    for _ in range(4):
        x, dx = ng.step_dense(x, st, prob, fun)
        s.append(float(np.max(np.abs(dx[r + 1 + p:]))))
    # the y-block corrections fall like e_{k+1} <= C e_k^2 until the rounding floor
    # (measured: 1.1e-2, 1.0e-3, 2.5e-6, 4.4e-11, i.e. C ~ 8)
    for k in (1, 2, 3):
        assert s[k] <= max(20 * s[k - 1] ** 2, 1e-12), s


@pytest.mark.parametrize("which", [14, 15])
def test_paper_problem_accuracy(which):
    """With the paper's n, m, sigma^2, gamma the solution is as accurate as the paper reports."""
    entry = [e for e in entries() if e["id"] == which][0]
    prob, fun, exact = paper_nonlinear(entry, tau=1e-16)
    out = ng.solve(prob, fun, tol=1e-12, max_iter=40, gauss_newton_steps=GN_STEPS)
    assert out["steps"][-1] <= 1e-12 * max(1.0, np.max(np.abs(out["x"])))
    mae = np.mean(np.abs(out["yhat"] - exact))
    assert mae <= 10 * entry["mae"], (mae, entry["mae"], out["steps"])


def test_seeded_second_order_family_recovers_its_manufactured_solution():
    """The seeded nonlinear second-order family (y'' = q - c1 y - c2 y^3 - c3 y'^2, initial
    value and slope) converges from the constant start and recovers y*."""
    for k in range(4):
        prob = workloads.nonlinear_second_order(k, n=400)

        def fun(idx, y, u, prob=prob):
            return workloads.nonlinear_second_order_rhs(prob, y, u[0], idx)

        out = ng.solve(prob, fun, tol=1e-12, max_iter=40, gauss_newton_steps=GN_STEPS)
        assert out["steps"][-1] <= 1e-12 * max(1.0, np.max(np.abs(out["x"]))), out["steps"]
        assert np.max(np.abs(out["yhat"] - prob["ystar"])) < 1e-5
