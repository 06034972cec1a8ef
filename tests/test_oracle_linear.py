"""Pins for oracle.linear (Lemma 1, Sec. 3.1 / App. A.3-A.4) against values and identities
that do not come from the oracle itself."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2510_04094_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_problems.json")
W7 = np.sqrt(1 - 0.0225)
B12 = (np.cos(1.0) - 2.0) / np.sin(1.0)

# Closed forms of the paper's benchmark problems (appendix problem list), in the
# paper's convention y^(p) = sum_k f_k y^(p-k) + r.  (f_k list, r, conditions, exact y)
CLOSED = {
    2: ([lambda t: -np.ones_like(t)], lambda t: 0 * t, [(0, 0, 1.0)], lambda t: np.exp(-t)),
    3: ([lambda t: -1e3 * np.ones_like(t)], lambda t: 1e3 * np.sin(t) + np.cos(t), [(0, 0, 0.0)], np.sin),
    7: ([lambda t: -0.3 * np.ones_like(t), lambda t: -np.ones_like(t)], lambda t: np.ones_like(t),
        [(0, 0, 0.0), (1, 0, 0.0)],
        lambda t: 1 - np.exp(-0.15 * t) * (np.cos(W7 * t) + 0.15 / W7 * np.sin(W7 * t))),
    8: ([lambda t: 0 * t, lambda t: -36 * np.ones_like(t)], lambda t: 0 * t, [(0, 0, -0.5), (1, 0, 1.0)],
        lambda t: -0.5 * np.cos(6 * t) + np.sin(6 * t) / 6),
    9: ([lambda t: -4 * np.ones_like(t), lambda t: -4 * np.ones_like(t)], lambda t: 0 * t,
        [(0, 0, 1.0), (1, 0, 1.0)], lambda t: (1 + 3 * t) * np.exp(-2 * t)),
    10: ([lambda t: -0.2 * np.ones_like(t), lambda t: -np.ones_like(t)],
         lambda t: -0.2 * np.exp(-t / 5) * np.cos(t), [(0, 0, 0.0), (1, 0, 1.0)],
         lambda t: np.exp(-t / 5) * np.sin(t)),
    12: ([lambda t: 0 * t, lambda t: -np.ones_like(t)], lambda t: 2 * np.ones_like(t),
         [(0, 0, 1.0), (0, -1, 0.0)], lambda t: 2 - np.cos(t) + B12 * np.sin(t)),
    16: ([lambda t: 0 * t] * 4, lambda t: 120 * t, [(0, 0, 1.0), (1, 0, 5.0), (0, -1, 3.0), (1, -1, 5.0)],
         lambda t: t ** 5 + 2),
}


def paper_problem(entry, tau):
    fk, rf, conds, exact = CLOSED[entry["id"]]
    n = entry["n"]
    t = np.linspace(entry["domain"][0], entry["domain"][1], n)
    prob = dict(p=entry["p"], n=n, m=entry["m"], t=t, f=np.stack([f(t) for f in fk]), r=rf(t),
                cond_d=[c[0] for c in conds], cond_i=[c[1] % n for c in conds],
                v=np.array([c[2] for c in conds]), sigma=np.sqrt(entry["sigma2"]),
                gamma=entry["gamma"], tau=tau, lidx=None)
    return prob, exact(t)


@pytest.mark.parametrize("entry", json.load(open(GOLDEN))["problems"], ids=lambda e: "problem%d" % e["id"])
def test_paper_benchmark_accuracy(entry):
    """With the paper's own n, m, sigma^2, gamma the solution is as accurate as the paper reports."""
    prob, exact = paper_problem(entry, tau=1e-16)
    sol = oracle.linear.solve(prob)
    mae = np.mean(np.abs(sol["yhat"] - exact))
    assert mae <= 10 * entry["mae"], (mae, entry["mae"])


def test_initial_conditions_hold_exactly():
    prob = workloads.linear_second_order(3, n=1500)
    sol = oracle.linear.solve(prob)
    y0 = oracle.linear.predict(sol, [0.0], prob["sigma"], 0)[0]
    dy0 = oracle.linear.predict(sol, [0.0], prob["sigma"], 1)[0]
    assert abs(y0 - prob["v"][0]) < 1e-12 * max(1, abs(prob["v"][0]))
    assert abs(dy0 - prob["v"][1]) < 1e-10 * max(1, abs(prob["v"][1]))


def test_boundary_conditions_hold_exactly():
    prob, _ = paper_problem(json.load(open(GOLDEN))["problems"][6], tau=1e-14)   # problem 12, BVP
    sol = oracle.linear.solve(prob)
    assert abs(sol["yhat"][0] - 1.0) < 1e-9
    assert abs(sol["yhat"][-1] - 0.0) < 1e-9


def nullspace_solution(sol, prob):
    """Brute force: minimise 1/2|omega|^2 + gamma/2 |G omega + c b - r|^2 subject to the
    conditions by parametrising the constraint set (null-space method, QR least squares)."""
    r = sol["r"]
    g, c, rr = sol["G"], sol["c"], sol["rvec"]
    ct = np.vstack([sol["H"], sol["delta"][None, :]]).T          # p x (r+1): conditions on (omega, b)
    v = np.asarray(prob["v"], dtype=np.float64)
    xp = np.linalg.lstsq(ct, v, rcond=None)[0]
    nsp = scipy.linalg.null_space(ct)
    dmat = np.diag(np.r_[np.ones(r), 0.0])
    mmat = np.hstack([g, c[:, None]])
    gam = np.sqrt(prob["gamma"])
    lhs = np.vstack([dmat @ nsp, gam * mmat @ nsp])
    rhs = np.concatenate([-dmat @ xp, gam * (rr - mmat @ xp)])
    z = scipy.linalg.lstsq(lhs, rhs)[0]
    return xp + nsp @ z


@pytest.mark.parametrize("maker", [
    lambda: workloads.linear_first_order(5, n=120, m=15),
    lambda: workloads.linear_second_order(4, n=300, m=20, gamma=1e4, tau=1e-10),
    lambda: dict(workloads.linear_first_order(5, n=150, m=18, gamma=1e5),
                 lidx=workloads.random_landmarks(5, 150, 18)),
    lambda: dict(workloads.linear_second_order(6, n=300, m=20, gamma=1e4, tau=1e-10),
                 lidx=workloads.random_landmarks(6, 300, 20, ends=False)),
])
def test_kkt_solution_equals_nullspace_least_squares(maker):
    prob = maker()
    sol = oracle.linear.solve(prob)
    x = nullspace_solution(sol, prob)
    r = sol["r"]
    yb = oracle.nystrom.kvec(0, prob["t"], sol["t_land"], prob["sigma"]) @ (sol["W"] @ x[:r]) + x[r]
    np.testing.assert_allclose(sol["yhat"], yb, atol=1e-8 * np.max(np.abs(yb)))


@pytest.mark.parametrize("maker", [
    lambda: workloads.linear_first_order(7, n=100, m=12, gamma=1e4),
    lambda: workloads.linear_second_order(8, n=160, m=16, gamma=1e5, tau=1e-10),
    lambda: dict(workloads.linear_first_order(9, n=100, m=12, gamma=1e4),
                 lidx=workloads.random_landmarks(9, 100, 12, ends=False)),
])
def test_primal_equals_dual_with_nystrom_kernel(maker):
    """Strong duality: Lemma 1's primal and the dual LS-SVM with kernel k_m^T W W^T k_m agree.
    (Moderate gamma: the dual's I/gamma diagonal is its only regularisation.)"""
    prob = maker()
    sol = oracle.linear.solve(prob)
    dsol = oracle.dual.solve(prob, oracle.dual.nystrom_kernel(sol["t_land"], prob["sigma"], sol["W"]))
    yd = dsol["predict"](prob["t"])
    np.testing.assert_allclose(sol["yhat"], yd, atol=1e-8 * np.max(np.abs(yd)))
    tq = np.linspace(prob["t"][0], prob["t"][-1], 37)
    np.testing.assert_allclose(oracle.linear.predict(sol, tq, prob["sigma"], 1), dsol["predict"](tq, 1),
                               atol=1e-7 * np.max(np.abs(dsol["predict"](tq, 1))))


def test_close_to_classical_lssvm():
    """The classical dual LS-SVM with the exact RBF kernel solves the same ODE; with m = n/2
    landmarks the two solutions are close (the paper reports well below 1% difference)."""
    prob = workloads.linear_first_order(2, n=120, m=60)
    sol = oracle.linear.solve(prob)
    csol = oracle.dual.solve(prob, oracle.dual.rbf_kernel(prob["sigma"]))
    yc = csol["predict"](prob["t"])
    assert np.max(np.abs(sol["yhat"] - yc)) < 1e-3 * np.max(np.abs(yc))


def test_manufactured_first_order_accuracy():
    errs = []
    for i in range(8):
        prob = workloads.linear_first_order(i)
        sol = oracle.linear.solve(prob)
        errs.append(np.max(np.abs(sol["yhat"] - prob["ystar"])) / np.max(np.abs(prob["ystar"])))
    assert np.median(errs) < 1e-2 and max(errs) < 5e-2


def test_random_landmarks_manufactured_accuracy():
    """Random landmark sets (m = 40 of n = 200 grid points, end points kept) reproduce the
    manufactured solution about as well as 40 equidistant landmarks (1e-6 .. 1.5e-5 with
    these seeds), and the given indices are the ones used.  (With m = 20 the random gaps
    reach 50 grid points = 2.6 sigma and the error grows to several percent.)"""
    errs = []
    for i in range(8):
        prob = workloads.linear_first_order(i, m=40)
        prob["lidx"] = workloads.random_landmarks(i, prob["n"], prob["m"])
        sol = oracle.linear.solve(prob)
        np.testing.assert_array_equal(sol["t_land"], prob["t"][prob["lidx"]])
        errs.append(np.max(np.abs(sol["yhat"] - prob["ystar"])) / np.max(np.abs(prob["ystar"])))
    assert np.median(errs) < 1e-5 and max(errs) < 1e-4


def test_kkt_matrix_is_symmetric():
    sol = oracle.linear.assemble(workloads.linear_second_order(1, n=500))
    np.testing.assert_allclose(sol["A"], sol["A"].T, rtol=1e-13, atol=1e-13 * np.max(np.abs(sol["A"])))
