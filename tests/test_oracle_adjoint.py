"""Pins for oracle.adjoint: complex-step and finite differences of the forward oracle solve."""
import numpy as np
import pytest

import oracle
from paper_2510_04094_amd import workloads


def loss_of(prob, t_obs, y_obs):
    sol = oracle.linear.solve(prob)
    yh = oracle.linear.predict(sol, t_obs, prob["sigma"], 0)
    return np.mean((yh - y_obs) ** 2), sol


def setup(p, inst, gamma=None, sigma=None, m=20, tau=1e-10):
    if p == 2:
        prob = workloads.linear_second_order(inst, n=400, m=m, obs=30, config=5, tau=tau,
                                             sigma=sigma, **({} if gamma is None else dict(gamma=gamma)))
    else:
        prob = workloads.linear_first_order(inst, n=150, m=15, **({} if gamma is None else dict(gamma=gamma)))
        rng = np.random.default_rng(inst)
        prob["t_obs"] = np.sort(rng.uniform(0, 1, 25))
        prob["y_obs"] = workloads.ystar_at(prob, prob["t_obs"]) + 1e-3 * rng.standard_normal(25)
    return prob


def gradient(prob):
    ell, sol = loss_of(prob, prob["t_obs"], prob["y_obs"])
    yh = oracle.linear.predict(sol, prob["t_obs"], prob["sigma"], 0)
    g = 2.0 * (yh - prob["y_obs"]) / yh.size
    return oracle.adjoint.grad(prob, prob["t_obs"], g)


def complex_step(prob, key, direction, h=1e-30):
    pc = dict(prob)
    pc[key] = np.asarray(prob[key]) + 1j * h * direction
    ell, _ = loss_of(pc, prob["t_obs"], prob["y_obs"])
    return np.imag(ell) / h


@pytest.mark.parametrize("p,inst", [(1, 0), (2, 0), (2, 3)])
def test_data_gradients_match_complex_step(p, inst):
    prob = setup(p, inst)
    gr = gradient(prob)
    rng = np.random.default_rng(10 + inst)
    for key, gkey in [("f", "dl_df"), ("r", "dl_dr"), ("v", "dl_dv")]:
        d = rng.standard_normal(np.shape(prob[key]))
        ref = complex_step(prob, key, d)
        got = float(np.sum(gr[gkey] * d))
        assert abs(got - ref) <= 1e-7 * abs(ref) + 1e-14, (key, got, ref)


@pytest.mark.parametrize("p,inst,gamma", [(1, 1, 1e3), (2, 1, 1e2), (2, 4, 1e4)])
def test_gamma_gradient_matches_complex_step(p, inst, gamma):
    """At moderate gamma the complex step pins both forms of dl/dgamma: the sum over the
    points -sum nu_i e_i and the KKT identity mu_omega^T omega / gamma."""
    prob = setup(p, inst, gamma=gamma)
    tol = 1e-7
    gr = gradient(prob)
    assert abs(gr["dl_dgamma_direct"] - gr["dl_dgamma"]) <= 1e-7 * abs(gr["dl_dgamma"])
    pc = dict(prob)
    h = 1e-30 * prob["gamma"]
    pc["gamma"] = prob["gamma"] + 1j * h
    ell, _ = loss_of(pc, prob["t_obs"], prob["y_obs"])
    ref = np.imag(ell) / h
    assert abs(gr["dl_dgamma"] - ref) <= tol * abs(ref) + 1e-30


@pytest.mark.parametrize("p,inst,gamma,sigma,m,tau", [
    (1, 2, None, None, 20, 1e-10), (2, 2, None, None, 20, 1e-10), (2, 5, None, None, 20, 1e-10),
    (2, 6, 1.0, None, 20, 1e-10),        # small gamma: the K_mm part matters
    (2, 7, 1.0, 1.0, 40, 1e-6),          # truncated basis (r < m): Daleckii-Krein with dropped pairs
])
def test_sigma_gradient_matches_central_difference(p, inst, gamma, sigma, m, tau):
    """Central difference in sigma.  The truncated case uses a cut-off of 1e-6 so that the
    retained eigenvectors (error ~ eps/gap) are accurate enough for a 1e-5 difference check."""
    prob = setup(p, inst, gamma=gamma, sigma=sigma, m=m, tau=tau)
    gr = gradient(prob)
    h = 1e-5
    vals = []
    ranks = []
    for s in (prob["sigma"] * (1 + h), prob["sigma"] * (1 - h)):
        pp = dict(prob)
        pp["sigma"] = s
        ell, sol = loss_of(pp, prob["t_obs"], prob["y_obs"])
        vals.append(ell)
        ranks.append(sol["r"])
    if ranks[0] != ranks[1]:
        pytest.skip("an eigenvalue crosses the cut-off within the difference step")
    ref = (vals[0] - vals[1]) / (2 * h * prob["sigma"])
    assert abs(gr["dl_dsigma"] - ref) <= 1e-5 * abs(ref), (gr["dl_dsigma"], ref)


@pytest.mark.parametrize("sigma,m,tau", [(None, 20, 1e-10), (1.0, 40, 1e-6)])
def test_sigma_gradient_has_both_parts(sigma, m, tau):
    """At small gamma the K_mm (Daleckii-Krein) part is not negligible, so the difference
    check above would catch a dropped term."""
    gr = gradient(setup(2, 6 if sigma is None else 7, gamma=1.0, sigma=sigma, m=m, tau=tau))
    assert gr["sol"]["r"] < m or sigma is None
    assert abs(gr["sigma_kmm"]) > 1e-3 * abs(gr["sigma_direct"])


@pytest.mark.parametrize("inst", [0, 1])
def test_gamma_and_sigma_gradients_match_high_precision(inst):
    """At gamma = 1e7 (the second-order family's) dl/dgamma is a product of residual-sized
    quantities: pinned against a 50-digit solve of the same tiny instance (tests/
    hp_reference.py) differentiated by a central difference, together with dl/dsigma (its
    K_mm eigenbasis part included)."""
    import hp_reference
    prob = workloads.linear_second_order(inst, n=60, m=10, obs=20, config=5)
    gr = gradient(prob)
    ref_g = hp_reference.dloss(prob, "gamma")
    ref_s = hp_reference.dloss(prob, "sigma")
    assert abs(gr["dl_dgamma"] - ref_g) <= 1e-10 * abs(ref_g), (gr["dl_dgamma"], ref_g)
    assert abs(gr["dl_dsigma"] - ref_s) <= 1e-10 * abs(ref_s), (gr["dl_dsigma"], ref_s)
