"""Pins for oracle.leverage (leverage-score landmark sampling, Sec. 4.1) against the
definition of ridge leverage scores on the full kernel matrix, identities of the scores, the
exact probabilities of weighted sampling without replacement, and the accuracy of a solve on
the sampled landmarks."""
import itertools

import numpy as np

import oracle
from oracle import leverage
from paper_2510_04094_amd import workloads


def test_scores_reduce_to_the_exact_ridge_leverage_when_m_equals_n():
    """m = n: the features reproduce K (Phi Phi^T = K), so l_i = diag(K (K + ridge I)^{-1})
    with K built directly from the kernel."""
    n = 40
    q = workloads.linear_first_order(0, n=n, m=n, sigma=0.05, tau=1e-14)
    t = q["t"]
    kfull = oracle.rbf.kernel(t[:, None], t[None, :], q["sigma"])
    for ridge in (1e-3, 1e-6):
        np.testing.assert_allclose(leverage.scores(q, ridge), leverage.exact_ridge_scores(kfull, ridge),
                                   rtol=0, atol=1e-9)


def test_score_identities():
    """0 <= l_i <= 1 and sum_i l_i = tr(Phi^T Phi (Phi^T Phi + ridge I)^{-1}) <= r."""
    q = workloads.linear_second_order(0, n=2000, m=40)
    s = leverage.scores(q)
    t = q["t"]
    tl = t[oracle.nystrom.landmark_indices(q)]
    _, _, r, w = oracle.nystrom.basis(tl, q["sigma"], q["tau"])
    phi = oracle.nystrom.features(0, t, tl, q["sigma"], w)
    g = phi.T @ phi
    lam = 1.0 / q["gamma"]
    assert np.all(s >= 0) and np.all(s <= 1 + 1e-12)
    np.testing.assert_allclose(np.sum(s), np.trace(g @ np.linalg.inv(g + lam * np.eye(r))), rtol=1e-9)
    assert np.sum(s) <= r + 1e-9


def test_exponential_keys_sample_without_replacement_with_the_right_probabilities():
    """n = 5, m = 2: the frequency of each pair over 40000 draws matches
    P({a, b}) = w_a/W w_b/(W - w_a) + w_b/W w_a/(W - w_b)."""
    w = np.array([0.1, 0.5, 0.2, 0.9, 0.3])
    W = w.sum()
    rng = np.random.default_rng(7)
    draws = 40000
    counts = {}
    for _ in range(draws):
        pair = tuple(leverage.sample(w, 2, 1.0 - rng.random(5), ends=False))
        counts[pair] = counts.get(pair, 0) + 1
    for a, b in itertools.combinations(range(5), 2):
        pr = w[a] / W * w[b] / (W - w[a]) + w[b] / W * w[a] / (W - w[b])
        sd = np.sqrt(pr * (1 - pr) / draws)
        assert abs(counts.get((a, b), 0) / draws - pr) <= 5 * sd, (a, b)


def test_sample_contract():
    q = workloads.linear_second_order(1, n=1500, m=30)
    s = leverage.scores(q)
    u = workloads.leverage_uniforms(1, q["n"])
    for ends in (True, False):
        idx = leverage.sample(s, q["m"], u, ends=ends)
        assert idx.size == q["m"] and np.all(np.diff(idx) > 0)
        assert idx[0] >= 0 and idx[-1] < q["n"]
        if ends:
            assert idx[0] == 0 and idx[-1] == q["n"] - 1


def test_leverage_landmarks_reach_the_manufactured_accuracy():
    """A solve on leverage-sampled landmarks recovers y* about as well as on equidistant ones
    (the paper finds the three strategies comparable)."""
    for k in range(3):
        q = workloads.linear_first_order(k, n=400, m=20, sigma=0.1)
        base = np.max(np.abs(oracle.linear.solve(q)["yhat"] - q["ystar"]))
        q2 = dict(q, lidx=leverage.sample(leverage.scores(q), q["m"], workloads.leverage_uniforms(k, q["n"])))
        err = np.max(np.abs(oracle.linear.solve(q2)["yhat"] - q["ystar"]))
        assert err <= max(20 * base, 1e-4), (k, err, base)
