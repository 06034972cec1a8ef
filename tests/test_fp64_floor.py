"""CPU pins of the FP64 parity floor (tests/fp64_floor.py): the claims its docstring makes
about the oracle's own sensitivity, measured on the oracle alone."""
import numpy as np

import fp64_floor
import oracle
from paper_2510_04094_amd import workloads


def test_well_conditioned_instances_have_no_floor_above_1e_minus_10():
    """Full-rank bases (sigma small against the landmark spacing): 1-ulp K_mm noise moves
    y_hat by far less than the FP64 bar, so the bar stays 1e-10."""
    for q in [workloads.linear_first_order(0), workloads.linear_second_order(4, n=1528, m=50)]:
        assert fp64_floor.floor(q) < 1e-11
        assert fp64_floor.bar(q) == 1e-10


def test_near_cutoff_instance_has_a_floor_near_1e_minus_10():
    """Second-order instance with an eigenvalue at 1.5e-8 lambda_1, just above the cut-off
    1e-8: the oracle's own y_hat moves by several 1e-11 under 1-ulp K_mm noise."""
    q = workloads.linear_second_order(1, n=1334, m=50)
    sol = oracle.linear.solve(q)
    lam = sol["lam"]
    assert 1e-8 < lam[sol["r"] - 1] / lam[0] < 2e-8
    assert fp64_floor.floor(q, sol["yhat"]) > 2e-11


def test_floor_catches_a_perturbation_of_that_size():
    """The measurement is not saturated: K_mm perturbed 100 times more than the eigensolver
    backward-error model moves y_hat well beyond the measured floor on the same instance."""
    q = workloads.linear_second_order(1, n=1334, m=50)
    ref = oracle.linear.solve(q)["yhat"]
    f1 = fp64_floor.floor(q, ref)
    orig = oracle.nystrom.landmark_gram

    def big(t, s):
        k = orig(t, s)
        e = np.random.default_rng(5).uniform(-1, 1, k.shape) * 200 * fp64_floor.EPS * np.linalg.norm(k, 2)
        return k + 0.5 * (e + e.T)

    oracle.nystrom.landmark_gram = big
    try:
        y = oracle.linear.solve(q)["yhat"]
    finally:
        oracle.nystrom.landmark_gram = orig
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) > 4 * f1
