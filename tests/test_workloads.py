"""CPU checks of the seeded input generators (no solver arithmetic): instances drawn one at
a time equal those of the whole batch, and the manufactured solutions satisfy their ODEs."""
import numpy as np
import pytest

from paper_2510_04094_amd import workloads


def test_uneven_batch_instance_alone_equals_batch_entry():
    batch = workloads.mixed_batch(count=40)
    assert sorted({q["p"] for q in batch}) == [1, 2]
    for i in (0, 7, 39):
        q = workloads.mixed_batch_instance(i, count=40)
        assert (q["p"], q["n"], q["m"]) == (batch[i]["p"], batch[i]["n"], batch[i]["m"])
        assert np.array_equal(q["f"], batch[i]["f"]) and np.array_equal(q["r"], batch[i]["r"])


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("bvp", [False, True])
def test_order_p_manufactured_solution_satisfies_the_ode(p, bvp):
    """Central differences of the closed-form y* reproduce y^(p) = sum f_k y^(p-k) + r, and
    the conditions are y*'s own values."""
    q = workloads.linear_order_p(0, p, n=4001, bvp=bvp)
    t = q["t"]
    h = 1e-3
    sol = q["sol"]

    def ys(k, tt):
        arg = sol["w"][None, :] * tt[:, None] + sol["ph"][None, :] + 0.5 * np.pi * k
        return np.sin(arg) @ (sol["c"] * sol["w"] ** k)

    # derivatives of y* by central differences of y* itself (independent of the generator's
    # closed-form derivative orders)
    tm = t[10:-10]
    stencil = {1: [(-0.5, -1), (0.5, 1)], 2: [(1, -1), (-2, 0), (1, 1)],
               3: [(-0.5, -2), (1, -1), (-1, 1), (0.5, 2)], 4: [(1, -2), (-4, -1), (6, 0), (-4, 1), (1, 2)]}
    d = [ys(0, tm)]
    for k in range(1, p + 1):
        d.append(sum(c * ys(0, tm + j * h) for c, j in stencil[k]) / h ** k)
    lhs = d[p] - sum(q["f"][k - 1, 10:-10] * d[p - k] for k in range(1, p + 1))
    assert np.max(np.abs(lhs - q["r"][10:-10])) <= 1e-3 * max(1.0, np.max(np.abs(q["r"])))
    for j, (dd, i) in enumerate(zip(q["cond_d"], q["cond_i"])):
        assert abs(q["v"][j] - ys(dd, t[i:i + 1])[0]) <= 1e-12
    assert len(q["cond_d"]) == p
