"""GPU parity of leverage-score landmark sampling (Sec. 4.1) against the oracle: the scores,
the sampled index sets, and a solve on the sampled basis."""
import numpy as np
import pytest
import torch

import fp64_floor
import oracle
from oracle import leverage
from paper_2510_04094_amd import workloads

pytestmark = pytest.mark.gpu


def instances():
    insts = [workloads.linear_first_order(i, n=400, m=20) for i in range(3)]
    insts += [workloads.linear_second_order(i, n=1500 + 111 * i, m=m) for i, m in enumerate((30, 50, 62))]
    return insts


def test_scores_match_oracle(gpu_lib):
    insts = instances()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    s = b.leverage_scores().cpu().numpy()
    for i, q in enumerate(insts):
        ref = leverage.scores(q)
        got = s[b.goff[i]:b.goff[i + 1]]
        # the scores are the feature-space projection of each grid point: like y_hat they
        # carry the eigenbasis rounding near the cut-off, hence the oracle's own FP64 bar
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= fp64_floor.bar_of(leverage.scores, q, ref), (i, err)


@pytest.mark.parametrize("ends", [True, False])
def test_sampled_landmarks_match_oracle(gpu_lib, ends):
    """The GPU draws the same index set as the oracle from the same uniforms (keys computed
    in both places from scores that agree to rounding; a difference is accepted only where
    the two keys at the boundary of the selection are within 1e-9 of each other)."""
    insts = instances()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    us = [workloads.leverage_uniforms(i, q["n"]) for i, q in enumerate(insts)]
    _, got = b.leverage_landmarks(us, ends=ends)
    for i, q in enumerate(insts):
        sc = leverage.scores(q)
        ref = leverage.sample(sc, q["m"], us[i], ends=ends)
        if not np.array_equal(got[i], ref):
            key = np.log(us[i]) / sc
            diff = np.setxor1d(got[i], ref)
            kk = np.sort(key[diff])
            assert kk[-1] - kk[0] <= 1e-9 * abs(kk[0]), (i, diff, key[diff])
        assert got[i].size == q["m"] and np.all(np.diff(got[i]) > 0)
        if ends:
            assert got[i][0] == 0 and got[i][-1] == q["n"] - 1


def test_solve_on_leverage_landmarks_matches_oracle(gpu_lib):
    insts = instances()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    us = [workloads.leverage_uniforms(i, q["n"]) for i, q in enumerate(insts)]
    _, lidx = b.leverage_landmarks(us)
    sampled = [dict(q, lidx=lidx[i]) for i, q in enumerate(insts)]
    b2 = gpu_lib.Batch(sampled, mode=gpu_lib.FP64)
    out = b2.solve()
    torch.cuda.synchronize()
    y = out["yhat"].cpu().numpy()
    for i, q in enumerate(sampled):
        ref = oracle.linear.solve(q)["yhat"]
        err = np.max(np.abs(y[b2.goff[i]:b2.goff[i + 1]] - ref)) / np.max(np.abs(ref))
        assert err <= fp64_floor.bar(q, ref), (i, err)
