"""Every launch choice of nyls_tuning computes the method: GPU against the oracle under each
single-knob change from the defaults (and all knobs flipped), in FP64 and mixed mode; the
tuning calls; and the autotuner with its cache."""
import numpy as np
import pytest
import torch

import fp64_floor
import oracle
from paper_2510_04094_amd import autotune, workloads

pytestmark = pytest.mark.gpu


def instances():
    # m = 50: a last slot block of 2 landmarks (tail layout) and a last Gram block of 4
    # columns; m = 34: a last Gram block of 4 columns; m = 33: a one-landmark tail;
    # m = 62: full blocks; m = 100: beyond the one-wave Gram and QL
    insts = [workloads.linear_second_order(i, n=2000 + 97 * i, m=m) for i, m in enumerate((50, 34, 62, 20))]
    insts += [workloads.linear_first_order(i, n=1200, m=m) for i, m in enumerate((33, 20))]
    insts += [workloads.linear_second_order(9, n=3000, m=100)]
    return insts


_REF = {}


def reference():
    if not _REF:
        for i, q in enumerate(instances()):
            y = oracle.linear.solve(q)["yhat"]
            _REF[i] = (y, fp64_floor.bar(q, y))
    return _REF


VARIANTS = [dict(), dict(eig_ql=1), dict(ql_lanes=16), dict(ql_lanes=37), dict(gram_valu=1),
            dict(tail_layout=0), dict(overlap=0),
            dict(eig_ql=1, gram_valu=1, tail_layout=0, overlap=0)]


def _errs(b, out, insts):
    y = out["yhat"].cpu().numpy()
    ref = reference()
    return [(float(np.max(np.abs(y[b.goff[i]:b.goff[i + 1]] - ref[i][0])) / np.max(np.abs(ref[i][0]))), ref[i][1])
            for i in range(len(insts))]


@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: ",".join("%s=%d" % kv for kv in v.items()) or "default")
def test_fp64_solve_under_each_tuning(gpu_lib, variant):
    insts = instances()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64, tuning=variant)
    assert b.get_tuning() == dict(gpu_lib.DEFAULT_TUNING, **variant)
    out = b.solve()
    torch.cuda.synchronize()
    for i, (err, bar) in enumerate(_errs(b, out, insts)):
        assert err <= bar, (i, insts[i]["m"], err, bar)
    assert not np.any(out["status"].cpu().numpy() & (gpu_lib.S_SINGULAR | gpu_lib.S_NONFINITE))


@pytest.mark.parametrize("variant", [dict(), dict(eig_ql=1), dict(tail_layout=0)],
                         ids=["default", "eig_ql=1", "tail_layout=0"])
def test_mixed_solve_under_each_tuning(gpu_lib, variant):
    insts = instances()
    b = gpu_lib.Batch(insts, mode=gpu_lib.MIXED, tuning=variant)
    out = b.solve()
    torch.cuda.synchronize()
    for i, (err, _) in enumerate(_errs(b, out, insts)):
        assert err <= 1e-6, (i, err)


def test_retuning_a_plan_between_solves(gpu_lib):
    """set_tuning on a live plan: the next solve follows the new choices and agrees with the
    first to the FP64 bar."""
    insts = instances()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    y0 = b.solve()["yhat"].clone()
    b.set_tuning(eig_ql=1, tail_layout=0, gram_valu=1)
    y1 = b.solve()["yhat"]
    torch.cuda.synchronize()
    for i, (err, bar) in enumerate(_errs(b, dict(yhat=y1), insts)):
        assert err <= bar, (i, err, bar)
    assert torch.max(torch.abs(y1 - y0)).item() <= 1e-6 * torch.max(torch.abs(y0)).item()


def test_invalid_tuning_is_rejected(gpu_lib):
    b = gpu_lib.Batch(instances()[:2], mode=gpu_lib.FP64)
    for bad in (dict(ql_lanes=0), dict(ql_lanes=65), dict(eig_ql=2), dict(overlap=-1)):
        with pytest.raises(gpu_lib.NylsError):
            b.set_tuning(**bad)
    assert b.get_tuning() == gpu_lib.DEFAULT_TUNING


def test_autotune_picks_a_measured_choice_and_caches_it(gpu_lib, tmp_path, monkeypatch):
    path = str(tmp_path / "tuning.json")
    monkeypatch.setenv("NYLS_TUNING_CACHE", path)
    insts = [workloads.linear_second_order(i, n=3000, m=50) for i in range(64)]
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    res = autotune.autotune(b, reps=2)
    assert res["tuning"] in [t for t, _ in res["tried"]]
    chosen_ms = [ms for t, ms in res["tried"] if t == res["tuning"]]
    assert res["ms"] in chosen_ms
    # nothing tried beats the choice by more than the tuner's 2 % margin
    assert min(ms for _, ms in res["tried"]) >= (1.0 - 0.02) * res["ms"] - 1e-9
    assert b.get_tuning() == res["tuning"]
    assert autotune.lookup(res["key"]) == res["tuning"]
    assert res["key"].endswith("|m<=64|p2|fp64")
    b2 = gpu_lib.Batch(insts[:8], mode=gpu_lib.FP64, tuning="cached")
    assert b2.get_tuning() == res["tuning"]
    out = b2.solve()
    torch.cuda.synchronize()
    y = out["yhat"].cpu().numpy()
    for i, q in enumerate(insts[:8]):
        ref = oracle.linear.solve(q)["yhat"]
        err = np.max(np.abs(y[b2.goff[i]:b2.goff[i + 1]] - ref)) / np.max(np.abs(ref))
        assert err <= fp64_floor.bar(q, ref), (i, err)
