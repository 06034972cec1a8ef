"""One instance split over many workgroups: the Gram and the refinement/output passes of a
long instance run as chunks of grid points, one workgroup per chunk, with the chunk sums
added in chunk order.  GPU against the oracle (and against the unsplit solve) for long
first-order instances up to the largest basis, forced splits of higher-order and boundary
problems, explicit time grids and a batch where only some instances split."""
import numpy as np
import pytest
import torch

import fp64_floor
import oracle
from paper_2510_04094_amd import workloads
from test_gpu_linear import FP64_HIGHER_ORDER, higher_order_instance

pytestmark = pytest.mark.gpu


def _solve(gpu_lib, insts, refine=None, **kw):
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64, **kw)
    out = b.solve(refine)
    torch.cuda.synchronize()
    y = out["yhat"].cpu().numpy()
    return b, out, [y[b.goff[i]:b.goff[i + 1]] for i in range(len(insts))]


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("m", [20, 50, 100, 128])
def test_long_first_order_instance_splits_at_the_fp64_bar(gpu_lib, m):
    """n = 5e4 on [0, 20], sigma = 0.3, cut-off 1e-10: split automatically (one instance),
    and the same instance unsplit; both at 1e-10 from the oracle."""
    q = workloads.linear_first_order(m, n=50000, m=m, t_end=20.0, sigma=0.3, tau=1e-10)
    ref = oracle.linear.solve(q)["yhat"]
    b, out, ys = _solve(gpu_lib, [q])
    assert b.get_tuning()["split"] == -1
    _, _, y0 = _solve(gpu_lib, [q], tuning=dict(split=0))
    assert _rel(ys[0], ref) <= 1e-10, _rel(ys[0], ref)
    assert _rel(y0[0], ref) <= 1e-10, _rel(y0[0], ref)
    info = b.info().cpu().numpy()
    assert 1 <= info[0, 5] <= 4
    assert int(out["status"].cpu().numpy()[0]) & (gpu_lib.S_SINGULAR | gpu_lib.S_NONFINITE | gpu_lib.S_REFINE_NOCONV) == 0


def test_forced_split_on_higher_orders_and_boundary_conditions(gpu_lib):
    """split = 512 on second- to fourth-order problems with initial and two-point boundary
    conditions (condition points inside the last chunk; instances shorter than a chunk run
    as one chunk) at the FP64 bar of the unsplit test."""
    insts = [higher_order_instance(name, tau) for name, tau in FP64_HIGHER_ORDER]
    insts += [workloads.linear_second_order(3, n=4000, m=50), workloads.linear_first_order(4, n=3000, m=33)]
    _, out, ys = _solve(gpu_lib, insts, tuning=dict(split=512))
    for i, q in enumerate(insts):
        ref = oracle.linear.solve(q)["yhat"]
        bar = 1e-10 if i < len(FP64_HIGHER_ORDER) else fp64_floor.bar(q, ref)
        assert _rel(ys[i], ref) <= bar, (i, q["p"], q["n"], _rel(ys[i], ref), bar)


def test_split_on_explicit_time_grids(gpu_lib):
    """Explicit (non-uniform storage) grids take the exact-exponential passes; split = 512."""
    insts = [workloads.linear_second_order(5, n=6000, m=50), workloads.linear_first_order(6, n=5000, m=33)]
    _, _, ys = _solve(gpu_lib, insts, explicit_grid=True, tuning=dict(split=512))
    for i, q in enumerate(insts):
        ref = oracle.linear.solve(q)["yhat"]
        assert _rel(ys[i], ref) <= fp64_floor.bar(q, ref), (i, _rel(ys[i], ref))


def test_batch_where_some_instances_split(gpu_lib):
    """Automatic split in a small batch: instances with n >= 4096 split, the others run one
    wavefront each; orders 1 to 3 and bases from 20 to 100."""
    insts = [workloads.linear_first_order(7, n=50000, m=100, t_end=20.0, sigma=0.3, tau=1e-10),
             workloads.linear_second_order(8, n=9000, m=50),
             workloads.linear_first_order(9, n=3000, m=20),
             workloads.linear_second_order(10, n=2000, m=62),
             workloads.linear_order_p(11, 3, n=6000, m=40, sigma=0.2, tau=1e-8)]
    _, out, ys = _solve(gpu_lib, insts)
    for i, q in enumerate(insts):
        ref = oracle.linear.solve(q)["yhat"]
        bar = 1e-10 if i == 0 else fp64_floor.bar(q, ref)
        assert _rel(ys[i], ref) <= bar, (i, _rel(ys[i], ref), bar)


def test_split_solution_feeds_predict_and_backward(gpu_lib):
    """The split solve leaves the same kind of solution in the workspace: y_hat at caller
    times and the adjoint gradients agree with the unsplit plan's."""
    q = workloads.linear_second_order(12, n=8000, m=50, obs=100)
    res = []
    for split in (512, 0):
        b = gpu_lib.Batch([q], mode=gpu_lib.FP64, tuning=dict(split=split))
        b.solve()
        yo, _ = b.predict([q["t_obs"]], 0)
        g = torch.tensor(2.0 * (yo.cpu().numpy() - q["y_obs"]) / q["y_obs"].size, device="cuda")
        gr = b.backward([q["t_obs"]], g)
        torch.cuda.synchronize()
        res.append((yo.cpu().numpy(), {k: v.cpu().numpy() for k, v in gr.items()}))
    (ya, ga), (yb, gb) = res
    assert _rel(ya, yb) <= 1e-9
    for k in ("dl_dr", "dl_dv", "dl_dsigma"):
        assert _rel(ga[k], gb[k]) <= 1e-6, (k, _rel(ga[k], gb[k]))


def test_split_without_refinement(gpu_lib):
    """refine = 0: the split path runs only the output pass; the result is the unrefined
    solve of the same system (close to the unsplit unrefined one) and no refinement flag."""
    q = workloads.linear_second_order(13, n=8000, m=50)
    _, out_s, ys = _solve(gpu_lib, [q], refine=0, tuning=dict(split=1024))
    _, out_u, yu = _solve(gpu_lib, [q], refine=0, tuning=dict(split=0))
    assert np.all(np.isfinite(ys[0]))
    assert _rel(ys[0], yu[0]) <= 1e-4
    assert int(out_s["status"].cpu().numpy()[0]) & gpu_lib.S_REFINE_NOCONV == 0


@pytest.mark.parametrize("split", [512, 2048])
def test_split_adjoint_matches_oracle(gpu_lib, split):
    """The adjoint of split instances (passes over chunks, chunk sums in chunk order) against
    the oracle's gradients with the bars of the unsplit adjoint test: orders 1 and 2, bases of
    20 to 62 landmarks (the m = 33 one with a last block of a single landmark)."""
    from test_gpu_adjoint import loss_grad_obs, rel
    insts = [workloads.linear_second_order(i, n=5000, m=m, obs=100, config=5) for i, m in enumerate((50, 62, 20))]
    insts.append(workloads.linear_first_order(3, n=4000, m=33))
    insts[-1]["t_obs"] = np.sort(np.random.default_rng(5).uniform(0.0, 1.0, 60))
    insts[-1]["y_obs"] = np.interp(insts[-1]["t_obs"], insts[-1]["t"], insts[-1]["ystar"])
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64, tuning=dict(split=split))
    b.solve()
    yo, off = b.predict([q["t_obs"] for q in insts], 0)
    yo = yo.cpu().numpy()
    g = [loss_grad_obs(yo[off[i]:off[i + 1]], q["y_obs"]) for i, q in enumerate(insts)]
    out = b.backward([q["t_obs"] for q in insts], g)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    info = b.info().cpu().numpy()
    for i, q in enumerate(insts):
        ref = oracle.adjoint.grad(q, q["t_obs"], g[i])
        o = slice(b.goff[i], b.goff[i + 1])
        for k in range(q["p"]):
            gf, rf = out["dl_df"][k, o], ref["dl_df"][k]
            assert np.max(np.abs(gf - rf)) <= 1e-5 * np.max(np.abs(rf)), ("df", i, k)
        assert np.max(np.abs(out["dl_dr"][o] - ref["dl_dr"])) <= 1e-5 * np.max(np.abs(ref["dl_dr"]))
        for j in range(q["p"]):
            assert rel(out["dl_dv"][i, j], ref["dl_dv"][j]) <= 1e-5, ("dv", i, j)
        scale = 1e-5 * abs(ref["dl_dsigma"]) + 1e-8 * np.max(np.abs(ref["sigma_terms"]))
        assert abs(out["dl_dsigma"][i] - ref["dl_dsigma"]) <= scale, ("dsigma", i)
        assert rel(out["dl_dgamma"][i], ref["dl_dgamma"]) <= 1e-5, ("dgamma", i)
        assert 1 <= info[i, 6] <= 3  # mu refinement passes
