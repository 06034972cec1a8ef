"""sigma and gamma changed on the device (nyls_plan_set_params) without rebuilding the plan,
and the differentiable solve captured in a HIP graph with them as inputs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_04094_amd import nyls as _nyls
from paper_2510_04094_amd import workloads

pytestmark = pytest.mark.gpu


def _insts():
    return [workloads.linear_second_order(i, n=1500, m=m, obs=40) for i, m in enumerate((30, 50, 62))]


def test_device_params_match_a_plan_built_with_them(gpu_lib):
    insts = _insts()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    s_new = np.array([q["sigma"] * 1.1 for q in insts])
    g_new = np.array([q["gamma"] * 0.5 for q in insts])
    st = b.set_params_device(torch.tensor(s_new, device="cuda"), torch.tensor(g_new, device="cuda"))
    y = b.solve()["yhat"].cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    moved = [dict(q, sigma=float(s), gamma=float(g)) for q, s, g in zip(insts, s_new, g_new)]
    ref = gpu_lib.Batch(moved, mode=gpu_lib.FP64).solve()["yhat"].cpu().numpy()
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    for i, q in enumerate(moved):
        yo = oracle.linear.solve(q)["yhat"]
        err = np.max(np.abs(y[b.goff[i]:b.goff[i + 1]] - yo)) / np.max(np.abs(yo))
        assert err <= 1e-9, (i, err)


def test_device_params_refuse_invalid_values(gpu_lib):
    insts = _insts()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    y0 = b.solve()["yhat"].clone()
    dt = insts[0]["dt"]
    bad_s = torch.tensor([-1.0, float("nan"), 2.0 * dt], device="cuda", dtype=torch.float64)
    st = b.set_params_device(bad_s, None).cpu().numpy()
    assert list(st) == [gpu_lib.S_PARAM_KEPT] * 3
    y1 = b.solve()["yhat"]
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)  # every instance kept its values
    st = b.set_params_device(None, torch.tensor([1e7, 0.0, float("inf")], device="cuda", dtype=torch.float64))
    assert list(st.cpu().numpy()) == [0, gpu_lib.S_PARAM_KEPT, gpu_lib.S_PARAM_KEPT]


def test_device_params_survive_retuning(gpu_lib):
    insts = _insts()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    s_new = torch.tensor([q["sigma"] * 0.9 for q in insts], device="cuda", dtype=torch.float64)
    b.set_params_device(s_new, None)
    y0 = b.solve()["yhat"].clone()
    b.set_tuning(eig_ql=1)
    y1 = b.solve()["yhat"]
    torch.cuda.synchronize()
    assert torch.max(torch.abs(y1 - y0)).item() <= 1e-9 * torch.max(torch.abs(y0)).item()


def test_solve_at_observations_replays_from_a_graph(gpu_lib):
    """Forward (solve + predict at the observations) and backward captured once, replayed with
    new sigma, gamma and forcing copied into the static inputs; each replay matches an eager
    run of the same inputs (replays interleaved with eager work)."""
    insts = _insts()
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    t_obs = [q["t_obs"] for q in insts]
    f0 = b.f.clone()
    r0 = b.r.clone()
    v0 = b.v.clone().reshape(len(insts), -1)
    s0 = torch.tensor([q["sigma"] for q in insts], device="cuda", dtype=torch.float64)
    g0 = torch.tensor([q["gamma"] for q in insts], device="cuda", dtype=torch.float64)
    y_obs = torch.tensor(np.concatenate([q["y_obs"] for q in insts]), device="cuda")

    def run(f, r, v, s, g):
        f = f.clone().requires_grad_(True)
        r = r.clone().requires_grad_(True)
        s = s.clone().requires_grad_(True)
        g = g.clone().requires_grad_(True)
        y = _nyls.solve_at_observations(b, t_obs, f, r, v, s, g)
        loss = torch.sum((y - y_obs) ** 2)
        loss.backward()
        return y.detach().clone(), r.grad.clone(), s.grad.clone(), g.grad.clone()

    # static inputs and an eager warm-up on a side stream (caches device copies of the times)
    sf, sr, sv, ss, sg = [x.clone() for x in (f0, r0, v0, s0, g0)]
    for p in (sr, ss, sg):
        p.requires_grad_(True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(sf, sr.detach(), sv, ss.detach(), sg.detach())
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        y_s = _nyls.solve_at_observations(b, t_obs, sf, sr, sv, ss, sg)
        loss_s = torch.sum((y_s - y_obs) ** 2)
        loss_s.backward()
    rng = np.random.default_rng(7)
    for rep in range(3):
        scale = torch.tensor(1.0 + 0.05 * rng.uniform(-1, 1, len(insts)), device="cuda")
        new = (f0 * (1.0 + 0.01 * rep), r0 * (1.0 - 0.02 * rep), v0, s0 * scale, g0 * (1.0 + 0.1 * rep))
        with torch.no_grad():
            sf.copy_(new[0])
            sr.copy_(new[1])
            sv.copy_(new[2])
            ss.copy_(new[3])
            sg.copy_(new[4])
            for p in (sr, ss, sg):
                p.grad = None if p.grad is None else p.grad.zero_()
        graph.replay()
        torch.cuda.synchronize()
        got = (y_s.detach().clone(), sr.grad.clone(), ss.grad.clone(), sg.grad.clone())
        ref = run(*new)  # eager, between the replays
        torch.cuda.synchronize()
        for name, a, e in zip(("y", "dr", "dsigma", "dgamma"), got, ref):
            err = (torch.max(torch.abs(a - e)) / torch.max(torch.abs(e))).item()
            assert err <= 1e-9, (rep, name, err)
