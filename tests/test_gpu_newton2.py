"""GPU parity of the Lemma 2 Newton iteration for second-order nonlinear ODEs y'' = F(t, y, y')
(the seeded family and the paper's boundary problems 14 and 15) against the oracle."""
import numpy as np
import pytest
import torch

import fp64_floor
import oracle
from oracle import newton_general as ng
from paper_2510_04094_amd import workloads

pytestmark = pytest.mark.gpu

GN_STEPS = 5


def family_fun(insts, goff):
    """F, dF, d2F of the seeded family on the device, per grid point of the whole batch."""
    total = int(goff[-1])
    c = np.zeros((3, total))
    q = np.zeros(total)
    for i, p in enumerate(insts):
        c[:, goff[i]:goff[i + 1]] = p["c"][:, None]
        q[goff[i]:goff[i + 1]] = p["q"]
    c = torch.tensor(c, device="cuda")
    q = torch.tensor(q, device="cuda")

    def fun(u, gauss_newton):
        y, yp = u[0], u[1]
        F = q - c[0] * y - c[1] * y ** 3 - c[2] * yp * yp
        dF = torch.stack([-c[0] - 3 * c[1] * y * y, -2 * c[2] * yp])
        z = torch.zeros_like(y)
        d2F = torch.stack([torch.stack([-6 * c[1] * y, z]), torch.stack([z, -2 * c[2] + z])])
        return F, dF, d2F
    return fun


def torch_paper_fun(which):
    def fun(u, gauss_newton):
        y, yp = u[0], u[1]
        z = torch.zeros_like(y)
        if which == 14:
            e = torch.exp(-y)
            return (-yp * yp + 2 * e, torch.stack([-2 * e, -2 * yp]),
                    torch.stack([torch.stack([2 * e, z]), torch.stack([z, z - 2])]))
        return (-y + 2 * yp * yp / y, torch.stack([-1 - 2 * yp * yp / (y * y), 4 * yp / y]),
                torch.stack([torch.stack([4 * yp * yp / y ** 3, -4 * yp / (y * y)]),
                             torch.stack([-4 * yp / (y * y), 4 / y])]))
    return fun


def oracle_fun(prob):
    def fun(idx, y, u):
        return workloads.nonlinear_second_order_rhs(prob, y, u[0], idx)
    return fun


def gpu_yhat(b, insts):
    yh, off = b.predict([p["t"] for p in insts], 0)
    torch.cuda.synchronize()
    yh = yh.cpu().numpy()
    return [yh[off[i]:off[i + 1]] for i in range(len(insts))]


@pytest.mark.parametrize("n,m,count", [(1000, 20, 6), (3000, 40, 4)])
def test_second_order_newton_matches_oracle(gpu_lib, n, m, count):
    insts = [workloads.nonlinear_second_order(i, n=n, m=m) for i in range(count)]
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    x, hist = b.newton_solve(family_fun(insts, b.goff), max_iter=30, tol=1e-12,
                             gauss_newton_steps=GN_STEPS)
    ys = gpu_yhat(b, insts)
    xs = x.cpu().numpy()
    iters = hist.shape[0]
    for i, p in enumerate(insts):
        # the oracle takes the same number of steps (the stopping test is relative to |x|_inf,
        # which omega can dominate: stopping one step apart would leave the y-block 1e-9 apart)
        ref = ng.solve(p, oracle_fun(p), tol=0.0, max_iter=iters, gauss_newton_steps=GN_STEPS)
        err = np.max(np.abs(ys[i] - ref["yhat"])) / np.max(np.abs(ref["yhat"]))
        assert err <= 1e-10, (i, err, hist[:, i].cpu().numpy(), ref["steps"])
        # the auxiliary y_i = y_hat_i + rho_i F_0,i carry the ODE residual rho, whose second
        # derivative of the model amplifies the eigenbasis rounding: their own FP64 bar
        def y_block(q):
            st = ng.solve(q, oracle_fun(q), tol=0.0, max_iter=iters, schur=True,
                          gauss_newton_steps=GN_STEPS)
            return st["x"][st["r"] + 3:]
        xo = ref["x"][ref["r"] + 3:]
        yg = xs[i, b.maxm + 3:b.maxm + 3 + p["n"]][ref["idx"]]
        err_y = np.max(np.abs(yg - xo)) / np.max(np.abs(xo))
        assert err_y <= fp64_floor.bar_of(y_block, p, xo), (i, err_y)
        assert np.max(np.abs(ys[i] - p["ystar"])) < 1e-5


def test_second_order_first_steps_track_oracle(gpu_lib):
    """Step by step from the same start (the Gauss-Newton steps and the first Newton steps):
    the y-block of every iterate agrees with the oracle's to the FP64 bar of those iterates.
    The y-block is compared rather than omega, whose components along features near the
    cut-off carry the eigenbasis rounding amplified (omega is not unique to rounding; the
    model it defines is)."""
    insts = [workloads.nonlinear_second_order(i, n=800, m=20) for i in range(3)]
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    fun = family_fun(insts, b.goff)
    x = b.newton_init()
    nsteps = GN_STEPS + 2
    got = []
    for k in range(nsteps):
        F, dF, d2F = fun(b.newton_state(x), k < GN_STEPS)
        if k < GN_STEPS:
            d2F = torch.zeros_like(d2F)
        b.newton_step(x, F.contiguous(), dF.contiguous(), d2F.contiguous())
        got.append(x.clone())
    got = torch.stack(got).cpu().numpy()
    for i, p in enumerate(insts):
        def iterates(q):
            st = ng.setup(q)
            xo = ng.initial_state(st, q)
            ys = []
            for k in range(nsteps):
                xo, _ = ng.step_schur(xo, st, q, oracle_fun(q), gauss_newton=k < GN_STEPS)
                ys.append(xo[st["r"] + 3:].copy())
            return np.concatenate(ys)
        ref = iterates(p)
        idx = ng.setup(p)["idx"]
        yg = np.concatenate([got[k, i, b.maxm + 3:b.maxm + 3 + p["n"]][idx] for k in range(nsteps)])
        err = np.max(np.abs(yg - ref)) / np.max(np.abs(ref))
        assert err <= fp64_floor.bar_of(iterates, p, ref), (i, err)


@pytest.mark.parametrize("which", [14, 15])
def test_paper_nonlinear_boundary_problems(gpu_lib, which):
    """The paper's problems 14 and 15 (y' inside F, two-point boundary conditions) with its
    n, m, sigma^2, gamma: GPU against oracle, and the accuracy the paper reports."""
    from test_oracle_newton_general import CLOSED, entries, paper_nonlinear
    entry = [e for e in entries() if e["id"] == which][0]
    prob, fun_np, exact = paper_nonlinear(entry, tau=1e-12)
    prob["t0"], prob["dt"] = float(prob["t"][0]), float(prob["t"][1] - prob["t"][0])
    prob["t"] = prob["t0"] + np.arange(prob["n"]) * prob["dt"]
    exact = CLOSED[which][2](prob["t"])
    b = gpu_lib.Batch([prob], mode=gpu_lib.FP64)
    x, hist = b.newton_solve(torch_paper_fun(which), max_iter=40, tol=1e-12,
                             gauss_newton_steps=GN_STEPS)
    y = gpu_yhat(b, [prob])[0]
    ref = ng.solve(prob, fun_np, tol=1e-12, max_iter=40, gauss_newton_steps=GN_STEPS)
    err = np.max(np.abs(y - ref["yhat"])) / np.max(np.abs(ref["yhat"]))
    assert err <= 1e-10, (err, hist[:, 0].cpu().numpy(), ref["steps"])
    assert np.mean(np.abs(y - exact)) <= 10 * entry["mae"]


def test_newton_rejects_mixed_orders(gpu_lib):
    insts = [workloads.riccati(0, n=300), workloads.nonlinear_second_order(0, n=300)]
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    with pytest.raises(gpu_lib.NylsError):
        b.newton_init()
