#!/usr/bin/env python3
"""Throughput of the batched Nystrom primal LS-SVM ODE solver on one MI355X.

A step is one pass of the whole hot path over a batch of synthetic second-order linear
ODE instances (n = 10^4 grid points, m = 50 landmarks, sigma ~ U(0.2, 1), gamma = 1e7,
cut-off 1e-8, 100 noisy observations each): basis (K_mm eigendecomposition), fused
operator Gram, KKT factorisation and solve, FP64 refinement, y_hat on the grid and at
the observations, the loss gradient and the adjoint gradients w.r.t. the ODE data,
conditions, sigma and gamma.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  `value` counts ODE solves (forward + adjoint) per second, only for
instances whose y_hat matches the CPU oracle to rel. 1e-6 (every instance of the batch is
checked, after the timed steps) and whose status bits report no failure.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32_mfma": 157.3e12, "hbm": 8.0e12}

# HBM traffic of the dominant kernel per launch on this workload, from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE in KiB) scaled by what the counters read for a 1 GiB device
# copy (fetch x2, write x1); reported only while the kernel's sources are unchanged.
TRAFFIC = {
    "backward": {
        "sources": ["paper_2510_04094_amd/csrc/adjoint.hip", "paper_2510_04094_amd/csrc/nyls_walk.h",
                    "paper_2510_04094_amd/csrc/nyls_dense.h", "paper_2510_04094_amd/csrc/nyls_internal.h"],
        "sha1": "fb793b96100193ff350f0670e346a0097096bdb0",
        "kib": {"mixed": (2126766.0, 1128630.5), "fp64": (2269630.2, 1129528.3)},
        "scale": (2.0, 1.0),
    },
}


def measured_traffic(kernel, mode, batch):
    """Calibrated HBM bytes per launch, or None when not measured for this kernel/source."""
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None or batch != 4096 or mode not in t["kib"]:
        return None
    h = hashlib.sha1()
    for f in t["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != t["sha1"]:
        return None
    fk, wk = t["kib"][mode]
    return (fk * t["scale"][0] + wk * t["scale"][1]) * 1024.0


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def make_instances(count, n, m, seed_config):
    from paper_2510_04094_amd import workloads
    return [workloads.linear_second_order(i, n=n, m=m, config=seed_config, obs=100)
            for i in range(count)]


def _oracle_job(args):
    """CPU oracle: forward solve + adjoint gradient of one instance (single thread)."""
    i, n, m, seed_config = args
    import oracle
    from paper_2510_04094_amd import workloads
    q = workloads.linear_second_order(i, n=n, m=m, config=seed_config, obs=100)
    t0 = time.perf_counter()
    sol = oracle.linear.solve(q)
    yo = oracle.linear.predict(sol, q["t_obs"], q["sigma"], 0)
    g = 2.0 * (yo - q["y_obs"]) / yo.size
    oracle.adjoint.grad(q, q["t_obs"], g)
    return time.perf_counter() - t0


def _oracle_err(args):
    """rel. l-inf distance of a GPU y_hat from the oracle's (second-order instance i)."""
    i, n, m, seed_config, got = args
    import oracle
    from paper_2510_04094_amd import workloads
    q = workloads.linear_second_order(i, n=n, m=m, config=seed_config, obs=100)
    ref = oracle.linear.solve(q)["yhat"]
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _floor_bar(args):
    """The FP64 parity bar of second-order instance i: max(1e-10, 4 x the oracle's own
    rounding floor), as the parity tests use it."""
    i, n, m, seed_config = args
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    import fp64_floor
    from paper_2510_04094_amd import workloads
    return fp64_floor.bar(workloads.linear_second_order(i, n=n, m=m, config=seed_config, obs=100))


def _oracle_err_newton(args):
    """rel. l-inf distance of a GPU Newton y_hat from the oracle's after the same number of
    Newton steps (Riccati instance i, two Gauss-Newton steps first)."""
    i, iters, got = args
    import oracle
    from paper_2510_04094_amd import workloads
    p = workloads.riccati(i)
    st = oracle.newton.setup(p)
    x = oracle.newton.initial_state(st, p)

    def fun(gn):
        return lambda idx, y: (p["q"][idx] - y * y, -2.0 * y, (0.0 if gn else -2.0) * np.ones_like(y))
    for k in range(iters):
        x, _ = oracle.newton.step_schur(x, st, p, fun(k < 2))
    r = st["r"]
    ref = oracle.nystrom.kvec(0, st["t"], st["t_land"], p["sigma"]) @ (st["W"] @ x[:r]) + x[r]
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _oracle_err_uneven(args):
    """The same for instance i of the uneven batch."""
    i, count, got = args
    import oracle
    from paper_2510_04094_amd import workloads
    q = workloads.mixed_batch_instance(i, count=count)
    ref = oracle.linear.solve(q)["yhat"]
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


_UNEVEN = {}


def _uneven_instances(count):
    if count not in _UNEVEN:
        from paper_2510_04094_amd import workloads
        _UNEVEN[count] = workloads.mixed_batch(count=count)
    return _UNEVEN[count]


def pool_map(fn, jobs, procs):
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(procs) as pool:
            return pool.map(fn, jobs)
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


# The GPU host grants one GPU's share of its cores, 16, to a process, whatever the affinity
# mask shows; worker pools stay within that.
CPU_SHARE = 16


def host_cores():
    """(processes used, cores in the affinity mask)."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    return max(1, min(c, CPU_SHARE)), c


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


FAIL_BITS = 2 | 4 | 8 | 32  # singular, non-finite, eigensolver or refinement not converged


def status_summary(status):
    """Counts of each status bit over the batch, and the mask of instances without failures."""
    names = {1: "truncated", 2: "singular", 4: "nonfinite", 8: "eig_noconv", 16: "small_pivot",
             32: "refine_noconv", 64: "fp64_resolved"}
    counts = {v: int(np.count_nonzero(status & k)) for k, v in names.items()}
    return counts, (status & FAIL_BITS) == 0


def check_all(fn, jobs, procs):
    """Oracle comparison of every instance, in a process pool (one job per instance)."""
    return np.array(pool_map(fn, jobs, procs))


def run_mode(nyls, insts, mode, steps, warmup, tune):
    import torch
    b = nyls.Batch(insts, mode=mode)
    tuned = None
    if tune:
        # launch choices for this batch: coordinate search over nyls_tuning, timing nyls_solve
        from paper_2510_04094_amd import autotune
        res = autotune.autotune(b, reps=3, save=False, log=log)
        tuned = {"tuning": res["tuning"], "solve_ms": res["ms"], "default_solve_ms": res["default_ms"],
                 "candidates": len(res["tried"])}
    t_obs = [q["t_obs"] for q in insts]
    y_obs = torch.tensor(np.concatenate([q["y_obs"] for q in insts]), dtype=torch.float64, device="cuda")
    tt, oo, off = b._offsets(t_obs)
    cnt = torch.tensor(np.diff(off), dtype=torch.float64, device="cuda")
    inst_of = torch.repeat_interleave(torch.arange(b.batch, device="cuda"), torch.tensor(np.diff(off), device="cuda"))
    lib = nyls.load()
    dl = dict(
        dl_df=torch.zeros(nyls.MAX_P, b.total, dtype=torch.float64, device="cuda"),
        dl_dr=torch.zeros(b.total, dtype=torch.float64, device="cuda"),
        dl_dv=torch.zeros(b.batch, nyls.MAX_P, dtype=torch.float64, device="cuda"),
        dl_ds=torch.zeros(b.batch, dtype=torch.float64, device="cuda"),
        dl_dg=torch.zeros(b.batch, dtype=torch.float64, device="cuda"),
    )
    yobs_hat = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    P = nyls._ptr

    def step():
        out = b.solve()
        nyls._check(lib.nyls_predict(b.plan, P(tt), P(oo), 0, P(yobs_hat), P(b.ws), nyls._stream()), "predict")
        g = 2.0 * (yobs_hat - y_obs) / cnt[inst_of]           # d(mean squared error)/d y_hat
        nyls._check(lib.nyls_backward(b.plan, P(tt), P(oo), P(g), P(dl["dl_df"]), P(dl["dl_dr"]),
                                      P(dl["dl_dv"]), P(dl["dl_ds"]), P(dl["dl_dg"]), P(b.ws),
                                      nyls._stream()), "backward")
        return out

    for _ in range(warmup):
        out = step()
    torch.cuda.synchronize()
    nyls.profile_reset()
    nyls.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nyls.profile_enable(False)
    prof = nyls.profile_read()
    info = b.info().cpu().numpy()
    return b, out, (t1 - t0) / steps, prof, info, tuned


EXP_FLOP = 28.0  # flop per FP64 exponential implied by the per-pass figure below


def work_model(kernel, n, m, p, r, n_obs):
    """Algorithmic work of one instance in one launch of `kernel` (the method's work table):
      adjoint               1.6e7 flop at n = 5000, m = 50, p = 2, i.e. 64 flop per (point,
                            landmark) pair: the mu solve's residual pass plus the gradient pass;
      refinement + output   one FP64 per-point pass: n m exponentials + 2 n m (p+1) FMA
                            (2e7 flop at n = 1e4, m = 50, p = 2: an exponential counts
                            EXP_FLOP flop);
      operator Gram         |I| (m(m+1)/2 + 2m) FMA, |I| = n - p residual points;
      eigen                 9 m^3 flop;  KKT  2 m^2 r + (2/3)(r+1+p)^3 flop;
      predict               m (EXP_FLOP + 2 (p+1)) flop per observation time.
    Returns (flops, peak, bound)."""
    pairs = n * m
    fp64 = (PEAK["fp64"], "alu")
    if kernel == "backward":
        return 64.0 * pairs, fp64
    if kernel == "points":
        return pairs * (EXP_FLOP + 4.0 * (p + 1)), fp64
    if kernel in ("gram64", "gram32"):
        f = 2.0 * (n - p) * (m * (m + 1) / 2 + 2 * m)
        return f, ((PEAK["fp32_mfma"], "mfma") if kernel == "gram32" else (PEAK["fp64"], "mfma"))
    if kernel == "eig":
        return 9.0 * m ** 3, fp64
    if kernel == "kkt":
        return 2.0 * m * m * r + 2.0 / 3.0 * (r + 1 + p) ** 3, fp64
    if kernel == "predict":
        return m * (EXP_FLOP + 2.0 * (p + 1)) * n_obs, fp64
    return 0.0, fp64


def executed_model(kernel, n, m, p, passes_fw, passes_bw):
    """What the one-wave passes execute per instance, as multiply-adds per (point, landmark)
    pair once kernel values exist (they come from a two-exponential recurrence per 64
    points): refinement pass p + 3, adjoint mu pass p + 2, gradient pass 4p + 6; times the
    measured pass counts.  Returns flops (2 per multiply-add), or None for other kernels."""
    pairs = n * m
    if kernel == "backward":
        return 2.0 * pairs * ((4 * p + 6) + (p + 2) * passes_bw)
    if kernel == "points":
        return 2.0 * pairs * (p + 3) * passes_fw
    return None


def plain_fp64_rate(nyls, insts):
    """Reference-style per-instance FP64 solve (explicit features, library GEMM)."""
    import torch
    b = nyls.Batch(insts, mode=nyls.FP64_EXPLICIT)
    b.solve(refine=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.solve(refine=0)
    torch.cuda.synchronize()
    return len(insts) / (time.perf_counter() - t0)


def long_single_ms(nyls, steps=3):
    """One long-time instance (first-order family, n = 5e4 over [0, 20], m = 100, sigma = 0.3,
    FP64 mode, split over point chunks automatically): ms per nyls_solve and per nyls_backward
    (100 observation times), and the same unsplit.  Its parity with the oracle is a GPU test."""
    import torch
    from paper_2510_04094_amd import workloads
    q = workloads.linear_first_order(0, n=50000, m=100, t_end=20.0, sigma=0.3, tau=1e-10)
    tob = [np.linspace(0.1, 19.9, 100)]
    g = torch.full((100,), 1e-3, dtype=torch.float64, device="cuda")
    res = {}
    for name, split in (("split", -1), ("unsplit", 0)):
        b = nyls.Batch([q], mode=nyls.FP64, tuning=dict(split=split))
        b.solve()
        b.backward(tob, g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.solve()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            b.backward(tob, g)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res[name] = {"solve_ms": (t1 - t0) * 1e3 / steps, "backward_ms": (t2 - t1) * 1e3 / steps}
        del b
    return res


def long_time_wide_ms(nyls, steps=3):
    """The long-time shape of the paper's large-scale table: one second-order instance with
    n = 5e4 on [0, 100], m = 200 landmarks, sigma^2 = 1, gamma = 1e7 (FP64; a basis this wide
    is always split, two wavefronts per chunk).  ms per nyls_solve and per nyls_backward (100
    observations), and the solve's stages from the library's HIP-event timing.  Its parity
    with the oracle is a GPU test."""
    import torch
    from paper_2510_04094_amd import workloads
    q = workloads.linear_second_order(0, n=50000, m=200, t_end=100.0, sigma=1.0, tau=1e-8, obs=100)
    b = nyls.Batch([q], mode=nyls.FP64)
    tob = [q["t_obs"]]
    g = torch.full((100,), 1e-3, dtype=torch.float64, device="cuda")
    b.solve()
    b.backward(tob, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.solve()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        b.backward(tob, g)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    nyls.profile_reset()
    nyls.profile_enable(True)
    b.solve()
    torch.cuda.synchronize()
    nyls.profile_enable(False)
    prof = nyls.profile_read()
    info = b.info().cpu().numpy()
    return {"solve_ms": (t1 - t0) * 1e3 / steps, "backward_ms": (t2 - t1) * 1e3 / steps,
            "stage_ms": {k: v[0] for k, v in prof.items() if v[1]}, "rank": int(info[0, 0]),
            "refinement_passes": float(info[0, 5]), "n": 50000, "m": 200,
            "note": "second-order family on [0, 100], sigma = 1, FP64; solve, and adjoint for 100 "
                    "observations; stages overlap (the Gram runs beside the eigensolver)"}


def uneven_batch_rate(nyls, mode, count, steps, procs, check, tune):
    """Solves/s of the uneven batch (orders 1 and 2, n ~ U{500..1e4}, m in {20, 50, 100}),
    forward only, one nyls_solve captured in a HIP graph and replayed; every instance checked
    against the oracle (rel. 1e-6) after the timed replays."""
    import torch
    insts = _uneven_instances(count)
    b = nyls.Batch(insts, mode=mode)
    tuned = None
    if tune:
        from paper_2510_04094_amd import autotune
        r = autotune.autotune(b, reps=2, save=False, log=log)
        tuned = {"tuning": r["tuning"], "solve_ms": r["ms"], "default_solve_ms": r["default_ms"]}
    b.solve()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.solve()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = b.solve()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    counts, good = status_summary(out["status"].cpu().numpy())
    res = {"solves_per_s": None, "ms_per_step": sec * 1e3, "instances": count, "status_counts": counts,
           "orders": {"1": int(np.sum(b.p == 1)), "2": int(np.sum(b.p == 2))},
           "mean_n": float(np.mean(b.n)), "note": "forward only, nyls_solve replayed from a HIP graph",
           "autotune": tuned}
    if check:
        y = out["yhat"].cpu().numpy()
        errs = check_all(_oracle_err_uneven, [(i, count, y[b.goff[i]:b.goff[i + 1]]) for i in range(count)], procs)
        ok = good & (errs <= 1e-6)
        res.update(max_rel_err=float(errs.max()), frac_ok=float(np.mean(ok)))
        res["solves_per_s"] = float(np.sum(ok)) / sec
    else:
        res["solves_per_s"] = float(np.sum(good)) / sec
    del graph, b, out
    torch.cuda.empty_cache()
    return res


def newton_rate(nyls, count, steps, procs, check):
    """Lemma 2 Newton on the Riccati batch (count instances of y' = q - y^2, n = 2000, m = 50,
    sigma = 0.1, gamma = 1e6): whole solves (two Gauss-Newton steps, then Newton to
    |dx| <= 1e-12 max(1, |x|), the right-hand side evaluated on the device, one host check
    of the stopping test per step), every instance checked against the oracle after the same
    number of steps."""
    import torch
    from paper_2510_04094_amd import workloads
    insts = [workloads.riccati(i) for i in range(count)]
    b = nyls.Batch(insts, mode=nyls.FP64)
    q = torch.tensor(np.concatenate([p["q"] for p in insts]), dtype=torch.float64, device="cuda")
    b.riccati_newton(q, max_iter=15, tol=1e-12, gauss_newton_steps=2)
    torch.cuda.synchronize()
    nyls.profile_reset()
    nyls.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        x, hist = b.riccati_newton(q, max_iter=15, tol=1e-12, gauss_newton_steps=2)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    nyls.profile_enable(False)
    prof = nyls.profile_read()
    iters = int(hist.shape[0])
    res = {"instances": count, "n": 2000, "m": 50, "ms_per_batch_solve": sec * 1e3, "newton_steps": iters,
           "solves_per_s": count / sec,
           "newton_step_kernel_ms": prof["newton"][0] / max(prof["newton"][1], 1),
           "note": "Riccati y' = q - y^2; whole Newton solves with a host stopping test per step"}
    if check:
        yh, off = b.predict([p["t"] for p in insts], 0)
        yh = yh.cpu().numpy()
        errs = check_all(_oracle_err_newton, [(i, iters, yh[off[i]:off[i + 1]]) for i in range(count)], procs)
        res["max_rel_err"] = float(errs.max())
    del b
    torch.cuda.empty_cache()
    return res


def legs(nyls, line, args, procs, insts):
    """The bench's legs beside the headline step (uneven batch, Newton, plain comparator,
    long single instances), each added to the line under its own key."""
    if args.uneven > 0:
        log("uneven batch")
        line["uneven_batch"] = {name: uneven_batch_rate(nyls, {"fp64": nyls.FP64, "mixed": nyls.MIXED}[name],
                                                        args.uneven, args.steps, procs, args.check, args.tune)
                                for name in args.modes.split(",")}
    if args.newton > 0:
        log("Newton leg")
        line["newton_riccati"] = newton_rate(nyls, args.newton, args.steps, procs, args.check)
    if args.plain > 0:
        log("plain per-instance FP64 solve")
        line["plain_fp64_per_instance"] = {"solves_per_s": plain_fp64_rate(nyls, insts[:args.plain]),
                                           "instances": args.plain, "note": "forward only"}
    if args.long:
        log("long single instances")
        line["long_single_instance"] = dict(long_single_ms(nyls), n=50000, m=100,
                                            note="first-order family on [0, 20], FP64; solve, and adjoint "
                                                 "for 100 observations")
        line["long_time_m200"] = long_time_wide_ms(nyls)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--m", type=int, default=50)
    ap.add_argument("--modes", default="fp64,mixed")
    ap.add_argument("--check", type=int, default=1, help="1: check every instance against the oracle")
    ap.add_argument("--tune", type=int, default=1, help="1: autotune the launch choices of each mode first")
    ap.add_argument("--plain", type=int, default=32, help="instances for the plain FP64 comparator")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle instances per timed run (0: 6 per process)")
    ap.add_argument("--cpu-runs", type=int, default=5, help="timed CPU runs (median reported)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--long", type=int, default=1,
                    help="time long single instances (n = 5e4, m = 100; and m = 200 on [0, 100])")
    ap.add_argument("--uneven", type=int, default=4096, help="instances of the uneven-batch leg (0: skip)")
    ap.add_argument("--newton", type=int, default=64, help="instances of the Newton (Riccati) leg (0: skip)")
    ap.add_argument("--headline", type=int, default=1,
                    help="0: skip the headline step (profiling runs of the other legs; the line "
                         "then holds only those legs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the batch is data-parallel over independent "
              "instances and the library runs on a single MI355X; use --gpus 1.")
        sys.exit(2)

    import torch
    from paper_2510_04094_amd import nyls
    nyls.load()
    torch.cuda.set_device(0)
    seed_config = 2
    procs, affinity = host_cores()
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.headline:
        line = {"headline": "skipped (--headline 0)"}
        legs(nyls, line, args, procs,
             make_instances(args.plain, args.n, args.m, seed_config) if args.plain > 0 else [])
        print(json.dumps(line))
        return
    insts = make_instances(args.batch, args.n, args.m, seed_config)

    results = {}
    for name in args.modes.split(","):
        mode = {"fp64": nyls.FP64, "mixed": nyls.MIXED}[name]
        b, out, sec, prof, info, tuned = run_mode(nyls, insts, mode, args.steps, args.warmup, args.tune)
        log("%s: %.2f ms per step; checking every instance against the oracle" % (name, sec * 1e3))
        counts, good = status_summary(out["status"].cpu().numpy())
        # every instance's y_hat against the oracle, after the timed steps (--check 0 skips
        # it for profiling runs; such a line counts instances by their status bits alone and
        # says so with max_rel_err = null).  Nothing the oracle computes reaches the GPU path.
        if args.check:
            y = out["yhat"].cpu().numpy()
            errs = check_all(_oracle_err, [(i, args.n, args.m, seed_config, y[b.goff[i]:b.goff[i + 1]])
                                           for i in range(args.batch)], procs)
            ok = good & (errs <= 1e-6)
            max_err = float(errs.max())
            above = {"count_above_1e-10": int(np.sum(errs > 1e-10)),
                     "worst_instances": [int(i) for i in np.argsort(-errs)[:5]]}
            if name == "fp64" and above["count_above_1e-10"]:
                # instances above 1e-10 are held to the oracle's own FP64 floor (K_mm
                # rounding and eigensolver backward error near the cut-off)
                hi = [int(i) for i in np.nonzero(errs > 1e-10)[0]]
                log("fp64: %d instances above 1e-10; computing their FP64 floor bars" % len(hi))
                bars = np.array(pool_map(_floor_bar, [(i, args.n, args.m, seed_config) for i in hi], procs))
                above["count_above_floor_bar"] = int(np.sum(errs[hi] > bars))
                above["max_err_over_bar"] = float(np.max(errs[hi] / bars))
        else:
            ok, max_err, above = good, None, None
        results[name] = dict(sec=sec, prof=prof, max_err=max_err, frac_ok=float(np.mean(ok)), above=above, tuned=tuned,
                             n_ok=int(np.sum(ok)), status=counts,
                             rate=float(np.sum(ok)) / sec, rank=float(info[:, 0].mean()),
                             passes_fw=float(info[:, 5].mean()), passes_bw=float(info[:, 6].mean()),
                             sweeps=float(info[:, 2].mean()))
        del b, out
        torch.cuda.empty_cache()

    best = max(results, key=lambda k: results[k]["rate"])
    r = results[best]
    prof = r["prof"]
    # dominant kernel of the step: algorithmic work of one launch / its average duration
    # (HIP events on the stream the kernels run on)
    kname = max(prof, key=lambda k: prof[k][0] / max(prof[k][1], 1) * (prof[k][1] > 0))
    kms, kcnt = prof[kname]
    avg_s = kms / max(kcnt, 1) / 1e3
    n_obs = 100
    flops_inst, (peak, bound) = work_model(kname, args.n, args.m, 2, r["rank"], n_obs)
    flops = flops_inst * args.batch
    achieved = flops / avg_s
    roofline = {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(kname, best, args.batch),
                "kernel": kname, "kernel_ms": avg_s * 1e3, "flops_per_launch": flops}
    ex = executed_model(kname, args.n, args.m, 2, r["passes_fw"], r["passes_bw"])
    if ex is not None:
        roofline["executed_fma_model"] = {
            "frac": ex * args.batch / avg_s / peak,
            "flops_per_launch": ex * args.batch,
            "passes": {"refinement": r["passes_fw"], "adjoint_refinement": r["passes_bw"]},
            "note": "multiply-adds the passes execute per (point, landmark) pair times the "
                    "measured pass counts; not the method's algorithmic work"}

    line = {
        "metric": "ODE solves/s at n=1e4,m=50 (batched+adjoint vs plain FP64) at rel err<=1e-6",
        "value": r["rate"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batch of %d linear 2nd-order ODEs, n=%d, m=%d, sigma~U(0.2,1), "
                               "gamma=1e7, tau=1e-8, 100 observations; forward + adjoint" % (args.batch, args.n, args.m),
                   "global_batch": args.batch, "seq_len": args.n, "parallelism": "none (1 GPU)",
                   "mode": best},
        "roofline": roofline,
        "modes": {k: {"solves_per_s": v["rate"], "ms_per_step": v["sec"] * 1e3, "max_rel_err": v["max_err"],
                      "frac_ok": v["frac_ok"], "instances_ok": v["n_ok"], "checked": "all" if args.check else "status only",
                      "errors": v["above"],
                      "status_counts": v["status"], "mean_rank": v["rank"], "mean_sweeps": v["sweeps"],
                      "refinement_passes": v["passes_fw"], "adjoint_passes": v["passes_bw"],
                      "autotune": v["tuned"],
                      "kernel_ms": {kk: vv[0] / max(vv[1], 1) for kk, vv in v["prof"].items() if vv[1]}}
                  for k, v in results.items()},
    }
    legs(nyls, line, args, procs, insts)
    if not args.no_cpu:
        log("CPU oracle baseline")
        count = args.cpu_sample or 6 * procs
        rates, cpu_s = [], []
        pool_map(_oracle_job, [(i, args.n, args.m, seed_config) for i in range(procs)], procs)  # warm-up
        for run in range(args.cpu_runs):
            t0 = time.perf_counter()
            times = pool_map(_oracle_job, [(run * count + i, args.n, args.m, seed_config) for i in range(count)],
                             procs)
            rates.append(count / (time.perf_counter() - t0))
            cpu_s.append(float(np.sum(times)))
        line["cpu_baseline"] = {"value": float(np.median(rates)), "unit": "solves/s", "cores": procs,
                                "kind": "oracle",
                                "sample": "median of %d runs, each %d instances of the same workload "
                                          "(forward + adjoint, about %.0f s CPU), NumPy FP64, one "
                                          "single-threaded process per core; %d processes on %s "
                                          "(%d cores in the affinity mask, %d granted per GPU)"
                                          % (args.cpu_runs, count, float(np.median(cpu_s)), procs,
                                             cpu_model(), affinity, CPU_SHARE)}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
