"""Python binding of libnyls.so (C ABI in include/nyls.h).

Argument marshalling only: device memory comes from torch tensors, work is enqueued
on torch's current HIP stream, and every computation runs in the library's kernels.
The library must be built (python -m paper_2510_04094_amd.build); nothing here falls
back to another implementation.
"""
import ctypes
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnyls.so")
MAX_P = 4
MAX_M = 256
MAX_N = 1 << 25

FP64, MIXED, FP64_EXPLICIT = 0, 1, 2
S_TRUNCATED, S_SINGULAR, S_NONFINITE, S_EIG_NOCONV, S_SMALL_PIVOT, S_REFINE_NOCONV = 1, 2, 4, 8, 16, 32
S_FP64_RESOLVED = 64
S_PARAM_KEPT = 128
S_PIVOT_OVERFLOW = 256

_lib = None


class NylsError(RuntimeError):
    pass


class Problem(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
        ("uniform", ctypes.c_int32),
        ("t0", ctypes.c_double), ("dt", ctypes.c_double),
        ("t", ctypes.c_void_p), ("lidx", ctypes.c_void_p),
        ("f", ctypes.c_void_p), ("r", ctypes.c_void_p), ("v", ctypes.c_void_p),
        ("cond_d", ctypes.c_int32 * MAX_P), ("cond_i", ctypes.c_int32 * MAX_P),
        ("sigma", ctypes.c_double), ("gamma", ctypes.c_double), ("tau", ctypes.c_double),
    ]


class Tuning(ctypes.Structure):
    """nyls_tuning: the plan's launch choices (include/nyls.h)."""
    _fields_ = [("eig_ql", ctypes.c_int32), ("ql_lanes", ctypes.c_int32), ("gram_valu", ctypes.c_int32),
                ("tail_layout", ctypes.c_int32), ("overlap", ctypes.c_int32), ("split", ctypes.c_int32)]


TUNING_FIELDS = tuple(name for name, _ in Tuning._fields_)
DEFAULT_TUNING = dict(eig_ql=0, ql_lanes=64, gram_valu=0, tail_layout=1, overlap=1, split=-1)


EXPORTS = {
    "nyls_plan_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_plan_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "nyls_plan_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "nyls_plan_destroy": (None, [ctypes.c_void_p]),
    "nyls_workspace_size": (ctypes.c_size_t, [ctypes.c_void_p]),
    "nyls_total_points": (ctypes.c_int64, [ctypes.c_void_p]),
    "nyls_max_m": (ctypes.c_int32, [ctypes.c_void_p]),
    "nyls_instance_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_basis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "nyls_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "nyls_assemble": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "nyls_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "nyls_solve_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_newton_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "nyls_newton_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_newton_state_stride": (ctypes.c_int64, [ctypes.c_void_p]),
    "nyls_newton_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "nyls_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_riccati_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_leverage_scores": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "nyls_leverage_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_profile_enable": (None, [ctypes.c_int32]),
    "nyls_profile_read": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "nyls_profile_reset": (None, []),
    "nyls_error_string": (ctypes.c_char_p, [ctypes.c_int32]),
}

KERNELS = ["eig", "gram64", "gram32", "kkt", "points", "features", "predict", "explicit",
           "newton", "backward"]


def profile_enable(on=True):
    load().nyls_profile_enable(1 if on else 0)


def profile_reset():
    load().nyls_profile_reset()


def profile_read():
    """{kernel name: (total ms, launches)} of the kernel timing since the last reset."""
    lib = load()
    out = {}
    for k, name in enumerate(KERNELS):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib.nyls_profile_read(k, ctypes.byref(ms), ctypes.byref(cnt)), "nyls_profile_read")
        out[name] = (ms.value, cnt.value)
    return out


def load(path=LIB_PATH):
    """Load the HIP library; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise NylsError("libnyls.so not built: run `python -m paper_2510_04094_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc, what):
    if rc != 0:
        raise NylsError("%s failed: %d (%s)" % (what, rc, _lib.nyls_error_string(rc).decode()))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Batch:
    """A batch of ODE instances resident on the GPU plus the library plan over them.

    `instances` are dicts as produced by paper_2510_04094_amd.workloads (numpy arrays);
    their coefficient, forcing and condition data are packed into device tensors that
    the plan points into.  `mode` is FP64, MIXED or FP64_EXPLICIT.
    """

    def __init__(self, instances, mode=FP64, device="cuda", explicit_grid=False, tuning=None):
        """explicit_grid: pass every grid as its time array (nyls_problem.uniform = 0)
        instead of (t0, dt).  tuning: None (the library's defaults), a dict of nyls_tuning
        fields, or "cached" (the autotuner's cached choice for this batch's key, defaults
        when there is none)."""
        lib = load()
        self.mode = mode
        self.device = torch.device(device)
        self.instances = instances
        nb = len(instances)
        ns = np.array([int(q["n"]) for q in instances], dtype=np.int64)
        ps = np.array([int(q["p"]) for q in instances], dtype=np.int64)
        self.n = ns
        self.p = ps
        self.m = np.array([int(q["m"]) for q in instances], dtype=np.int64)
        self.goff = np.concatenate([[0], np.cumsum(ns)])
        fo = np.concatenate([[0], np.cumsum(ns * ps)])
        has_lin = all(("f" in q and "r" in q) for q in instances)
        f_host = np.zeros(int(fo[-1]))
        r_host = np.zeros(int(self.goff[-1]))
        v_host = np.zeros(nb * MAX_P)
        for i, q in enumerate(instances):
            if has_lin:
                f_host[fo[i]:fo[i + 1]] = np.asarray(q["f"], dtype=np.float64).reshape(-1)
                r_host[self.goff[i]:self.goff[i + 1]] = np.asarray(q["r"], dtype=np.float64)
            v_host[i * MAX_P:i * MAX_P + ps[i]] = np.asarray(q["v"], dtype=np.float64)
        self.f = torch.tensor(f_host, dtype=torch.float64, device=self.device)
        self.r = torch.tensor(r_host, dtype=torch.float64, device=self.device)
        self.v = torch.tensor(v_host, dtype=torch.float64, device=self.device)
        self.t = None
        if explicit_grid:
            self.t = torch.tensor(np.concatenate([np.asarray(q["t"], dtype=np.float64) for q in instances]),
                                  dtype=torch.float64, device=self.device)
        self._foff = fo
        self._lidx_host = []
        probs = (Problem * nb)()
        for i, q in enumerate(instances):
            pr = probs[i]
            pr.p, pr.n, pr.m = int(q["p"]), int(q["n"]), int(q["m"])
            pr.t0, pr.dt = float(q["t0"]), float(q["dt"])
            if explicit_grid:
                pr.uniform = 0
                pr.t = self.t.data_ptr() + 8 * int(self.goff[i])
            else:
                pr.uniform = 1
                pr.t = None
            if q.get("lidx") is not None:
                arr = (ctypes.c_int32 * pr.m)(*[int(x) for x in q["lidx"]])
                self._lidx_host.append(arr)
                pr.lidx = ctypes.cast(arr, ctypes.c_void_p)
            else:
                pr.lidx = None
            if has_lin:
                pr.f = self.f.data_ptr() + 8 * int(fo[i])
                pr.r = self.r.data_ptr() + 8 * int(self.goff[i])
            else:
                pr.f = None
                pr.r = None
            pr.v = self.v.data_ptr() + 8 * i * MAX_P
            for j in range(MAX_P):
                pr.cond_d[j] = int(q["cond_d"][j]) if j < pr.p else 0
                pr.cond_i[j] = int(q["cond_i"][j]) if j < pr.p else 0
            pr.sigma, pr.gamma, pr.tau = float(q["sigma"]), float(q["gamma"]), float(q["tau"])
        self._probs = probs
        handle = ctypes.c_void_p()
        _check(lib.nyls_plan_create(ctypes.cast(probs, ctypes.c_void_p), nb, mode, ctypes.byref(handle)),
               "nyls_plan_create")
        self.plan = handle
        self.batch = nb
        self.maxm = int(lib.nyls_max_m(handle))
        self.total = int(lib.nyls_total_points(handle))
        nbytes = int(lib.nyls_workspace_size(handle))
        self.ws = torch.zeros(max(nbytes, 8), dtype=torch.uint8, device=self.device)
        # bumped by every call that leaves a new basis / factorisation / solution in ws
        self.ws_version = 0
        if tuning == "cached":
            from . import autotune
            tuning = autotune.lookup(autotune.batch_key(self))
        if tuning:
            self.set_tuning(**tuning)

    def get_tuning(self):
        t = Tuning()
        _check(_lib.nyls_plan_get_tuning(self.plan, ctypes.byref(t)), "nyls_plan_get_tuning")
        return {k: int(getattr(t, k)) for k in TUNING_FIELDS}

    def set_tuning(self, **fields):
        """nyls_plan_set_tuning with the given fields changed (host call; no work of this
        plan may be in flight)."""
        cur = self.get_tuning()
        for k, v in fields.items():
            if k not in cur:
                raise NylsError("unknown tuning field %r" % k)
            cur[k] = int(v)
        t = Tuning(**cur)
        _check(_lib.nyls_plan_set_tuning(self.plan, ctypes.byref(t)), "nyls_plan_set_tuning")
        # the workspace size depends on the split choice: grow it when needed (its contents
        # are rebuilt by the next solve)
        nbytes = int(_lib.nyls_workspace_size(self.plan))
        if nbytes > self.ws.numel():
            self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
            self.ws_version += 1

    def __del__(self):
        if getattr(self, "plan", None) is not None and _lib is not None:
            _lib.nyls_plan_destroy(self.plan)
            self.plan = None

    # --- per-instance views of flat outputs ---------------------------------------
    def split_points(self, flat):
        return [flat[self.goff[i]:self.goff[i + 1]] for i in range(self.batch)]

    # --- work functions -------------------------------------------------------------
    def solve(self, refine=None):
        """nyls_solve: returns dict(yhat [total], omega [batch, maxm], bias, lam, status)."""
        if refine is None:
            refine = 4 if self.mode != FP64_EXPLICIT else 0
        dev = self.device
        out = dict(
            yhat=torch.empty(self.total, dtype=torch.float64, device=dev),
            omega=torch.empty(self.batch, self.maxm, dtype=torch.float64, device=dev),
            bias=torch.empty(self.batch, dtype=torch.float64, device=dev),
            lam=torch.empty(self.batch, MAX_P, dtype=torch.float64, device=dev),
            status=torch.empty(self.batch, dtype=torch.int32, device=dev),
        )
        _check(_lib.nyls_solve(self.plan, refine, _ptr(out["omega"]), _ptr(out["bias"]), _ptr(out["lam"]),
                               _ptr(out["yhat"]), _ptr(out["status"]), _ptr(self.ws), _stream()),
               "nyls_solve")
        self.ws_version += 1
        return out

    def solve_static(self, refine=None):
        """nyls_solve_static: the solve with the library's own device workspace (no
        allocation inside the call); same outputs as solve().  Leaves self.ws untouched."""
        if refine is None:
            refine = 4
        dev = self.device
        out = dict(
            yhat=torch.empty(self.total, dtype=torch.float64, device=dev),
            omega=torch.empty(self.batch, self.maxm, dtype=torch.float64, device=dev),
            bias=torch.empty(self.batch, dtype=torch.float64, device=dev),
            lam=torch.empty(self.batch, MAX_P, dtype=torch.float64, device=dev),
            status=torch.empty(self.batch, dtype=torch.int32, device=dev),
        )
        _check(_lib.nyls_solve_static(self.plan, refine, _ptr(out["omega"]), _ptr(out["bias"]),
                                      _ptr(out["lam"]), _ptr(out["yhat"]), _ptr(out["status"]),
                                      _stream()), "nyls_solve_static")
        return out

    def assemble(self):
        kn = self.maxm + 1 + MAX_P
        kkt = torch.zeros(self.batch, kn * kn, dtype=torch.float64, device=self.device)
        rhs = torch.zeros(self.batch, kn, dtype=torch.float64, device=self.device)
        _check(_lib.nyls_assemble(self.plan, _ptr(kkt), _ptr(rhs), _ptr(self.ws), _stream()), "nyls_assemble")
        self.ws_version += 1
        return kkt, rhs

    def _offsets(self, t_eval_list):
        """Device copies of per-instance evaluation times and their offsets.  The last few
        time sets are kept on the device, so repeated calls with the same times (a training
        loop, a graph capture after an eager warm-up) copy nothing from the host."""
        counts = [len(t) for t in t_eval_list]
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        host = np.concatenate([np.asarray(x, dtype=np.float64) for x in t_eval_list])
        key = (host.tobytes(), off.tobytes())
        cache = self.__dict__.setdefault("_offset_cache", {})
        hit = cache.get(key)
        if hit is not None:
            return hit[0], hit[1], off
        t = torch.tensor(host, dtype=torch.float64, device=self.device)
        o = torch.tensor(off, dtype=torch.int64, device=self.device)
        if len(cache) >= 8:
            cache.pop(next(iter(cache)))
        cache[key] = (t, o)
        return t, o, off

    def features(self, t_eval_list, dmax):
        """nyls_features at per-instance times: returns (phi [E, dmax+1, maxm], eigval, rank, offsets)."""
        t, o, off = self._offsets(t_eval_list)
        phi = torch.empty(int(off[-1]), dmax + 1, self.maxm, dtype=torch.float64, device=self.device)
        eig = torch.empty(self.batch, self.maxm, dtype=torch.float64, device=self.device)
        rank = torch.empty(self.batch, dtype=torch.int32, device=self.device)
        _check(_lib.nyls_features(self.plan, _ptr(t), _ptr(o), dmax, _ptr(phi), _ptr(eig), _ptr(rank),
                                  _ptr(self.ws), _stream()), "nyls_features")
        self.ws_version += 1
        return phi, eig, rank, off

    def predict(self, t_eval_list, d=0):
        t, o, off = self._offsets(t_eval_list)
        out = torch.empty(int(off[-1]), dtype=torch.float64, device=self.device)
        _check(_lib.nyls_predict(self.plan, _ptr(t), _ptr(o), d, _ptr(out), _ptr(self.ws), _stream()),
               "nyls_predict")
        return out, off

    # --- landmark sampling ---------------------------------------------------------------
    def leverage_scores(self, ridge=0.0):
        """nyls_leverage_scores: ridge leverage scores [total] of every grid point in the
        feature space of this plan's basis (ridge 0: 1/gamma per instance)."""
        out = torch.empty(self.total, dtype=torch.float64, device=self.device)
        _check(_lib.nyls_leverage_scores(self.plan, float(ridge), _ptr(out), _ptr(self.ws), _stream()),
               "nyls_leverage_scores")
        self.ws_version += 1
        return out

    def leverage_landmarks(self, uniforms, ends=True, ridge=0.0):
        """Leverage-score landmarks of every instance (nyls_leverage_scores, then
        nyls_leverage_sample with the caller's uniforms [total] or per-instance list):
        returns (scores, list of ascending int64 index arrays) for new instances' lidx."""
        scores = self.leverage_scores(ridge)
        if not torch.is_tensor(uniforms):
            uniforms = torch.tensor(np.concatenate([np.asarray(u, dtype=np.float64) for u in uniforms]),
                                    dtype=torch.float64, device=self.device)
        lidx = torch.empty(self.batch, self.maxm, dtype=torch.int32, device=self.device)
        _check(_lib.nyls_leverage_sample(self.plan, _ptr(scores), _ptr(uniforms.contiguous()),
                                         1 if ends else 0, _ptr(lidx), _stream()), "nyls_leverage_sample")
        host = lidx.cpu().numpy()
        return scores, [host[i, :int(self.m[i])].astype(np.int64) for i in range(self.batch)]

    # --- nonlinear (Lemma 2) -----------------------------------------------------------
    def newton_init(self):
        """nyls_newton_init: returns the state tensor x [batch, stride]."""
        stride = int(_lib.nyls_newton_state_stride(self.plan))
        x = torch.zeros(self.batch, stride, dtype=torch.float64, device=self.device)
        _check(_lib.nyls_newton_init(self.plan, _ptr(x), _ptr(self.ws), _stream()), "nyls_newton_init")
        self.ws_version += 1
        self._newton_bufs = [torch.empty(self.total, dtype=torch.float64, device=self.device) for _ in range(3)]
        self._step_inf = torch.empty(self.batch, dtype=torch.float64, device=self.device)
        self._status = torch.empty(self.batch, dtype=torch.int32, device=self.device)
        return x

    def newton_step(self, x, F, dF, d2F):
        """nyls_newton_step with caller-evaluated F [total], dF [p, total], d2F [p, p, total]
        (contiguous; for first-order plans Fy and Fyy [total]); returns step_inf [batch]."""
        _check(_lib.nyls_newton_step(self.plan, _ptr(F), _ptr(dF), _ptr(d2F), _ptr(x), _ptr(self._step_inf),
                                     _ptr(self._status), _ptr(self.ws), _stream()), "nyls_newton_step")
        self.ws_version += 1
        return self._step_inf

    def newton_state(self, x):
        """nyls_newton_state: u [p, total] with u[0] = y_i and, for p = 2, u[1] = y_hat'(t_i)."""
        p = int(self.p.max())
        u = torch.empty(p, self.total, dtype=torch.float64, device=self.device)
        _check(_lib.nyls_newton_state(self.plan, _ptr(x), _ptr(u), _ptr(self.ws), _stream()),
               "nyls_newton_state")
        return u

    def newton_solve(self, fun, max_iter=30, tol=1e-12, gauss_newton_steps=5):
        """Newton on y^(p) = F(t, y, .., y^(p-1)) for every instance.  fun(u, gauss_newton)
        maps the state values u [p, total] (nyls_newton_state) to (F [total], dF [p, total],
        d2F [p, p, total]) on the device; the first `gauss_newton_steps` steps pass zero
        second derivatives (Gauss-Newton).  Stops when every instance's |dx|_inf <= tol *
        max(1, |x|_inf).  Returns (x, steps [iters, batch])."""
        x = self.newton_init()
        hist = []
        for k in range(max_iter):
            F, dF, d2F = fun(self.newton_state(x), k < gauss_newton_steps)
            if k < gauss_newton_steps:
                d2F = torch.zeros_like(d2F)
            si = self.newton_step(x, F.contiguous(), dF.contiguous(), d2F.contiguous()).clone()
            hist.append(si)
            xinf = torch.clamp(torch.max(torch.abs(x), dim=1).values, min=1.0)
            if bool(torch.all(si <= tol * xinf)):
                break
        return x, torch.stack(hist)

    def riccati_eval(self, q, x, gauss_newton):
        F, Fy, Fyy = self._newton_bufs
        _check(_lib.nyls_riccati_eval(self.plan, _ptr(q), _ptr(x), 1 if gauss_newton else 0, _ptr(F), _ptr(Fy),
                                      _ptr(Fyy), _stream()), "nyls_riccati_eval")
        return F, Fy, Fyy

    def riccati_newton(self, q, max_iter=15, tol=1e-12, gauss_newton_steps=2):
        """Newton on y' = q(t) - y^2 for every instance: the first `gauss_newton_steps`
        steps use the Gauss-Newton y-block, then exact Newton; stops when every instance's
        |dx|_inf <= tol * max(1, |x|_inf).  Returns (x, steps [iters, batch])."""
        x = self.newton_init()
        hist = []
        for k in range(max_iter):
            F, Fy, Fyy = self.riccati_eval(q, x, k < gauss_newton_steps)
            si = self.newton_step(x, F, Fy, Fyy).clone()
            hist.append(si)
            xinf = torch.clamp(torch.max(torch.abs(x), dim=1).values, min=1.0)
            if bool(torch.all(si <= tol * xinf)):
                break
        return x, torch.stack(hist)

    # --- adjoint --------------------------------------------------------------------------
    def set_params(self, sigma=None, gamma=None):
        """Change per-instance sigma and/or gamma ([batch] host arrays): rebuilds the plan
        (host validation, which may change the recurrence choice, and descriptor upload) and
        keeps its tuning."""
        lib = load()
        tuning = self.get_tuning()
        for i in range(self.batch):
            if sigma is not None:
                self._probs[i].sigma = float(sigma[i])
            if gamma is not None:
                self._probs[i].gamma = float(gamma[i])
        handle = ctypes.c_void_p()
        _check(lib.nyls_plan_create(ctypes.cast(self._probs, ctypes.c_void_p), self.batch, self.mode,
                                    ctypes.byref(handle)), "nyls_plan_create")
        lib.nyls_plan_destroy(self.plan)
        self.plan = handle
        self.set_tuning(**tuning)

    def set_params_device(self, sigma=None, gamma=None):
        """nyls_plan_set_params: sigma and/or gamma from device tensors [batch] (float64),
        without a host synchronisation (capturable).  Returns the int32 status tensor:
        S_PARAM_KEPT where a value was not taken (see the header)."""
        status = torch.empty(self.batch, dtype=torch.int32, device=self.device)
        args = []
        for x in (sigma, gamma):
            if x is None:
                args.append(None)
            else:
                x = x.to(device=self.device, dtype=torch.float64).reshape(-1).contiguous()
                if x.numel() != self.batch:
                    raise NylsError("set_params_device: expected %d values" % self.batch)
                args.append(x)
        self._param_args = args  # keep the tensors alive until the kernel has read them
        _check(_lib.nyls_plan_set_params(self.plan, _ptr(args[0]), _ptr(args[1]), _ptr(status), _stream()),
               "nyls_plan_set_params")
        if sigma is not None or gamma is not None:
            self._params_on_device = True
        return status

    def params(self):
        """Per-instance (sigma, gamma) of the last host-side setting, as numpy arrays (values
        set with set_params_device live on the device only)."""
        return (np.array([self._probs[i].sigma for i in range(self.batch)]),
                np.array([self._probs[i].gamma for i in range(self.batch)]))

    def f_index(self):
        """Index of every entry of the flat coefficient array f (instance blocks [p][n]) in the
        flattened [4][total points] layout of nyls_backward's dl/df."""
        if getattr(self, "_fidx", None) is None:
            parts = []
            for i in range(self.batch):
                p, n, g0 = int(self.p[i]), int(self.n[i]), int(self.goff[i])
                k = np.arange(p)[:, None]
                parts.append((k * self.total + g0 + np.arange(n)[None, :]).reshape(-1))
            self._fidx = torch.tensor(np.concatenate(parts), dtype=torch.int64, device=self.device)
        return self._fidx

    def info(self):
        """[batch][8] diagnostics (rank, status, sweeps, last refinement change, Gram basis,
        refinement passes of solve and of backward), as a float64 device tensor."""
        out = torch.zeros(self.batch, 8, dtype=torch.float64, device=self.device)
        _check(_lib.nyls_instance_info(self.plan, _ptr(self.ws), _ptr(out), _stream()), "nyls_instance_info")
        return out

    def basis(self):
        """nyls_basis after a call that formed the basis: (lam [batch][maxm],
        U [batch][maxm][maxm]) as float64 device tensors, K_mm = U diag(lam) U^T."""
        lam = torch.empty(self.batch, self.maxm, dtype=torch.float64, device=self.device)
        u = torch.empty(self.batch, self.maxm, self.maxm, dtype=torch.float64, device=self.device)
        _check(_lib.nyls_basis(self.plan, _ptr(self.ws), _ptr(lam), _ptr(u), _stream()), "nyls_basis")
        return lam, u

    def backward(self, t_obs_list, g_obs_list):
        """nyls_backward after solve(): gradients of a loss with dl/dy_hat(s_j) = g_j."""
        t, o, off = self._offsets(t_obs_list)
        if torch.is_tensor(g_obs_list):
            g = g_obs_list.to(device=self.device, dtype=torch.float64).contiguous()
        else:
            g = torch.tensor(np.concatenate([np.asarray(x, dtype=np.float64) for x in g_obs_list]),
                             dtype=torch.float64, device=self.device)
        dev = self.device
        out = dict(
            dl_df=torch.zeros(MAX_P, self.total, dtype=torch.float64, device=dev),
            dl_dr=torch.zeros(self.total, dtype=torch.float64, device=dev),
            dl_dv=torch.zeros(self.batch, MAX_P, dtype=torch.float64, device=dev),
            dl_dsigma=torch.zeros(self.batch, dtype=torch.float64, device=dev),
            dl_dgamma=torch.zeros(self.batch, dtype=torch.float64, device=dev),
        )
        _check(_lib.nyls_backward(self.plan, _ptr(t), _ptr(o), _ptr(g), _ptr(out["dl_df"]), _ptr(out["dl_dr"]),
                                  _ptr(out["dl_dv"]), _ptr(out["dl_dsigma"]), _ptr(out["dl_dgamma"]),
                                  _ptr(self.ws), _stream()), "nyls_backward")
        return out


class SolveAtObservations(torch.autograd.Function):
    """y_hat at observation times as a differentiable function of the ODE data.

    forward(batch, t_obs_list, f, r, v, sigma, gamma) -> y_obs [sum of observation counts]
      f [sum p_i n_i] (instance blocks [p][n], the layout of Batch.f), r [total points],
      v [batch, 4] (condition values, zero-padded), sigma [batch], gamma [batch].
    The values are written into the batch's device arrays and sigma / gamma into the plan's
    device descriptors (nyls_plan_set_params, no host synchronisation), then nyls_solve and
    nyls_predict run; backward calls nyls_backward, which reuses the factorisation, and maps
    dl/df, dl/dr, dl/dv, dl/dsigma, dl/dgamma onto the inputs.  Forward and backward can be
    captured in a HIP graph with static input tensors.
    """

    @staticmethod
    def _load_and_solve(batch, f, r, v, sigma, gamma):
        with torch.no_grad():
            batch.f.copy_(f.detach().reshape(-1))
            batch.r.copy_(r.detach().reshape(-1))
            batch.v.copy_(v.detach().reshape(-1))
            # sigma and gamma go to the plan's descriptors on the device (no host round trip,
            # so forward and backward can be captured in a graph); outside a capture a value
            # the device update refuses (a sigma that breaks the plan's recurrence choice) is
            # taken by rebuilding the plan instead
            status = batch.set_params_device(sigma.detach(), gamma.detach())
            if not torch.cuda.is_current_stream_capturing() and bool(torch.any(status != 0)):
                batch.set_params(sigma=sigma.detach().cpu().numpy(), gamma=gamma.detach().cpu().numpy())
            batch.solve()
        return batch.ws_version

    @staticmethod
    def forward(ctx, batch, t_obs_list, f, r, v, sigma, gamma):
        ctx.ws_version = SolveAtObservations._load_and_solve(batch, f, r, v, sigma, gamma)
        with torch.no_grad():
            y, _ = batch.predict(t_obs_list, 0)
        ctx.batch = batch
        ctx.t_obs_list = t_obs_list
        ctx.shapes = (f.shape, r.shape, v.shape)
        ctx.save_for_backward(f.detach(), r.detach(), v.detach(), sigma.detach(), gamma.detach())
        return y

    @staticmethod
    def backward(ctx, grad_y):
        b = ctx.batch
        if b.ws_version != ctx.ws_version:
            # the batch's workspace holds another solve (e.g. a second forward before this
            # backward): solve this graph's inputs again so the adjoint reuses its own factors
            SolveAtObservations._load_and_solve(b, *ctx.saved_tensors)
        out = b.backward(ctx.t_obs_list, grad_y.detach())
        fs, rs, vs = ctx.shapes
        df = out["dl_df"].reshape(-1)[b.f_index()].reshape(fs)
        dv = out["dl_dv"].reshape(vs)
        return (None, None, df, out["dl_dr"].reshape(rs), dv, out["dl_dsigma"], out["dl_dgamma"])


def solve_at_observations(batch, t_obs_list, f, r, v, sigma, gamma):
    """Functional form of SolveAtObservations (see there)."""
    return SolveAtObservations.apply(batch, t_obs_list, f, r, v, sigma, gamma)
