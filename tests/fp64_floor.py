"""The FP64 parity bar of one instance: 1e-10, or the oracle's own rounding floor where that
is larger.

Any FP64 evaluation of the Nystrom basis perturbs K_mm and its eigendecomposition:
  * the entries K = exp(-z^2), z = (t_s - t_z) / sigma, carry the rounding of z (relative
    2^-53, so 2 z^2 2^-53 in K) and that of the exponential;
  * 1/sigma or 1/sigma^2 is rounded once for all kernel values, which acts like sigma moved
    by one unit in the last place;
  * a backward-stable symmetric eigensolver (LAPACK's or the library's) returns the exact
    eigenpairs of K_mm + E with |E| of the order eps |K_mm|_2, an absolute perturbation that
    is large relative to the small entries.
Where K_mm keeps eigenvalues close to the cut-off tau lambda_1 (the second-order family at
tau = 1e-8) these move y_hat by up to ~1e-9; on well-conditioned instances by < 1e-11.
floor() measures, on the oracle alone, the largest change of y_hat under each of them
(random symmetric perturbations of those sizes, a few seeds), and bar() = max(1e-10,
4 x floor): 1e-10 wherever the oracle itself is stable at that level.

The backward perturbation's spectral norm is about 1.6 sqrt(m) eps |K_mm|_2 (15 to 18 eps for
m = 78 .. 128, the order of what LAPACK's own eigensolver leaves on these matrices).  A caller
that has measured the backward error of an eigendecomposition can pass it as `bnorm` (in
units of eps |K_mm|_2): the random perturbation is then scaled to that spectral norm.
"""
import contextlib

import numpy as np

import oracle

EPS = 2.0 ** -53


@contextlib.contextmanager
def _perturbed_kmm(kind, seed, bnorm=None):
    orig = oracle.nystrom.landmark_gram

    def noisy(t_land, sigma):
        k = orig(t_land, sigma)
        rng = np.random.default_rng(seed)
        if kind == "entries":
            z2 = ((t_land[:, None] - t_land[None, :]) / sigma) ** 2
            e = 2.0 * z2 * rng.uniform(-EPS, EPS, k.shape) + rng.uniform(-2 * EPS, 2 * EPS, k.shape)
            return k * (1.0 + 0.5 * (e + e.T))
        e = rng.uniform(-2 * EPS, 2 * EPS, k.shape) * np.linalg.norm(k, 2)
        e = 0.5 * (e + e.T)
        if bnorm is not None:
            e *= bnorm * EPS * np.linalg.norm(k, 2) / np.linalg.norm(e, 2)
        return k + e

    oracle.nystrom.landmark_gram = noisy
    try:
        yield
    finally:
        oracle.nystrom.landmark_gram = orig


def _yhat(q):
    return oracle.linear.solve(q)["yhat"]


def floor_of(fn, q, ref=None, seeds=3, bnorm=None):
    """Largest rel. l-inf change of the oracle quantity fn(q) (an array) under the FP64
    perturbations above."""
    if ref is None:
        ref = fn(q)
    nrm = np.max(np.abs(ref))
    worst = 0.0
    for kind in ("entries", "backward"):
        for s in range(seeds):
            with _perturbed_kmm(kind, 1000 + s, bnorm):
                y = fn(q)
            worst = max(worst, float(np.max(np.abs(y - ref)) / nrm))
    for sgn in (1.0, -1.0):
        y = fn(dict(q, sigma=float(q["sigma"]) * (1.0 + sgn * 2 * EPS)))
        worst = max(worst, float(np.max(np.abs(y - ref)) / nrm))
    return worst


def floor(q, ref=None, seeds=3, bnorm=None):
    """Largest rel. l-inf change of the oracle's y_hat under the FP64 perturbations above."""
    return floor_of(_yhat, q, ref, seeds, bnorm)


def bar_of(fn, q, ref=None, bnorm=None):
    return max(1e-10, 4.0 * floor_of(fn, q, ref, bnorm=bnorm))


def bar(q, ref=None, bnorm=None):
    return bar_of(_yhat, q, ref, bnorm)
