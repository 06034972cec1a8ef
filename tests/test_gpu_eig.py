"""The eigendecomposition K_mm = U Lambda U^T of App. A.2 (eq32) on every eigensolver path,
read back with nyls_basis: backward error |K - U Lambda U^T|_2 <= 128 eps |K|_2, U orthogonal
to 256 eps, eigenvalues within the two backward and orthogonality errors of the oracle's
(LAPACK) ones (Weyl),
eigenvector signs by the largest-magnitude entry.  The paths: the lane-parallel QL staged
through the workspace (m <= 64, the default), one wavefront per instance (tuning eig_ql),
two rows per lane (64 < m <= 128, few such instances), the staged form for 32 or more
instances with 64 < m <= 128, and the workspace solver of the wide bases (m > 128)."""
import numpy as np
import pytest
import torch

import fp64_floor
import oracle
from paper_2510_04094_amd import workloads

pytestmark = pytest.mark.gpu

EPS = fp64_floor.EPS


def backward_error(k, lam, u):
    nk = np.linalg.norm(k, 2)
    be = np.linalg.norm(k - (u * lam[None, :]) @ u.T, 2) / nk / EPS
    oe = np.linalg.norm(u.T @ u - np.eye(len(lam)), 2) / EPS
    return be, oe


def _insts(kind):
    if kind == "m<=64":
        return workloads.mixed_batch(count=40, n_lo=500, n_hi=2000, ms=(20, 33, 50, 64))
    if kind == "64<m<=128 few":
        return workloads.mixed_batch(count=12, n_lo=500, n_hi=2000, ms=(65, 100, 128, 40))
    if kind == "64<m<=128 many":
        return workloads.mixed_batch(count=40, n_lo=500, n_hi=2000, ms=(65, 100, 128))
    return [workloads.linear_second_order(7, n=6000, m=200, t_end=40.0, sigma=0.7),
            workloads.linear_first_order(8, n=5000, m=256, t_end=20.0, sigma=0.3, tau=1e-10),
            workloads.linear_second_order(9, n=3000, m=129, t_end=10.0, sigma=0.4)]


CASES = [("m<=64", None), ("m<=64", 1), ("64<m<=128 few", None), ("64<m<=128 many", None),
         ("64<m<=128 many", 1), ("m>128", None)]


@pytest.mark.parametrize("kind,eig_ql", CASES, ids=["%s-ql%s" % c for c in CASES])
def test_eigendecomposition_is_backward_stable(gpu_lib, kind, eig_ql):
    insts = _insts(kind)
    tun = dict(gpu_lib.DEFAULT_TUNING, eig_ql=1) if eig_ql else None
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64, tuning=tun)
    times = [q["t"][:4] for q in insts]
    b.features(times, dmax=0)
    lam_g, u_g = b.basis()
    torch.cuda.synchronize()
    lam_g, u_g = lam_g.cpu().numpy(), u_g.cpu().numpy()
    worst = 0.0
    for i, q in enumerate(insts):
        m = q["m"]
        k = oracle.nystrom.landmark_gram(q["t"][oracle.nystrom.landmark_indices(q)], q["sigma"])
        lam_o, u_o = oracle.nystrom.eig_desc(k)
        lam, u = lam_g[i, :m], u_g[i, :m, :m]
        be, oe = backward_error(k, lam, u)
        be_o, oe_o = backward_error(k, lam_o, u_o)
        worst = max(worst, be)
        assert be <= 128 and oe <= 256, (i, m, be, oe)
        assert np.all(np.diff(lam) <= 0), i
        # U Lambda U^T has eigenvalues within oe eps |K| of Lambda
        assert np.max(np.abs(lam - lam_o)) <= (be + oe + be_o + oe_o) * EPS * np.linalg.norm(k, 2), i
        piv = np.argmax(np.abs(u), axis=0)
        assert np.all(u[piv, np.arange(m)] > 0), i
        assert np.all(lam_g[i, m:] == 0) and np.all(u_g[i, m:, :] == 0) and np.all(u_g[i, :, m:] == 0)
    print(kind, "largest backward error %.1f eps" % worst)
