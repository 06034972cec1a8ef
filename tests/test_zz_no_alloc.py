"""nyls_solve_static (the solve whose workspace is the library's own device array, for
callers that cannot allocate) against nyls_solve on the same plans: two calls in a row, the
second on a smaller batch, so the second starts from what the first left in the array."""
import numpy as np
import pytest
import torch

from paper_2510_04094_amd import workloads

pytestmark = pytest.mark.gpu


def _compare(gpu_lib, insts, mode):
    b = gpu_lib.Batch(insts, mode=mode)
    ref = b.solve()
    got = b.solve_static()
    torch.cuda.synchronize()
    for key in ("yhat", "omega", "bias", "lam", "status"):
        a, r = got[key].cpu().numpy(), ref[key].cpu().numpy()
        if key == "status":
            assert np.array_equal(a, r), key
        else:
            # same kernels on the same inputs: equal up to the FP64 bar of the path
            scale = max(np.max(np.abs(r)), 1e-300)
            assert np.max(np.abs(a - r)) <= 1e-10 * scale, (key, np.max(np.abs(a - r)) / scale)
    return b


@pytest.mark.parametrize("mode_name", ["FP64", "MIXED"])
def test_static_workspace_solve_matches_solve(gpu_lib, mode_name):
    mode = getattr(gpu_lib, mode_name)
    first = [workloads.linear_second_order(i, n=3000, m=50) for i in range(6)]
    first += [workloads.linear_first_order(i) for i in range(4)]
    _compare(gpu_lib, first, mode)
    second = [workloads.linear_second_order(10 + i, n=1200, m=30) for i in range(3)]
    _compare(gpu_lib, second, mode)


def test_static_workspace_rejects_oversized_plans(gpu_lib):
    import ctypes
    insts = [workloads.linear_second_order(i, n=600, m=100) for i in range(400)]
    b = gpu_lib.Batch(insts, mode=gpu_lib.FP64)
    lib = gpu_lib.load()
    assert lib.nyls_workspace_size(b.plan) > (64 << 20)
    y = torch.empty(b.total, dtype=torch.float64, device=b.device)
    rc = lib.nyls_solve_static(b.plan, 4, None, None, None, ctypes.c_void_p(y.data_ptr()), None,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -5
