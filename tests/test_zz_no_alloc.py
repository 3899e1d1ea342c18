"""lsw_apply_noalloc (the application for callers that cannot allocate: scratch in the library's
per-GPU static array) through the C ABI, against lsw_apply of the same handle: equal results on two
calls in a row, the second with a smaller input (another handle on a smaller grid, and fewer
right-hand sides on the first handle), in 2D (both sweep modes, FP64 and complex64) and 3D; a handle
whose scratch need exceeds the array is refused with LSW_EINVAL, as is a windowed one."""
import math

import numpy as np
import pytest
import torch

from oracle.discretization import extend_normal
from paper_1909_01467_amd import inputs
from paper_1909_01467_amd.lsweeps import LSW_EINVAL, NOALLOC_SCRATCH_BYTES, LswError, Solver

pytestmark = pytest.mark.gpu


def medium(nx, ny, p):
    X, Y = np.meshgrid(inputs.bulk_coords(nx), np.arange(1, ny + 1) / (nx + 1))
    return extend_normal(1.0 + 0.2 * np.sin(3 * X) * np.cos(2 * Y), p)


def solver2d(nx, ny, p, q, r, **kw):
    m = medium(nx, ny, p)
    omega = 2 * math.pi * nx / 10
    return Solver(torch.from_numpy(m).cuda(), omega, 1.0 / (nx + 1), (nx, ny), p, q, r, **kw), m.size


def compare(s, X, precision):
    Z_ref = s.apply(X)
    Z = s.apply_noalloc(X)
    torch.cuda.synchronize()
    err = (torch.linalg.norm(Z - Z_ref) / torch.linalg.norm(Z_ref)).item()
    print("[case] noalloc vs apply", tuple(X.shape), precision, err, flush=True)
    # the same kernels on the same inputs: equal up to the order of nothing (bitwise in practice)
    assert err <= (1e-15 if precision == "fp64" else 1e-7), err


@pytest.mark.parametrize("mode", ["compressed", "chain"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_apply_equals_apply_on_two_calls_second_smaller(precision, mode):
    s1, N1 = solver2d(45, 38, 5, 3, 2, precision=precision, sweep_mode=mode, nrhs_max=2)
    s2, N2 = solver2d(30, 26, 4, 2, 2, precision=precision, sweep_mode=mode)
    st = s1.stats()
    assert 0 < st["noalloc_bytes"] <= NOALLOC_SCRATCH_BYTES
    X1 = torch.from_numpy(inputs.complex_normal((2, N1), 1)).cuda()
    X2 = torch.from_numpy(inputs.complex_normal(N2, 2)).cuda()
    compare(s1, X1, precision)          # first call: the larger input
    compare(s2, X2, precision)          # second call: a smaller grid through the same array
    compare(s1, X1[:1], precision)      # and fewer right-hand sides on the first handle
    s1.close()
    s2.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_apply_3d_equals_apply(precision):
    n, p = (11, 10, 9), (3, 3, 3)
    mb = 1.0 + 0.1 * np.random.default_rng(3).random((n[2], n[1], n[0]))
    m = extend_normal(mb, p)
    omega = 2 * math.pi * n[0] / 8
    s = Solver(torch.from_numpy(m).cuda(), omega, 1.0 / (n[0] + 1), n, p, 2, 2, precision=precision, nrhs_max=2)
    X = torch.from_numpy(inputs.complex_normal((2, m.size), 3)).cuda()
    compare(s, X, precision)
    compare(s, X[1:], precision)
    s.close()


def test_noalloc_apply_refuses_what_does_not_fit():
    s, N = solver2d(511, 511, 10, 8, 8, precision="mixed", nrhs_max=8)
    assert s.stats()["noalloc_bytes"] > NOALLOC_SCRATCH_BYTES
    with pytest.raises(LswError) as e:
        s.apply_noalloc(torch.zeros(N, dtype=torch.complex128, device="cuda"))
    assert e.value.code == LSW_EINVAL and "scratch" in str(e.value)
    s.close()
    s, N = solver2d(45, 38, 5, 3, 2, windows=True)
    with pytest.raises(LswError) as e:
        s.apply_noalloc(torch.zeros(N, dtype=torch.complex128, device="cuda"))
    assert e.value.code == LSW_EINVAL
    s.close()
