"""The allocation-free entry point rbt_solve_ex_noalloc against rbt_solve_ex:
the same kernels on the same inputs give bit-identical factors, solutions
and info, on two calls in a row (the second smaller, so the array holds the
first call's contents), and sizes beyond the library's array are refused."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2312_09376_amd import _lib, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_09376_amd import rbt as r
    r.lib()
    return r


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)).cuda().t()


def noalloc(rbt, A, B, depth, seed):
    n, k = A.shape[0], B.shape[1]
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = rbt.lib().rbt_solve_ex_noalloc(n, k, rbt._p(A), rbt._ld(A), rbt._p(B), rbt._ld(B), depth,
                                        seed, rbt._p(info), rbt._stream(A.device))
    return rc, info


@pytest.mark.parametrize("sizes", [[(20000, 1), (1003, 1)], [(3000, 2), (129, 3)],
                                   [(2100, 16), (300, 1)]])
def test_noalloc_matches_solve_ex(rbt, sizes):
    for n, k in sizes:
        A = workloads.randn_matrix(n, seed=n)
        B = workloads.randn(n, k, seed=k)
        A1, B1 = dev(A), dev(B)
        _, _, info1, _ = rbt.solve_(A1, B1, 2, 2023)
        A2, B2 = dev(A), dev(B)
        rc, info2 = noalloc(rbt, A2, B2, 2, 2023)
        torch.cuda.synchronize()
        assert rc == 0
        assert int(info1.item()) == int(info2.item()) == 0
        assert torch.equal(A1, A2) and torch.equal(B1, B2), (n, k)


def test_noalloc_rejects_oversize(rbt):
    n = 40000  # workspace about 181 MiB > the library's 96 MiB array
    A = torch.empty((1, 1), dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = rbt.lib().rbt_solve_ex_noalloc(n, 1, rbt._p(A), n, rbt._p(A), n, 2, 1, rbt._p(info),
                                        rbt._stream(A.device))
    assert rc == _lib.RBT_ERR_WORKSPACE
    assert rbt.lib().rbt_workspace_size(n, 1, 2, _lib.RBT_FP64) > (_lib.RBT_NOALLOC_SCRATCH_MB << 20)
