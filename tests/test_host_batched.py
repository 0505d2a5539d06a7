"""The batched solver's kernel source (k_batched.hip) and host plan, built
as host C++ with an emulation of the device's execution model
(tests/hostemu: workgroups on host threads, work-items as fibers, barriers
and wavefront operations as rendezvous) under AddressSanitizer. Every
buffer is its own allocation and in the workspace only the plan's header,
table and each system's areas are addressable, so an access out of bounds,
a barrier reached from different places, a wavefront operation reached by
part of a wavefront, a deadlock or a loop that does not end fails the test.

These are CPU tests of the kernel's control flow and addressing on edge
cases and of its results against LAPACK; the GPU tests check the device
build against the oracle."""
import numpy as np
import pytest

from paper_2312_09376_amd import workloads

emu = pytest.importorskip("tests.hostemu.emu")

EPS = 2.0 ** -52
FP32, BF16 = 1, 2  # RBT_FP32, RBT_BF16
NEVER = 2 ** 63 - 1


@pytest.fixture(scope="module")
def exe():
    if emu.clang() is None:
        pytest.skip("clang++ not available")
    return emu.build()


def relfro(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def check_run(out, batch, grid):
    _, _, _, _, _, chk = out
    assert chk["divergent_barriers"] == 0
    assert chk["plan_intact"]
    # every workgroup takes one ticket past the last system
    assert chk["ticket"] == batch + grid


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_batch_matches_lapack(exe, prec):
    """Ragged sizes (one tile, a tile plus one row, several tiles) and
    nrhs up to the maximum: FP64-accurate solutions, low-precision path."""
    ns = [1, 37, 64, 65, 130, 201]
    ks = [1, 3, 16, 2, 1, 5]
    As = [workloads.dominant(n, seed=s) for s, n in enumerate(ns)]
    Bs = [workloads.randn(n, k, seed=s + 20) for s, (n, k) in enumerate(zip(ns, ks))]
    out = emu.run_batched(As, Bs, depth=2, prec=prec, seed=3, max_iter=30, grid=4, threads=4)
    Xs, iters, berr, info, path, _ = out
    check_run(out, len(ns), 4)
    for s, (A, B, X) in enumerate(zip(As, Bs, Xs)):
        n = A.shape[0]
        assert info[s] == 0 and path[s] == 0, (s, info[s], path[s])
        assert berr[s] <= 10 * n * EPS, (s, berr[s])
        assert relfro(X, np.linalg.solve(A, B)) <= 10 * np.linalg.cond(A, np.inf) * 10 * n * EPS


def test_fallback_to_fp64_factors(exe):
    """N(0,1) systems with BF16 trailing updates: refinement of the
    low-precision factors stalls and the FP64 factors (path 1) solve."""
    ns = [130, 90]
    As = [workloads.randn_matrix(n, seed=s + 40) for s, n in enumerate(ns)]
    Bs = [workloads.randn(n, 2, seed=s) for s, n in enumerate(ns)]
    out = emu.run_batched(As, Bs, depth=2, prec=BF16, seed=5, max_iter=10, grid=2, threads=2)
    Xs, iters, berr, info, path, _ = out
    check_run(out, 2, 2)
    for s, (A, B, X) in enumerate(zip(As, Bs, Xs)):
        n = A.shape[0]
        assert info[s] == 0 and path[s] in (0, 1) and berr[s] <= 10 * n * EPS, (s, path[s], berr[s])
        assert relfro(X, np.linalg.solve(A, B)) <= 10 * np.linalg.cond(A, np.inf) * 10 * n * EPS
    assert (path == 1).any()


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_zero_pivot_and_empty_systems(exe, prec):
    """One system with an exact zero pivot at column 71 (depth 0: no
    transform), one with n = 0 and one without right-hand sides."""
    A0 = np.eye(100)
    A0[70, 70] = 0.0
    A0[70, 71] = A0[71, 70] = 1.0
    ns, ks = [100, 0, 50], [1, 3, 0]
    As = [A0, np.zeros((0, 0)), workloads.dominant(50, seed=3)]
    Bs = [np.ones((n, k)) for n, k in zip(ns, ks)]
    out = emu.run_batched(As, Bs, depth=0, prec=prec, seed=1, max_iter=3, grid=3, threads=3)
    _, iters, berr, info, path, _ = out
    check_run(out, 3, 3)
    assert info[0] == 71
    assert not (berr[0] <= 1.0)  # NaN/Inf never looks converged
    assert iters[0] == 0  # a NaN error ends the refinement
    assert info[1] == 0 and iters[1] == 0 and berr[1] == 0.0
    assert info[2] == 0 and berr[2] == 0.0


def test_schedule_does_not_change_results(exe):
    """The tile-count threshold, the grid and the number of concurrently
    running workgroups change the schedule only: bit-identical outputs."""
    ns = [200, 70, 129, 5]
    ks = [2, 1, 3, 1]
    As = [workloads.dominant(n, seed=s + 7) for s, n in enumerate(ns)]
    Bs = [workloads.randn(n, k, seed=s) for s, (n, k) in enumerate(zip(ns, ks))]
    ref = None
    for ct2, grid, threads in [(NEVER, 4, 4), (0, 4, 4), (100, 2, 2), (NEVER, 1, 1)]:
        out = emu.run_batched(As, Bs, depth=2, prec=BF16, seed=9, max_iter=30, ct2_min_n=ct2,
                              grid=grid, threads=threads)
        check_run(out, len(ns), grid)
        flat = list(out[0]) + list(out[1:5])
        if ref is None:
            ref = flat
        else:
            assert all(np.array_equal(a, b) for a, b in zip(flat, ref)), (ct2, grid, threads)


@pytest.mark.parametrize("depth,kind,sides", [(0, 0, 2), (1, 0, 2), (3, 0, 2), (2, 1, 2), (2, 0, 1)])
def test_depths_and_variants(exe, depth, kind, sides):
    """Depths 0-3, rotation butterflies (kind 1) and the one-sided RBT."""
    ns, ks = [97, 64, 33], [2, 1, 4]
    As = [workloads.dominant(n, seed=s + 3) for s, n in enumerate(ns)]
    Bs = [workloads.randn(n, k, seed=s + 9) for s, (n, k) in enumerate(zip(ns, ks))]
    out = emu.run_batched(As, Bs, depth=depth, prec=FP32, seed=2, max_iter=30, grid=3, threads=3,
                          kind=kind, sides=sides)
    Xs, iters, berr, info, path, _ = out
    check_run(out, 3, 3)
    for s, (A, B, X) in enumerate(zip(As, Bs, Xs)):
        n = A.shape[0]
        assert info[s] == 0 and berr[s] <= 10 * n * EPS, (s, berr[s], path[s])
        assert relfro(X, np.linalg.solve(A, B)) <= 10 * np.linalg.cond(A, np.inf) * 10 * n * EPS
