"""The capturable refinement (RBT_OPT_CAPTURABLE): the stationary refinement
of Sec. 5 without host tests. It is checked against the host-tested
refinement (same kernels in the same order, so bit-identical solution, step
count and backward error), then captured in a HIP graph and replayed with
eager work between the replays; every replay must reproduce the eager result
exactly. Cases: FP64 factors converging after a few steps, a tolerance that
cannot be met (all max_iter steps run), and FP32 / BF16-update factors whose
classical refinement takes several steps."""
import numpy as np
import pytest
import torch

from paper_2312_09376_amd import _lib, workloads

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def rbt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_09376_amd import rbt as r
    r.lib()
    return r


@pytest.fixture
def capturable(rbt):
    def set_mode(on):
        rbt.set_option(_lib.RBT_OPT_CAPTURABLE, 1 if on else 0)
    yield set_mode
    rbt.set_option(_lib.RBT_OPT_CAPTURABLE, 0)


def dev(a):
    a = np.asarray(a, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


# (name, n, nrhs, matrix, precision, tol scale (of n eps), max_iter)
CASES = [
    ("fp64-randn", 1500, 3, "randn", "fp64", 10.0, 10),
    ("fp64-unreachable", 700, 2, "shifted", "fp64", 1e-6, 3),
    ("fp32-dominant", 900, 4, "dominant", "fp32", 10.0, 30),
    ("bf16-dominant", 1100, 1, "dominant", "bf16", 10.0, 30),
]


def make(case):
    _, n, k, mat, _, _, _ = case
    A = {"randn": workloads.randn_matrix, "shifted": workloads.shifted,
         "dominant": workloads.dominant}[mat](n, seed=n)
    B = workloads.randn(n, k, seed=k + 1)
    return dev(A), dev(B)


def run(rbt, case, A, B, LU, X, work):
    _, n, k, _, prec, tol_scale, max_iter = case
    tol = tol_scale * n * EPS
    if prec == "fp64":
        out = rbt.solve_refine(A, B, 2, 2023, tol=tol, max_iter=max_iter, LU=LU, X=X, work=work)
    else:
        p = rbt.RBT_FP32 if prec == "fp32" else rbt.RBT_BF16
        out = rbt.solve_mixed(A, B, 2, 2023, prec=p, solver=rbt.RBT_IR_CLASSIC, tol=tol,
                              max_iter=max_iter, LU=LU, X=X, work=work)
    _, _, iters, berr, info, _ = out
    return iters, berr, info


def buffers(rbt, case):
    _, n, k, _, prec, _, _ = case
    dt = torch.float64 if prec == "fp64" else torch.float32
    LU = torch.empty_strided((n, n), (1, n), dtype=dt, device="cuda")
    X = torch.empty_strided((n, k), (1, n), dtype=torch.float64, device="cuda")
    p = {"fp64": rbt.RBT_FP64, "fp32": rbt.RBT_FP32, "bf16": rbt.RBT_BF16}[prec]
    work = torch.zeros(max(rbt.workspace_size(n, k, 2, p), 256), dtype=torch.uint8, device="cuda")
    return LU, X, work


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_capturable_matches_host_tested(rbt, capturable, case):
    A, B = make(case)
    LU, X, work = buffers(rbt, case)
    capturable(False)
    it0, be0, info0 = run(rbt, case, A, B, LU, X, work)
    X0, LU0 = X.clone(), LU.clone()
    capturable(True)
    X.zero_()
    it1, be1, info1 = run(rbt, case, A, B, LU, X, work)
    torch.cuda.synchronize()
    assert int(info0.item()) == int(info1.item()) == 0
    assert int(it0.item()) == int(it1.item()), (int(it0.item()), int(it1.item()))
    assert torch.equal(be0, be1) and torch.equal(X0, X) and torch.equal(LU0, LU)
    _, n, _, _, _, tol_scale, max_iter = case
    if tol_scale < 1.0:
        assert int(it1.item()) == max_iter
    else:
        assert float(be1.item()) <= tol_scale * n * EPS


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_capturable_graph_replay(rbt, capturable, case):
    A, B = make(case)
    LU, X, work = buffers(rbt, case)
    capturable(True)
    it_e, be_e, info_e = run(rbt, case, A, B, LU, X, work)
    torch.cuda.synchronize()
    X_e, it_e, be_e = X.clone(), int(it_e.item()), be_e.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(rbt, case, A, B, LU, X, work)  # warm-up on the capture stream's side
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        it_g, be_g, info_g = run(rbt, case, A, B, LU, X, work)
    for rep in range(3):
        X.fill_(float("nan"))
        LU.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(X, X_e), rep
        assert int(it_g.item()) == it_e and torch.equal(be_g, be_e) and int(info_g.item()) == 0
        # eager work between replays
        Y = torch.randn(512, 512, device="cuda", dtype=torch.float64)
        (Y @ Y).sum().item()


def test_capturable_rejects_unsupported(rbt, capturable):
    capturable(True)
    n = 64
    A = dev(workloads.dominant(n, seed=1))
    B = dev(workloads.randn(n, 17, seed=2))
    with pytest.raises(RuntimeError):
        rbt.solve_refine(A, B, 2, 2023)
    with pytest.raises(RuntimeError):
        rbt.solve_mixed(A, B[:, :1], 2, 2023,
                        solver=rbt.RBT_IR_GMRES)
