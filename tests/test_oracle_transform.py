"""Pins of the oracle's coefficient generator and butterfly transforms
(Sec. 3, Eq. 1-3; worked example Eq. 6; Theorem 3)."""
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import coeffs, structure, transform, solve
from tests import qsqrt2
from tests.qsqrt2 import Q2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- generator

def test_splitmix64_published_sequence():
    lines = [l.strip() for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
             if l.strip() and not l.startswith("#")]
    seed = int(lines[0].split()[1])
    expected = [int(x) for x in lines[1:]]
    assert coeffs.splitmix64_sequence(seed, len(expected)) == expected
    # the counter form is the same sequence
    assert [coeffs.draw(seed, c) for c in range(len(expected))] == expected


def test_coefficient_range_and_independence_of_n():
    U, V = coeffs.generate(300, 3, seed=11)
    lo, hi = math.exp(-1 / 20), math.exp(1 / 20)
    for C in (U, V):
        assert (C >= lo).all() and (C < hi).all()
    U2, V2 = coeffs.generate(100, 2, seed=11)
    assert np.array_equal(U2, U[:100, :2]) and np.array_equal(V2, V[:100, :2])
    r = 20 * np.log(U)      # back to r ~ U[-1, 1)
    assert abs(r.mean()) < 0.05 and abs(r.var() - 1 / 3) < 0.03
    assert not np.array_equal(U, V)


# ---------------------------------------------------------- worked example

def _parse_golden_eq6():
    blocks, cur = {}, None
    for line in open(os.path.join(GOLDEN, "eq6_worked_example.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.isalpha() or line == "UtAV":
            cur = line
            blocks[cur] = []
        else:
            blocks[cur].append(line.split())
    return blocks


def _eval(tok, r):
    sign = -1.0 if tok.startswith("-") else 1.0
    val = 1.0
    for f in tok.lstrip("-").split("*"):
        val *= r[int(f[1:])] if f.startswith("r") else float(f)
    return sign * val


def test_worked_example_eq6():
    """Depth 1, n = 4: fixes the pairing i <-> i + n/2, the sign pattern and
    that the random diagonal multiplies the butterfly from the right."""
    g = _parse_golden_eq6()
    r = {i: v for i, v in enumerate([0, 1.3, 0.7, 1.9, 0.45, 1.1, 0.9, 1.7, 0.6])}
    A = np.array([[_eval(t, r) for t in row] for row in g["A"]])
    U_paper = np.array([[_eval(t, r) for t in row] for row in g["U"]])
    V_paper = np.array([[_eval(t, r) for t in row] for row in g["V"]])
    expect = np.array([[_eval(t, r) for t in row] for row in g["UtAV"]])
    Uc = np.array([[r[1]], [r[2]], [r[3]], [r[4]]])
    Vc = np.array([[r[5]], [r[6]], [r[7]], [r[8]]])
    # the paper's U and V omit the 1/sqrt(2) of Eq. 2
    assert np.allclose(math.sqrt(2) * transform.dense_rbt(4, 1, Uc), U_paper, rtol=0, atol=1e-15)
    assert np.allclose(math.sqrt(2) * transform.dense_rbt(4, 1, Vc), V_paper, rtol=0, atol=1e-15)
    got = transform.two_sided(A, Uc, Vc, 1)
    assert np.allclose(2 * got, expect, rtol=0, atol=1e-14)
    assert np.allclose(transform.two_sided_dense(A, Uc, Vc, 1), got, rtol=0, atol=1e-15)
    # not strongly nonsingular: the first pivot is exactly zero
    _, info = solve.genp_unblocked(got)
    assert info == 1
    # Algorithm 1's RBT2, read literally, scales before mixing; that order
    # gives a different matrix (non-zero off-diagonal 2x2 blocks).
    O = transform.layer_matrix(4, 1, 1)
    alg1 = O @ (np.diag(Uc[:, 0]) @ A @ np.diag(Vc[:, 0])) @ O
    assert not np.allclose(2 * alg1, expect, atol=1e-3)


# ------------------------------------------------------- factor properties

def test_butterfly_orthogonal_symmetric():
    for m in range(1, 12):
        for mu in range(0, m // 2 + 1):
            O = transform.butterfly_matrix(m, mu, m - 2 * mu)
            assert np.allclose(O, O.T, atol=0)
            assert np.allclose(O @ O, np.eye(m), atol=1e-15)


def test_unit_coefficients_give_orthogonal_u():
    for d in range(1, 6):
        for n in range(1, 70):
            Ud = transform.dense_rbt(n, d, np.ones((n, d)))
            assert np.allclose(Ud.T @ Ud, np.eye(n), atol=1e-14), (n, d)


def test_hadamard_special_case():
    """All r = 1 and 2^d | n: U = (H_{2^d} kron I_{n/2^d}) / 2^(d/2) with the
    Sylvester Hadamard matrix; full depth: H_n / sqrt(n)."""
    for d in range(1, 5):
        g = 1 << d
        for n in (g, 2 * g, 3 * g, 8 * g):
            Ud = transform.dense_rbt(n, d, np.ones((n, d)))
            H = np.kron(scipy.linalg.hadamard(g), np.eye(n // g)) / 2 ** (d / 2)
            assert np.allclose(Ud, H, atol=1e-14)
    for k in range(1, 7):
        n = 1 << k
        Ud = transform.dense_rbt(n, k, np.ones((n, k)))
        assert np.allclose(Ud, scipy.linalg.hadamard(n) / math.sqrt(n), atol=1e-14)


def test_parker_recursion():
    """2^d | n: the layered product (Eq. 3) equals the recursive construction
    U = (U_0 (+) U_1) O R of Lemma 2."""
    rng = np.random.default_rng(5)
    for d in (1, 2, 3, 4):
        for n in ((1 << d), 3 * (1 << d), 64):
            if n % (1 << d):
                continue
            C = np.exp(rng.uniform(-1, 1, (n, d)) / 20)
            assert np.allclose(transform.dense_rbt(n, d, C),
                               transform.dense_rbt_recursive_parker(C), atol=1e-14)


@pytest.mark.parametrize("granule", [1, 3, 8])
def test_packed_equals_dense(granule):
    """Packed O(d n^2) application = product with the dense Eq. 2/Eq. 3
    factors, for the non-tiled (granule 1) and tiled reference sizes."""
    rng = np.random.default_rng(7 + granule)
    for d in range(0, 6 if granule == 1 else 4):
        for n in list(range(1, 40)) + [63, 64, 65, 97]:
            U = np.exp(rng.uniform(-1, 1, (n, d)) / 20)
            V = np.exp(rng.uniform(-1, 1, (n, d)) / 20)
            A = rng.standard_normal((n, n))
            X = rng.standard_normal((n, 3))
            Ud = transform.dense_rbt(n, d, U, granule)
            assert np.allclose(transform.apply_transpose_left(X, U, d, granule), Ud.T @ X, atol=1e-13)
            assert np.allclose(transform.apply_left(X, U, d, granule), Ud @ X, atol=1e-13)
            assert np.allclose(transform.two_sided(A, U, V, d, granule),
                               transform.two_sided_dense(A, U, V, d, granule), atol=1e-13)


def test_exact_dense_factor_matches():
    """The float dense factor equals the same product in exact Q(sqrt2)
    arithmetic built directly from Eq. 2 and Eq. 3 (dyadic coefficients)."""
    rnd = random.Random(3)
    for (n, d) in [(5, 2), (7, 3), (9, 2), (6, 1), (11, 3)]:
        C = [[Fraction(rnd.randint(900, 1100), 1024) for _ in range(d)] for _ in range(n)]
        U = _exact_rbt(n, d, C)
        Uf = transform.dense_rbt(n, d, np.array([[float(c) for c in row] for row in C]))
        assert np.allclose(np.array([[float(x) for x in row] for row in U]), Uf, atol=1e-15)


def _exact_rbt(n, d, C):
    """U = O_d R_d ... O_1 R_1 in Q(sqrt2), straight from Eq. 2 / Eq. 3."""
    Uex = qsqrt2.eye(n)
    for layer in range(1, d + 1):
        O = [[Q2() for _ in range(n)] for _ in range(n)]
        for (s, h, mu, nu) in structure.layer_butterflies(n, d, layer):
            for t in range(mu):
                a, b = s + t, s + h + t
                O[a][a] = qsqrt2.INV_SQRT2
                O[a][b] = qsqrt2.INV_SQRT2
                O[b][a] = qsqrt2.INV_SQRT2
                O[b][b] = -qsqrt2.INV_SQRT2
            for t in range(mu, mu + nu):
                O[s + t][s + t] = Q2(1)
        R = [[Q2(C[i][layer - 1]) if i == j else Q2() for j in range(n)] for i in range(n)]
        Uex = qsqrt2.matmul(O, qsqrt2.matmul(R, Uex))
    return Uex


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_theorem3_full_depth_strongly_nonsingular(n):
    """Theorem 3: with depth ceil(log2 n) + 1 semi-Parker RBTs on both sides,
    U^T A V is strongly nonsingular with probability 1 (exact arithmetic).
    A is the pair-swap permutation of Eq. 6 extended to any n (an odd last
    row maps to itself); its leading 1x1 block is singular."""
    d = math.ceil(math.log2(n)) + 1
    rnd = random.Random(100 + n)
    swap = [(i ^ 1) if (i ^ 1) < n else i for i in range(n)]
    A = [[Q2(1 if j == swap[i] else 0) for j in range(n)] for i in range(n)]
    Cu = [[Fraction(rnd.randint(1, 10 ** 6), 10 ** 6) for _ in range(d)] for _ in range(n)]
    Cv = [[Fraction(rnd.randint(1, 10 ** 6), 10 ** 6) for _ in range(d)] for _ in range(n)]
    Ue, Ve = _exact_rbt(n, d, Cu), _exact_rbt(n, d, Cv)
    At = qsqrt2.matmul(qsqrt2.transpose(Ue), qsqrt2.matmul(A, Ve))
    piv = qsqrt2.leading_pivots(At)
    assert len(piv) == n and not any(p.is_zero() for p in piv)
    # the untransformed matrix has a zero leading pivot
    assert qsqrt2.leading_pivots(A)[0].is_zero()


def test_eq1_exact_solution_invariance():
    """Eq. 1 in exact arithmetic: V (U^T A V)^-1 U^T b = A^-1 b for any
    coefficients, whenever the elimination without pivoting succeeds."""
    rnd = random.Random(9)
    for (n, d) in [(4, 2), (5, 2), (7, 2), (6, 3), (9, 2)]:
        A = [[Q2(rnd.randint(-9, 9)) for _ in range(n)] for _ in range(n)]
        for i in range(n):
            A[i][i] = A[i][i] + 25
        b = [Q2(rnd.randint(-9, 9)) for _ in range(n)]
        Cu = [[Fraction(rnd.randint(1, 999), 1000) for _ in range(d)] for _ in range(n)]
        Cv = [[Fraction(rnd.randint(1, 999), 1000) for _ in range(d)] for _ in range(n)]
        Ue, Ve = _exact_rbt(n, d, Cu), _exact_rbt(n, d, Cv)
        At = qsqrt2.matmul(qsqrt2.transpose(Ue), qsqrt2.matmul(A, Ve))
        bt = [r[0] for r in qsqrt2.matmul(qsqrt2.transpose(Ue), [[x] for x in b])]
        xt = qsqrt2.solve(At, bt)
        x = [r[0] for r in qsqrt2.matmul(Ve, [[v] for v in xt])]
        assert x == qsqrt2.solve(A, b)
        # and the float oracle reproduces it
        Af = np.array([[float(v) for v in row] for row in A])
        bf = np.array([float(v) for v in b])
        Uf = np.array([[float(c) for c in row] for row in Cu])
        Vf = np.array([[float(c) for c in row] for row in Cv])
        xf, _, info = solve.rbt_solve(Af, bf, Uf, Vf, d)
        assert info == 0
        assert np.allclose(xf, [float(v) for v in x], rtol=1e-12, atol=1e-14)


# ---- rotation butterflies (Sec. 3) and the one-sided RBT (Sec. 7) ----

@pytest.mark.parametrize("granule", [1, 4])
def test_rotation_rbt_at_45_degrees_is_the_hadamard_butterfly(granule):
    """A rotation by 45 degrees on every pair is the butterfly of Eq. 2, so the
    rotation RBT then equals the Eq. 3 RBT with unit diagonals."""
    for d in (1, 2, 3):
        for n in (1, 5, 8, 13, 64, 77):
            C = np.ones((n, d))
            for layer, part in enumerate(structure.partners(n, d, granule), start=1):
                for a, b in enumerate(part):
                    if b >= 0:
                        C[a, layer - 1] = np.sqrt(0.5)  # cos 45 = sin 45
            R = transform.dense_rotation_rbt(n, d, C, granule)
            H = transform.dense_rbt(n, d, np.ones((n, d)), granule)
            assert np.allclose(R, H, atol=1e-15), (n, d)


def test_rotation_rbt_orthogonal_and_packed_equals_dense():
    rng = np.random.default_rng(3)
    for d in (1, 2, 3, 5):
        for n in (1, 2, 7, 16, 33, 100):
            U, V = coeffs.generate_rotations(n, d, 99)
            # cos^2 + sin^2 = 1 on every pair (the defining constraint)
            for layer, part in enumerate(structure.partners(n, d), start=1):
                for a, b in enumerate(part):
                    if b > a:
                        assert abs(U[a, layer - 1] ** 2 + U[b, layer - 1] ** 2 - 1) < 1e-15
                    elif b < 0:
                        assert U[a, layer - 1] == 1.0
            Ud = transform.dense_rotation_rbt(n, d, U)
            assert np.allclose(Ud.T @ Ud, np.eye(n), atol=1e-14)
            X = rng.standard_normal((n, 3))
            assert np.allclose(transform.rotation_apply_transpose_left(X, U, d), Ud.T @ X,
                               atol=1e-13)
            assert np.allclose(transform.rotation_apply_left(X, U, d), Ud @ X, atol=1e-13)
            A = rng.standard_normal((n, n))
            Vd = transform.dense_rotation_rbt(n, d, V)
            assert np.allclose(transform.two_sided_kind(A, U, V, d, "rotation"), Ud.T @ A @ Vd,
                               atol=1e-12)
            assert np.allclose(transform.two_sided_kind(A, U, V, d, "diag", sides=1),
                               transform.dense_rbt(n, d, U).T @ A, atol=1e-12)


@pytest.mark.parametrize("kind,sides", [("rotation", 2), ("diag", 1), ("rotation", 1)])
def test_kind_and_sides_solve_the_system(kind, sides):
    """Eq. 1 holds for any invertible U, V: rotation and one-sided RBTs give
    A^-1 b (exact rational check is in Q(sqrt2) only for Eq. 3; here against
    LAPACK on a well-conditioned matrix)."""
    from oracle import solve
    from paper_2312_09376_amd import workloads
    n, d = 120, 2
    A = workloads.shifted(n, seed=4)
    B = workloads.randn(n, 2, seed=5)
    U, V = (coeffs.generate_rotations(n, d, 7) if kind == "rotation"
            else coeffs.generate(n, d, 7))
    X, _, info = solve.rbt_solve_kind(A, B, U, V, d, kind=kind, sides=sides)
    assert info == 0
    assert np.allclose(X, np.linalg.solve(A, B), rtol=1e-10, atol=1e-12)
