"""Pins of the oracle's butterfly structure (Sec. 3: Eq. 2-4, Algorithm 1)."""
import itertools

import numpy as np
import pytest

from oracle import structure, transform

SIZES = list(range(1, 130)) + [255, 256, 257, 1000, 1001, 1003]


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_every_index_once_per_layer(d):
    for n in SIZES:
        for layer, p in enumerate(structure.partners(n, d), start=1):
            seen = np.zeros(n, dtype=int)
            for (s, h, mu, nu) in structure.layer_butterflies(n, d, layer):
                seen[s:s + mu + nu] += 1
                seen[s + h:s + h + mu] += 1
            assert (seen == 1).all(), (n, d, layer)
            for i, j in enumerate(p):
                if j >= 0:
                    assert p[j] == i
                    assert abs(i - j) == structure.reference_size(n, d) >> layer


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_alignment_rule_eq4(d):
    """Children of butterfly j in layer l are 2j (size mu+nu) and 2j+1 (size mu)."""
    for n in SIZES:
        m = structure.reference_size(n, d)
        for layer in range(1, d):
            h = m >> layer
            parent = {s: (mu, nu) for (s, hh, mu, nu) in structure.layer_butterflies(n, d, layer)}
            child = {s: (mu, nu) for (s, hh, mu, nu) in structure.layer_butterflies(n, d, layer + 1)}
            for s, (mu, nu) in parent.items():
                top = child.get(s)
                bot = child.get(s + h)
                assert top is not None and 2 * top[0] + top[1] == mu + nu
                if mu > 0:
                    assert bot is not None and 2 * bot[0] + bot[1] == mu
                else:
                    assert bot is None


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_loops_match_recursive_alignment(d):
    """Algorithm 1's loop nest equals the Eq. 4 / Lemma 2 recursion with the
    global half-sizes (independent code paths)."""
    for n in SIZES:
        m = structure.reference_size(n, d)
        rec = structure.recursive_sizes(n, m // 2, d)
        for layer in range(1, d + 1):
            loops = [(2 * mu + nu, mu, nu) for (s, h, mu, nu) in structure.layer_butterflies(n, d, layer)]
            assert loops == rec[layer - 1], (n, d, layer)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_semi_parker(d):
    """Every butterfly but the last of a layer is a Parker butterfly (Sec. 3)."""
    for n in SIZES:
        for layer in range(1, d + 1):
            bl = structure.layer_butterflies(n, d, layer)
            for (s, h, mu, nu) in bl[:-1]:
                assert nu == 0 or 2 * mu + nu == 1


def test_parker_when_divisible():
    for d in range(1, 6):
        for n in range(1 << d, 300, 1 << d):
            assert structure.reference_size(n, d) == n
            for layer in range(1, d + 1):
                assert all(nu == 0 for (_, _, _, nu) in structure.layer_butterflies(n, d, layer))


def test_closed_form_groups():
    """Index i = r + t q (q = m/2^d): its layer-l partner is i with bit d-l of t
    flipped when that index is < n, otherwise i is unpaired.  So the two-sided
    transform splits into independent 2^d x 2^d groups."""
    for d in range(1, 6):
        for n in SIZES:
            m = structure.reference_size(n, d)
            q = m >> d
            P = structure.partners(n, d)
            for layer in range(1, d + 1):
                for i in range(n):
                    r, t = i % q, i // q
                    j = r + (t ^ (1 << (d - layer))) * q
                    assert P[layer - 1][i] == (j if j < n else -1)


def test_examples_from_the_rules():
    """Structures at the benchmark sizes (derived from Algorithm 1 by hand)."""
    def mn(n, d, layer):
        return [(mu, nu) for (_, _, mu, nu) in structure.layer_butterflies(n, d, layer)]
    assert structure.reference_size(20011, 2) == 20012
    assert mn(20011, 2, 1) == [(10005, 1)]
    assert mn(20011, 2, 2) == [(5003, 0), (5002, 1)]
    assert mn(30001, 2, 1) == [(14999, 3)]
    assert mn(30001, 2, 2) == [(7501, 0), (7498, 3)]
    assert mn(20000, 2, 1) == [(10000, 0)] and mn(20000, 2, 2) == [(5000, 0), (5000, 0)]
    # n = 9: the last layer-2 butterfly is the identity (mu = 0, nu = 3)
    assert mn(9, 2, 2) == [(3, 0), (0, 3)]
    # n = 5 (m = 8): layer 1 pairs 0<->4 only; the second layer-2 slot holds row 4 alone
    assert mn(5, 2, 1) == [(1, 3)]
    assert mn(5, 2, 2) == [(2, 0), (0, 1)]


def _lemma1_cases(max_m):
    for m in range(1, max_m + 1):
        for mu in range(0, m // 2 + 1):
            nu = m - 2 * mu
            yield m, mu, nu


def test_lemma1_minors_brute_force():
    """Lemma 1: det O[alpha, gamma] = 0 iff alpha and gamma differ mod (mu+nu),
    otherwise 2^(-k/2) <= |det| <= 1 (1-based indices)."""
    count = 0
    for m, mu, nu in _lemma1_cases(8):
        O = transform.butterfly_matrix(m, mu, nu)
        mod = mu + nu
        for k in range(1, m + 1):
            for alpha in itertools.combinations(range(1, m + 1), k):
                ra = sorted(a % mod for a in alpha)
                for gamma in itertools.combinations(range(1, m + 1), k):
                    rg = sorted(g % mod for g in gamma)
                    det = np.linalg.det(O[np.ix_([a - 1 for a in alpha], [g - 1 for g in gamma])])
                    count += 1
                    if ra != rg:
                        assert abs(det) < 1e-12
                    else:
                        assert 2.0 ** (-k / 2) * (1 - 1e-12) <= abs(det) <= 1 + 1e-12
    assert count == 82770   # all k x k minors of every O^<m>_{mu,nu}, m <= 8


# ---- tiled reference size (Sec. 3, after Algorithm 1) and Eq. 8 (Sec. 6.4) ----

@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("nb", [1, 2, 3, 8, 16])
def test_tiled_butterflies_align_to_tiles(d, nb):
    """With m = 2^d nb ceil(n / (2^d nb)) every butterfly of every layer
    starts and splits on a tile boundary, so a tile never straddles two
    halves (the purpose the paper gives for the tiled m)."""
    for n in list(range(1, 80)) + [255, 1000, 1003]:
        m = structure.reference_size(n, d, nb)
        assert m % ((1 << d) * nb) == 0 and m >= n and m - n < (1 << d) * nb
        for layer in range(1, d + 1):
            for (s, h, mu, nu) in structure.layer_butterflies(n, d, layer, nb):
                assert s % nb == 0 and h % nb == 0, (n, d, nb, layer, s, h)
        if nb == 1:
            assert m == structure.reference_size(n, d)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_tiled_top_half_in_tiles(d):
    """Sec. 6: the top half of layer 1 is 2^(d-1) ceil(n_t 2^-d) tiles,
    n_t = ceil(n / n_b); it equals half the tiled reference size."""
    for nb in (4, 7, 512):
        for n in (1, 5, 100, 1001, 23040, 69120, 150000):
            nt = -(-n // nb)
            tiles = (1 << (d - 1)) * (-(-nt // (1 << d)))
            assert structure.reference_size(n, d, nb) // 2 == tiles * nb


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("nb", [1, 3, 8])
def test_tiled_structure_keeps_eq4_and_orthogonality(d, nb):
    """The tiled structure is still a depth-d RBT of Eq. 3: Eq. 4 alignment
    (recursive builder at the tiled half-size) and orthogonal layers."""
    for n in (1, 7, 13, 40, 77, 129):
        m = structure.reference_size(n, d, nb)
        rec = structure.recursive_sizes(n, m // 2, d)
        for layer in range(1, d + 1):
            loops = [(2 * mu + nu, mu, nu)
                     for (s, h, mu, nu) in structure.layer_butterflies(n, d, layer, nb)]
            assert loops == rec[layer - 1], (n, d, nb, layer)
            O = transform.layer_matrix(n, d, layer, nb)
            assert np.allclose(O @ O.T, np.eye(n), atol=1e-15)


def _paper_sweep():
    """tests/golden/comm_free_sizes.txt: the Sec. 6.4 statements."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "comm_free_sizes.txt")
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, rest = line.split("=", 1)
                vals[key.strip()] = [int(v) for v in rest.split()]
    return vals


def test_paper_sweep_communication_statements():
    """Sec. 6.4: with tiles of 512, depth 2 and a 4 x 4 process grid, the
    sizes 23040 i (i = 1..11) need no communication exactly for 23040,
    138240 and 253440, and only one layer communicates for 69120, 184320
    and 207360 (brute force over every pair of the tiled structure)."""
    g = _paper_sweep()
    nb, d, p, q = g["nb"][0], g["depth"][0], g["grid"][0], g["grid"][1]
    none, one = [], []
    for i in range(1, 12):
        n = g["base"][0] * i
        layers = structure.communicating_layers(n, d, nb, p, q, granule=nb)
        if not layers:
            none.append(n)
        elif len(layers) == 1:
            one.append(n)
    assert none == g["no_communication"]
    assert one == g["one_layer"]


@pytest.mark.parametrize("p,q", [(4, 4), (2, 3), (3, 2), (4, 6), (1, 5)])
def test_eq8_size_is_communication_free(p, q):
    """Eq. 8: with the granule lcm(p, q) n_b no layer needs another process's
    data, for any n; its top half of layer 1 is the formula of Eq. 8 in
    tiles."""
    nb, d = 4, 2
    gran = structure.comm_free_granule(nb, p, q)
    lcm = gran // nb
    rng = np.random.default_rng(p * 10 + q)
    for n in [1, 9, 64, 97] + list(rng.integers(100, 1200, size=6)):
        n = int(n)
        assert structure.communicating_layers(n, d, nb, p, q, granule=gran) == []
        nt = -(-n // nb)
        eq8_tiles = lcm * (1 << (d - 1)) * (-(-nt // ((1 << d) * lcm)))
        assert structure.reference_size(n, d, gran) // 2 == eq8_tiles * nb
    # the plain tiled size does communicate for some n on a grid with p, q > 1
    if p > 1:
        assert any(structure.communicating_layers(n, d, nb, p, q, granule=nb)
                   for n in range(50, 400, 7))
