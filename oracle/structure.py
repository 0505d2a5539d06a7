"""Butterfly structure of a depth-d generalized (semi-Parker) RBT.  ORACLE: test
infrastructure only (see oracle/__init__.py).

Layer numbering follows Eq. 3: layer 1 is the single butterfly of full size n
(applied last by U^T, first by U), layer l has 2^(l-1) butterfly slots.  The
packed coefficient column k of Algorithm 1 is layer k+1.

Readings (listed in the design doc):
  * m is the non-tiled reference size 2^d * ceil(n / 2^d) (Sec. 3, text after
    Algorithm 1); with a granule g > 1 it is the tiled reference size
    2^d * g * ceil(n / (2^d * g)) of the same passage (g = the tile size
    n_b), and with g = lcm(p, q) * n_b the communication-free size of Eq. 8
    (Sec. 6.4) for a p x q process grid.
  * every layer uses the global half-size h_l = m / 2^l, as Algorithm 1 does;
    it is not recomputed per child (Eq. 4 allows either).
  * a slot whose start is >= n holds no index and is skipped; slot extents are
    clipped at n on both halves.
  * inside a butterfly of half-size h starting at s the top half is
    [s, s+h) and the bottom half [s+h, s+2h), both clipped at n;
    mu = |bottom|, nu = |top| - mu (Eq. 2), pairs are (s+t, s+h+t) for t < mu,
    and rows s+t for mu <= t < |top| are unpaired (factor 1, Eq. 2).

Parity: pinned by Lemma 1 brute force, the Hadamard special case, the Eq. 6
worked example, the recursive builder (Lemma 2 recursion) and Eq. 4
invariants (tests/test_oracle_structure.py); the tiled and Eq. 8 sizes by
tile alignment of every butterfly, the Sec. 6 statement of the top half in
tiles, and the Sec. 6.4 statements of which sizes need communication.
"""
import math


def reference_size(n, d, granule=1):
    """Reference size m = 2^d g ceil(n / (2^d g)) (Sec. 3, after Alg. 1):
    g = 1 is the non-tiled size 2^d ceil(n / 2^d), g = n_b the tiled one."""
    g = (1 << d) * granule
    return g * ((n + g - 1) // g)


def comm_free_granule(nb, p, q):
    """Granule of Eq. 8 (Sec. 6.4): lcm(p, q) tiles of size nb, for a p x q
    process grid; the top half of layer 1 is then
    lcm(p, q) 2^(d-1) ceil(n_t 2^-d / lcm(p, q)) tiles."""
    return (p * q // math.gcd(p, q)) * nb


def layer_butterflies(n, d, layer, granule=1):
    """Butterflies of one layer (Eq. 3 numbering, 1 <= layer <= d).

    Returns a list of (start, h, mu, nu): the butterfly covers rows
    [start, start + 2*mu + nu), its first mu rows pair with rows h further
    down, and rows start+mu .. start+mu+nu-1 are unpaired.  Follows the loop
    nest of Algorithm 1 with its global half-size h = m / 2^layer.
    """
    m = reference_size(n, d, granule)
    h = m >> layer
    out = []
    for b in range(1 << (layer - 1)):
        s = 2 * b * h
        if s >= n:
            continue
        top = min(h, n - s)
        bottom = max(0, min(h, n - s - h))
        out.append((s, h, bottom, top - bottom))
    return out


def partners(n, d, granule=1):
    """partner[l-1][i]: index paired with i in layer l, or -1 if unpaired.

    Built from the butterfly list above (pairs (s+t, s+h+t), t < mu).
    """
    table = []
    for layer in range(1, d + 1):
        p = [-1] * n
        for (s, h, mu, nu) in layer_butterflies(n, d, layer, granule):
            for t in range(mu):
                p[s + t] = s + h + t
                p[s + h + t] = s + t
        table.append(p)
    return table


def recursive_sizes(size, h, depth):
    """Butterfly sizes per layer from the Eq. 4 alignment rule.

    Recursion of Lemma 2 (a depth-d RBT of size `size` is a block-diagonal of
    two depth-(d-1) RBTs of sizes mu+nu and mu, times one butterfly, times a
    diagonal), with the split of the top butterfly at half-size h and the
    children splitting at h/2.  Returns a list per layer of (size, mu, nu).
    Independent of `layer_butterflies`; the tests check the two agree.
    """
    if depth == 0:
        return []
    top = min(h, size)
    bottom = size - top
    mu, nu = bottom, top - bottom
    here = [(size, mu, nu)]
    if depth == 1:
        return [here]
    left = recursive_sizes(mu + nu, h // 2, depth - 1)
    right = recursive_sizes(mu, h // 2, depth - 1) if mu > 0 else [[] for _ in range(depth - 1)]
    deeper = [left[k] + right[k] for k in range(depth - 1)]
    return [here] + deeper


def communicating_layers(n, d, nb, p, q, granule=1):
    """Layers whose two-sided application needs data from another process
    when A is distributed 2-D block-cyclically in nb x nb tiles over a p x q
    grid (tile row I on process row I mod p, tile column J on process column
    J mod q): layer l communicates if a pair (i, j) of it has its two rows on
    different process rows (the U side) or its two columns on different
    process columns (the V side). Brute force over all pairs."""
    out = []
    for layer, part in enumerate(partners(n, d, granule), start=1):
        rows = cols = False
        for i, j in enumerate(part):
            if j > i:
                rows = rows or (i // nb) % p != (j // nb) % p
                cols = cols or (i // nb) % q != (j // nb) % q
        if rows or cols:
            out.append(layer)
    return out
