"""Random diagonal coefficients of the RBT.  ORACLE: test infrastructure only.

The paper draws each diagonal entry as exp(r/20) with r uniform on [-1, 1]
(Sec. 6, experimental setup) and stores U and V packed as n x d arrays whose
column k is the diagonal of R_{k+1} (Sec. 3, packed storage, Alg. 1).  It
does not fix a generator, so this project defines one (reading listed in
the design doc):

  draw(seed, c)  = the c-th output (0-based) of SplitMix64 started at state
                   `seed` (Steele, Lea, Flood, OOPSLA 2014), i.e.
                   mix(seed + (c + 1) * 0x9E3779B97F4A7C15 mod 2^64)
  counter        c = 128 * i + 64 * side + (layer - 1),  side 0 = U, 1 = V
  uniform        u = (draw >> 11) * 2^-53 in [0, 1)
  r              2u - 1 in [-1, 1)      (exact in binary64)
  coefficient    exp(r / 20)

so index i's coefficient in a layer depends on (seed, side, layer, i) only,
not on n or d.  This module is written from the generator's published
definition in plain Python integers and shares nothing with the C++ one.

Parity: pinned by the published SplitMix64 output sequence for seed 1234567
(tests/golden/splitmix64_seed1234567.txt) and by the range of exp(r/20).
"""
import math

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def splitmix64_sequence(seed, count):
    """First `count` outputs of SplitMix64 from state `seed` (stateful form)."""
    state = seed & _MASK
    out = []
    for _ in range(count):
        state = (state + _GAMMA) & _MASK
        out.append(_mix(state))
    return out


def draw(seed, counter):
    """Counter form: the counter-th output of SplitMix64 from state seed."""
    return _mix((seed + (counter + 1) * _GAMMA) & _MASK)


def counter(side, layer, i):
    return 128 * i + 64 * side + (layer - 1)


def coefficient(seed, side, layer, i):
    u = (draw(seed, counter(side, layer, i)) >> 11) * (2.0 ** -53)
    r = 2.0 * u - 1.0
    return math.exp(r / 20.0)


def generate(n, d, seed):
    """Packed U, V (n x d, FP64): column k is the diagonal of R_{k+1}."""
    if d > 64:
        raise ValueError("depth above 64 is not representable in the counter")
    U = np.empty((n, d), dtype=np.float64)
    V = np.empty((n, d), dtype=np.float64)
    for layer in range(1, d + 1):
        for i in range(n):
            U[i, layer - 1] = coefficient(seed, 0, layer, i)
            V[i, layer - 1] = coefficient(seed, 1, layer, i)
    return U, V


def angle(seed, side, layer, i):
    """Random angle of the rotation butterflies (Sec. 3, the butterflies based
    on block rotations): theta = 2 pi u with u uniform on [0, 1), drawn from
    the same counter as the diagonal coefficients at the top index i of the
    pair (reading listed in the design doc: the paper fixes no law)."""
    u = (draw(seed, counter(side, layer, i)) >> 11) * (2.0 ** -53)
    return 2.0 * math.pi * u


def generate_rotations(n, d, seed, granule=1):
    """Packed rotation coefficients (n x d for U and V): for a pair (a, b) of
    layer l (a in the top half), C[a, l-1] = cos(theta_a) and
    C[b, l-1] = sin(theta_a); an unpaired index holds 1 (its rotation is by
    0 degrees: the identity)."""
    from . import structure
    if d > 64:
        raise ValueError("depth above 64 is not representable in the counter")
    out = []
    for side in (0, 1):
        C = np.ones((n, d), dtype=np.float64)
        for layer, part in enumerate(structure.partners(n, d, granule), start=1):
            for a, b in enumerate(part):
                if b > a:
                    t = angle(seed, side, layer, a)
                    C[a, layer - 1] = math.cos(t)
                    C[b, layer - 1] = math.sin(t)
        out.append(C)
    return out[0], out[1]
