"""Reference draw of the random projection matrix A1 (test infrastructure).

Algorithm 1 (Sec. 3.1.3) starts the bilateral random projection from a
standard Gaussian matrix A1 of size n x r (Sec. 3.1.1).  The library draws it
from a 64-bit seed with a counter-based generator so that the same seed gives
the same A1 on any device.  This module re-implements that generator from the
published definitions, independently of the library:

* SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): the i-th output (i = 0, 1, ...) of the stream
  seeded with ``seed`` is ``mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)``
  with the variant-13 finaliser (shifts 30, 27, 31 and the two odd
  multipliers below).
* 53-bit uniforms in (0, 1): ``((z >> 11) + 0.5) * 2**-53``.
* Box-Muller (Box & Muller, Ann. Math. Stat. 1958): outputs 2j and 2j+1 give
  u1, u2 and the pair ``sqrt(-2 ln u1) * (cos(2 pi u2), sin(2 pi u2))``.

Element (i, c) of the row-major n x r matrix is Gaussian number i*r + c.
Pure Python integers and the C math library (through ``math``) are used so
that the result is bit-identical to a C implementation on the same host.

Pinning: the SplitMix64 outputs are checked against the published reference
vectors for seed 1234567 in the tests; the Gaussian draw is checked by its
moments.  Parity of the library's own generator against this one is bitwise.
"""

import math

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def splitmix64(seed: int, i: int) -> int:
    """Return output ``i`` of the SplitMix64 stream seeded with ``seed``."""
    z = (seed + (i + 1) * _GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * _M1) & _MASK
    z = ((z ^ (z >> 27)) * _M2) & _MASK
    return z ^ (z >> 31)


def uniform53(seed: int, i: int) -> float:
    """Uniform number in the open interval (0, 1) from output ``i``."""
    return ((splitmix64(seed, i) >> 11) + 0.5) * (2.0 ** -53)


def gaussian(seed: int, j: int) -> float:
    """Standard Gaussian number ``j`` of the stream (Box-Muller pairs)."""
    pair = j // 2
    u1 = uniform53(seed, 2 * pair)
    u2 = uniform53(seed, 2 * pair + 1)
    rad = math.sqrt(-2.0 * math.log(u1))
    ang = (2.0 * math.pi) * u2
    return rad * (math.cos(ang) if j % 2 == 0 else math.sin(ang))


def a1_gaussian(seed: int, n: int, r: int) -> np.ndarray:
    """Draw the n x r standard Gaussian projection matrix A1 for ``seed``."""
    out = np.empty(n * r, dtype=np.float64)
    for j in range(n * r):
        out[j] = gaussian(seed, j)
    return out.reshape(n, r)
