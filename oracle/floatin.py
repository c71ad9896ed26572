"""Float input (test infrastructure): the snap of float32 coordinates to an
integer lattice, then the exact hull of the lattice points.

The paper's GPU program keeps coordinates as single-precision floats
(Sec. 3, Fig. "point_datatypes") and says nothing about robustness.  The
reading taken here: all 3n coordinates are scaled by one power of two,
    s = 2^(bits - E),   E = the least integer with max |c| <= 2^E,
and rounded to the nearest integer (ties to even).  Scaling a float32 by a
power of two is exact in float64, so the only rounding is that last step;
every lattice coordinate satisfies |q| <= 2^bits.  Floats within a factor
2^(bits - 23) of the largest magnitude land on the lattice unchanged.  The
hull is then the exact perturbed hull of the lattice points (perturbation
by input index), the same definition as for integer input; bits = 30 needs
the wide range of ``oracle.hull_wide``.
"""
import numpy as np

from . import hull_wide

MAX_BITS = 30


def exponent_bound(p32):
    """E: the least integer with max |c| <= 2^E (0 for an all-zero input)."""
    a = np.abs(np.asarray(p32, dtype=np.float32).astype(np.float64)).max(initial=0.0)
    if not np.isfinite(a):
        raise ValueError("non-finite coordinate")
    if a == 0.0:
        return 0
    m, e = np.frexp(a)  # a = m * 2^e, 0.5 <= m < 1
    return int(e) - 1 if m == 0.5 else int(e)


def lattice(p32, bits):
    """int64 lattice points [n, 3] of float32 points [n, 3]."""
    if not 1 <= bits <= MAX_BITS:
        raise ValueError("bits must be in [1, 30]")
    p = np.asarray(p32, dtype=np.float32).reshape(-1, 3)
    E = exponent_bound(p)
    q = np.rint(np.ldexp(p.astype(np.float64), bits - E))
    return q.astype(np.int64)


def hull_f32(p32, bits, lower_only=False):
    """Outward faces (input indices) of the hull of the lattice points."""
    return hull_wide(lattice(p32, bits), lower_only=lower_only)
