"""Perturbed predicates at concrete, tiny epsilons, in exact big-integer
arithmetic (test infrastructure).

This is the pin for the symbolic perturbation used by the oracle: instead of
expanding anything in epsilon, it actually moves every point to
    (x + e1*i, y + e2*i^2, z + e3*i^3),    e1 = 2^-K, e2 = 2^-4K, e3 = 2^-8K,
scales all coordinates by 2^(8K) so that they become integers, and evaluates the
textbook determinants exactly.  When K exceeds the bit length of every
coefficient that can occur (plus a margin), the sign of any such determinant
or difference of ratios equals the sign of its first nonzero epsilon
coefficient, so these values are the limit the oracle computes symbolically.

Each ratio of consecutive monomial weights that can occur (e1, e2/e1^2,
e3/(e2*e1^2)) is at most 2^-K, so K > log2(#terms * max|coefficient|) is
enough; ``choose_k`` takes the input's coordinate and index ranges and adds a
wide margin.
"""
from fractions import Fraction


def choose_k(max_abs_coord, max_index):
    cb = max(int(max_abs_coord), 1).bit_length() + 1   # coordinate difference bits
    ib = max(int(max_index), 1).bit_length()            # index bits
    # Every coefficient of D or N is at most 2^(2cb + 4ib + 1) in magnitude, so
    # a coefficient of N_A*D_B - N_B*D_A (a sum of at most four such products)
    # is below 2^(4cb + 8ib + 4); orientations in 3-d are smaller still.  With
    # at most 12 monomials, K = 4cb + 8ib + 16 leaves a margin of 2^8.
    return 4 * cb + 8 * ib + 16


class Perturbed:
    """Points (x, y, z, index) moved by concrete epsilons and scaled to integers."""

    def __init__(self, pts, idx, K, zsign=1):
        S = 8 * K
        self.K = K
        self.X = [int(p[0]) * (1 << S) + int(i) * (1 << (S - K)) for p, i in zip(pts, idx)]
        self.Y = [int(p[1]) * (1 << S) + int(i) ** 2 * (1 << (S - 4 * K)) for p, i in zip(pts, idx)]
        self.Z = [zsign * (int(p[2]) * (1 << S) + int(i) ** 3) for p, i in zip(pts, idx)]

    def D(self, a, b, c):
        """xy orientation of (a, b, c): z-component of (b - a) x (c - a)."""
        X, Y = self.X, self.Y
        return (X[b] - X[a]) * (Y[c] - Y[a]) - (X[c] - X[a]) * (Y[b] - Y[a])

    def N(self, a, b, c):
        """xz orientation of (a, b, c)."""
        X, Z = self.X, self.Z
        return (X[b] - X[a]) * (Z[c] - Z[a]) - (X[c] - X[a]) * (Z[b] - Z[a])

    def tau(self, a, b, c):
        """Kinetic event time N / D as an exact rational."""
        return Fraction(self.N(a, b, c), self.D(a, b, c))

    def orient3d(self, a, b, c, d):
        """det[b - a; c - a; d - a]."""
        X, Y, Z = self.X, self.Y, self.Z
        ux, uy, uz = X[b] - X[a], Y[b] - Y[a], Z[b] - Z[a]
        vx, vy, vz = X[c] - X[a], Y[c] - Y[a], Z[c] - Z[a]
        wx, wy, wz = X[d] - X[a], Y[d] - Y[a], Z[d] - Z[a]
        return ux * (vy * wz - vz * wy) - uy * (vx * wz - vz * wx) + uz * (vx * wy - vy * wx)


def sign(v):
    return (v > 0) - (v < 0)
