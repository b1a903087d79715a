"""Exact polynomial arithmetic over the rationals, for hand-integration pins.

A polynomial in three variables is a dict {(i, j, k): Fraction}.  Integrals
over the reference domains are exact closed forms, so a residual built here
involves no quadrature at all.
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial


class Poly:
    __slots__ = ("c",)

    def __init__(self, c=None):
        self.c = {k: Fraction(v) for k, v in (c or {}).items() if v != 0}

    @staticmethod
    def const(v):
        return Poly({(0, 0, 0): Fraction(v)})

    @staticmethod
    def var(i):
        e = [0, 0, 0]
        e[i] = 1
        return Poly({tuple(e): Fraction(1)})

    def __add__(self, o):
        o = o if isinstance(o, Poly) else Poly.const(o)
        r = dict(self.c)
        for k, v in o.c.items():
            r[k] = r.get(k, 0) + v
        return Poly(r)

    __radd__ = __add__

    def __neg__(self):
        return Poly({k: -v for k, v in self.c.items()})

    def __sub__(self, o):
        return self + (-(o if isinstance(o, Poly) else Poly.const(o)))

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if not isinstance(o, Poly):
            o = Fraction(o)
            return Poly({k: v * o for k, v in self.c.items()})
        r = {}
        for k1, v1 in self.c.items():
            for k2, v2 in o.c.items():
                k = (k1[0] + k2[0], k1[1] + k2[1], k1[2] + k2[2])
                r[k] = r.get(k, 0) + v1 * v2
        return Poly(r)

    __rmul__ = __mul__

    def diff(self, i):
        r = {}
        for k, v in self.c.items():
            if k[i] > 0:
                kk = list(k)
                kk[i] -= 1
                r[tuple(kk)] = r.get(tuple(kk), 0) + v * k[i]
        return Poly(r)

    def integrate(self, mono_integral):
        return sum((v * mono_integral(*k) for k, v in self.c.items()), Fraction(0))


def cube_mono(lo=-1, hi=1):
    """Integral of x^i y^j z^k over [lo, hi]^3."""
    lo, hi = Fraction(lo), Fraction(hi)

    def f(i, j, k):
        r = Fraction(1)
        for e in (i, j, k):
            r *= (hi ** (e + 1) - lo ** (e + 1)) / (e + 1)
        return r
    return f


def simplex_mono(i, j, k):
    """Integral of r^i s^j t^k over the unit tetrahedron: i! j! k! / (i+j+k+3)!."""
    return Fraction(factorial(i) * factorial(j) * factorial(k), factorial(i + j + k + 3))


def prism_mono(i, j, k):
    """Integral of r^i s^j zeta^k over triangle(0,0),(1,0),(0,1) x [-1, 1]."""
    tri = Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
    line = Fraction(1 - (-1) ** (k + 1), k + 1)
    return tri * line


def collapsed_pyramid_mono(i, j, k):
    """Integral of a^i b^j c^k (1-c)^2 over a, b in [-1, 1], c in [0, 1]
    (collapsed coordinates of the reference pyramid)."""
    ia = Fraction(1 - (-1) ** (i + 1), i + 1)
    ib = Fraction(1 - (-1) ** (j + 1), j + 1)
    # int_0^1 c^k (1-c)^2 dc = 2 k! / (k+3)!
    ic = Fraction(2 * factorial(k), factorial(k + 3))
    return ia * ib * ic


def det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def inv3(m):
    d = det3(m)
    adj = [[m[1][1] * m[2][2] - m[1][2] * m[2][1], m[0][2] * m[2][1] - m[0][1] * m[2][2], m[0][1] * m[1][2] - m[0][2] * m[1][1]],
           [m[1][2] * m[2][0] - m[1][0] * m[2][2], m[0][0] * m[2][2] - m[0][2] * m[2][0], m[0][2] * m[1][0] - m[0][0] * m[1][2]],
           [m[1][0] * m[2][1] - m[1][1] * m[2][0], m[0][1] * m[2][0] - m[0][0] * m[2][1], m[0][0] * m[1][1] - m[0][1] * m[1][0]]]
    return [[Fraction(adj[i][j]) / d for j in range(3)] for i in range(3)]
