"""Forward-mode dual numbers over numpy arrays (oracle test infrastructure).

A ``Dual`` carries a value array ``v`` and a tangent array ``d`` whose last
axis indexes the seeded directions.  Every operation applies the ordinary
chain rule, so the oracle's pointwise Jacobians are exact (up to rounding),
not finite differences.  Non-smooth points follow the convention
d|x|/dx = sign(x) with sign(0) = 0.
"""
from __future__ import annotations

import numpy as np


class Dual:
    __slots__ = ("v", "d")
    __array_priority__ = 1000

    def __init__(self, v, d):
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)

    # --- helpers -----------------------------------------------------------
    def _lift(self, o):
        if isinstance(o, Dual):
            return o
        o = np.asarray(o, dtype=np.float64)
        return Dual(o, np.zeros(o.shape + (self.d.shape[-1],)))

    def __add__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v + o.v, self.d + o.d)
        return Dual(self.v + o, self.d + np.zeros_like(np.asarray(o, dtype=float))[..., None])

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __sub__(self, o):
        return self + (-o)

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v * o.v, self.d * o.v[..., None] + o.d * self.v[..., None])
        o = np.asarray(o, dtype=np.float64)
        return Dual(self.v * o, self.d * o[..., None])

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            q = self.v / o.v
            return Dual(q, (self.d - o.d * q[..., None]) / o.v[..., None])
        o = np.asarray(o, dtype=np.float64)
        return Dual(self.v / o, self.d / o[..., None])

    def __rtruediv__(self, o):
        o = np.asarray(o, dtype=np.float64)
        q = o / self.v
        return Dual(q, -self.d * (q / self.v)[..., None])

    def __pow__(self, e):
        # real constant exponent only
        e = float(e)
        return Dual(self.v ** e, self.d * (e * self.v ** (e - 1.0))[..., None])


def value(x):
    return x.v if isinstance(x, Dual) else np.asarray(x, dtype=np.float64)


def exp(x):
    if isinstance(x, Dual):
        e = np.exp(x.v)
        return Dual(e, x.d * e[..., None])
    return np.exp(x)


def log(x):
    if isinstance(x, Dual):
        return Dual(np.log(x.v), x.d / x.v[..., None])
    return np.log(x)


def sqrt(x):
    if isinstance(x, Dual):
        s = np.sqrt(x.v)
        return Dual(s, x.d / (2.0 * s)[..., None])
    return np.sqrt(x)


def absval(x):
    if isinstance(x, Dual):
        return Dual(np.abs(x.v), x.d * np.sign(x.v)[..., None])
    return np.abs(x)


def sqrt_abs(x):
    """sqrt(|x|) with derivative sign(x)/(2 sqrt|x|), taken as 0 at x = 0."""
    if isinstance(x, Dual):
        s = np.sqrt(np.abs(x.v))
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.where(s > 0.0, np.sign(x.v) / (2.0 * np.where(s > 0.0, s, 1.0)), 0.0)
        return Dual(s, x.d * g[..., None])
    return np.sqrt(np.abs(x))


def where(cond, a, b):
    """Elementwise select; the derivative follows the selected branch."""
    cond = np.asarray(cond)
    if isinstance(a, Dual) or isinstance(b, Dual):
        n = (a.d if isinstance(a, Dual) else b.d).shape[-1]
        A = a if isinstance(a, Dual) else Dual(a, np.zeros(np.shape(a) + (n,)))
        B = b if isinstance(b, Dual) else Dual(b, np.zeros(np.shape(b) + (n,)))
        return Dual(np.where(cond, A.v, B.v), np.where(cond[..., None], A.d, B.d))
    return np.where(cond, a, b)


def seed(values, n_dir, offset):
    """Dual copies of the component arrays ``values`` (a list), seeding
    component i in direction offset + i of n_dir directions."""
    out = []
    for i, x in enumerate(values):
        x = np.asarray(x, dtype=np.float64)
        d = np.zeros(x.shape + (n_dir,))
        d[..., offset + i] = 1.0
        out.append(Dual(x, d))
    return out


def const(values, n_dir):
    """Dual copies with zero tangents."""
    out = []
    for x in values:
        x = np.asarray(x, dtype=np.float64)
        out.append(Dual(x, np.zeros(x.shape + (n_dir,))))
    return out


def jac(outputs):
    """Stack tangents of a list of Duals: [..., n_out, n_dir]."""
    return np.stack([o.d for o in outputs], axis=-2)


def vals(outputs):
    return np.stack([value(o) for o in outputs], axis=-1)
