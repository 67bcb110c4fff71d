"""Approximation spaces and quadrature of one macro-element (oracle, FP64).

Oracle test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import this package.

A macro-element is an axis-aligned box split into 2x2x2 hexahedral
sub-elements of degree p (Sec. 3.1: conforming submesh, C0 local space
W_p(K); here with tensor Q_p elements).  Along each axis the macro space is
spanned by 2p+1 piecewise Lagrange functions on GLL points of the two
sub-intervals of the reference segment [0, 2]; the middle node is shared.
Volume integrals use p+1 Gauss points per sub-interval and axis, face
integrals the matching 2-D rule on the four sub-faces (Sec. 3.1 eq. C31,
C32 evaluated by quadrature).  The trace space on a macro-face is the
restriction of the macro space to that face: (2p+1)^2 nodes.

Everything here is written as dense tables (one row per quadrature point,
one column per basis function) built from 1-D factors with Kronecker
products, so that integrals below are plain weighted sums.
"""
from __future__ import annotations

import functools

import numpy as np

FACE_AXIS = (0, 0, 1, 1, 2, 2)
FACE_SIDE = (0, 1, 0, 1, 0, 1)


def gll_points(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points on [-1,1]: +-1 and the roots of P_p'."""
    if p == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def _lagrange(nodes, x):
    """Values and derivatives of the Lagrange polynomials on ``nodes`` at ``x``."""
    m = len(nodes)
    L = np.ones((len(x), m))
    dL = np.zeros((len(x), m))
    for i in range(m):
        for j in range(m):
            if j == i:
                continue
            L[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
        # derivative by the product rule
        for k in range(m):
            if k == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[k]))
            for j in range(m):
                if j == i or j == k:
                    continue
                term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            dL[:, i] += term
    return L, dL


@functools.lru_cache(maxsize=None)
def tables_1d(p: int):
    """1-D macro tables on the reference segment [0, 2].

    Returns dict with
      nodes [2p+1]   node positions,
      xq, wq [2(p+1)] Gauss points / weights (p+1 per sub-interval),
      B, D [2(p+1)][2p+1] basis values and d/dxi at the Gauss points,
      end [2][2p+1] basis values at xi = 0 and xi = 2.
    """
    g = gll_points(p)
    local = (g + 1.0) / 2.0
    n1d = 2 * p + 1
    nodes = np.concatenate([local, 1.0 + local[1:]])
    xg, wg = np.polynomial.legendre.leggauss(p + 1)
    xl, wl = (xg + 1.0) / 2.0, wg / 2.0
    xq = np.concatenate([xl, 1.0 + xl])
    wq = np.concatenate([wl, wl])
    B = np.zeros((2 * (p + 1), n1d))
    D = np.zeros((2 * (p + 1), n1d))
    for e in range(2):
        rows = slice(e * (p + 1), (e + 1) * (p + 1))
        Le, dLe = _lagrange(local, xq[rows] - e)
        B[rows, e * p:e * p + p + 1] = Le
        D[rows, e * p:e * p + p + 1] = dLe
    end = np.zeros((2, n1d))
    end[0, 0] = 1.0
    end[1, n1d - 1] = 1.0
    return dict(nodes=nodes, xq=xq, wq=wq, B=B, D=D, end=end, n1d=n1d, nq1=2 * (p + 1))


def _kron3(tz, ty, tx):
    """Table over (point, function) with x fastest in both indices."""
    return np.kron(tz, np.kron(ty, tx))


@functools.lru_cache(maxsize=None)
def reference_tables(p: int):
    """Dense reference-element tables (h = 1 per sub-element axis).

    vol_phi [G][n], vol_dphi [3][G][n] (d/dxi_j), vol_w [G];
    for each face f: face_phi [6][S][n] (volume basis on the face),
    face_psi [6][S][nf] (trace basis), face_w [6][S] (reference weights).
    Volume points are ordered g = g1 + nq1 (g2 + nq1 g3); face points
    s = s1 + nq1 s2 over the two tangential axes in increasing order.
    """
    t = tables_1d(p)
    B, D, w = t["B"], t["D"], t["wq"]
    vol_phi = _kron3(B, B, B)
    vol_dphi = np.stack([_kron3(B, B, D), _kron3(B, D, B), _kron3(D, B, B)])
    vol_w = np.kron(w, np.kron(w, w))
    face_phi, face_psi, face_w = [], [], []
    for f in range(6):
        d = FACE_AXIS[f]
        endrow = t["end"][FACE_SIDE[f]][None, :]  # [1][n1d]
        facs = []
        for ax in (2, 1, 0):                       # kron order z, y, x
            facs.append(endrow if ax == d else B)
        # face points: the normal axis contributes a single row
        face_phi.append(np.kron(facs[0], np.kron(facs[1], facs[2])))
        face_psi.append(np.kron(B, B))
        face_w.append(np.kron(w, w))
    return dict(vol_phi=vol_phi, vol_dphi=vol_dphi, vol_w=vol_w,
                face_phi=np.stack(face_phi), face_psi=np.stack(face_psi),
                face_w=np.stack(face_w), n1d=t["n1d"], nq1=t["nq1"])


def face_normal(f: int) -> np.ndarray:
    n = np.zeros(3)
    n[FACE_AXIS[f]] = -1.0 if FACE_SIDE[f] == 0 else 1.0
    return n


def tangent_axes(f: int):
    d = FACE_AXIS[f]
    return tuple(a for a in range(3) if a != d)


def physical(h):
    """Scale factors of a macro with sub-element sizes h = (hx, hy, hz):
    volume weight factor, d/dx_j = (1/h_j) d/dxi_j, face weight factor."""
    h = np.asarray(h, dtype=np.float64)
    vol = h[..., 0] * h[..., 1] * h[..., 2]
    face = []
    for f in range(6):
        t1, t2 = tangent_axes(f)
        face.append(h[..., t1] * h[..., t2])
    return vol, 1.0 / h, np.stack(face, axis=-1)
