"""Tetrahedral macro-elements: spaces, quadrature and affine geometry (oracle, FP64).

Oracle test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import this package.  Nothing on the GPU
path depends on it.

Sec. 3.1 (geometric hierarchy, the local space W_p(K), Fig. 1): a
macro-element K is a tetrahedron resolved by a conforming submesh of eight
tetrahedra, continuous inside K and discontinuous across its boundary.
Here the submesh is the red refinement of K: the four corner tetrahedra cut
off at the edge midpoints, and the inner octahedron split into four
tetrahedra along one of its three diagonals (the paper does not say which;
this module always takes the diagonal between the midpoints of edges 0-2
and 1-3 of the reference macro-tetrahedron).

With equispaced Lagrange nodes of degree p on every sub-tetrahedron, the
nodes of all eight are exactly the points of the degree-2p lattice of K:
    n  = (2p+1)(2p+2)(2p+3)/6 nodes   (84 at p = 3),
and the trace space on a macro-face, the restriction of W_p(K) to it
(continuous piecewise P_p on the face's four sub-triangles), has
    nf = (2p+1)(2p+2)/2 nodes         (28 at p = 3),
the counts behind the degree-of-freedom tables of Sec. 7.

Reference macro-tetrahedron: vertices V0 = (0,0,0), V1 = (1,0,0),
V2 = (0,1,0), V3 = (0,0,1).  Macro node a sits at (i,j,k)/(2p) with
i + j + k <= 2p, ordered with i fastest, then j, then k.  Face f is the
face opposite vertex f; its vertices are the other three in increasing
order (P0, P1, P2), and face node c sits at P0 + (i (P1-P0) + j (P2-P0))/(2p)
with i + j <= 2p, i fastest.

Quadrature (the paper gives none for simplices): on each sub-tetrahedron
the collapsed-coordinate (Stroud conical product) rule with p+1 points per
direction, exact for total degree 2p+1, the same exactness per direction as
the p+1 Gauss points per sub-interval used on hexahedra; on each face
sub-triangle the matching two-dimensional collapsed rule.

A physical macro-element is the affine image x = X0 + J xi of the
reference one (J = [X1-X0, X2-X0, X3-X0]), so physical gradients are
J^-T times reference gradients and the weights scale by |det J|; face
weights scale by |(X_P1 - X_P0) x (X_P2 - X_P0)|, and the outward normal
is constant per face.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np
from scipy.special import roots_jacobi

VERTS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


# --------------------------------------------------------------------------
# counts and lattices
# --------------------------------------------------------------------------
def n_nodes(p: int) -> int:
    """Macro nodes of a tetrahedral macro-element of degree p."""
    m = 2 * p
    return (m + 1) * (m + 2) * (m + 3) // 6


def nf_nodes(p: int) -> int:
    """Trace nodes on one macro-face."""
    m = 2 * p
    return (m + 1) * (m + 2) // 2


def lattice3(m: int) -> np.ndarray:
    """Integer points (i, j, k), i + j + k <= m, i fastest: [N][3]."""
    return np.array([(i, j, k) for k in range(m + 1) for j in range(m + 1 - k)
                     for i in range(m + 1 - j - k)], dtype=np.int64)


def lattice2(m: int) -> np.ndarray:
    """Integer points (i, j), i + j <= m, i fastest: [N][2]."""
    return np.array([(i, j) for j in range(m + 1) for i in range(m + 1 - j)], dtype=np.int64)


def _index3(m):
    return {tuple(int(x) for x in r): a for a, r in enumerate(lattice3(m))}


def _index2(m):
    return {tuple(int(x) for x in r): a for a, r in enumerate(lattice2(m))}


# --------------------------------------------------------------------------
# red refinement
# --------------------------------------------------------------------------
def subtets() -> np.ndarray:
    """The eight sub-tetrahedra [8][4][3] in half-units (vertex coordinates
    times 2: corners at 0 or 2, edge midpoints at 1)."""
    V = (2 * VERTS).astype(np.int64)
    mid = {(a, b): (V[a] + V[b]) // 2 for a in range(4) for b in range(a + 1, 4)}
    corner = [
        [V[0], mid[0, 1], mid[0, 2], mid[0, 3]],
        [mid[0, 1], V[1], mid[1, 2], mid[1, 3]],
        [mid[0, 2], mid[1, 2], V[2], mid[2, 3]],
        [mid[0, 3], mid[1, 3], mid[2, 3], V[3]],
    ]
    # octahedron around the diagonal m02 - m13; the other four midpoints form
    # the cycle m01, m12, m23, m03 (consecutive ones share a vertex of K)
    ring = [mid[0, 1], mid[1, 2], mid[2, 3], mid[0, 3]]
    inner = [[mid[0, 2], mid[1, 3], ring[i], ring[(i + 1) % 4]] for i in range(4)]
    return np.array(corner + inner, dtype=np.int64)


def face_vertices(f: int):
    """Vertices (P0, P1, P2) of face f (opposite vertex f), increasing."""
    return tuple(v for v in range(4) if v != f)


def subtris() -> np.ndarray:
    """The four sub-triangles [4][3][2] of the face parameter triangle
    {(s, t): s, t >= 0, s + t <= 1} in half-units."""
    return np.array([[[0, 0], [1, 0], [0, 1]],
                     [[1, 0], [2, 0], [1, 1]],
                     [[0, 1], [1, 1], [0, 2]],
                     [[1, 0], [1, 1], [0, 1]]], dtype=np.int64)


# --------------------------------------------------------------------------
# Lagrange bases on simplices (equispaced nodes)
# --------------------------------------------------------------------------
def _exponents(p, dim):
    return [e for e in itertools.product(range(p + 1), repeat=dim) if sum(e) <= p]


def _monomials(x, p):
    """Values and gradients of the monomials of total degree <= p at points
    x [N][dim]: V [N][nm], dV [dim][N][nm]."""
    x = np.atleast_2d(x)
    dim = x.shape[1]
    ex = _exponents(p, dim)
    V = np.ones((x.shape[0], len(ex)))
    dV = np.zeros((dim, x.shape[0], len(ex)))
    for c, e in enumerate(ex):
        for d in range(dim):
            V[:, c] *= x[:, d] ** e[d]
        for d in range(dim):
            if e[d] == 0:
                continue
            g = e[d] * x[:, d] ** (e[d] - 1)
            for d2 in range(dim):
                if d2 != d:
                    g = g * x[:, d2] ** e[d2]
            dV[d, :, c] = g
    return V, dV


@functools.lru_cache(maxsize=None)
def _lagrange_coef(p, dim):
    """Coefficients C [nm][nn]: the Lagrange function of local node b is
    monomials(x) @ C[:, b], nodes = lattice/p (i fastest)."""
    nodes = (lattice3(p) if dim == 3 else lattice2(p)) / float(p)
    V, _ = _monomials(nodes, p)
    return np.linalg.inv(V)


def lagrange(x, p, dim):
    """Values [N][nn] and reference gradients [dim][N][nn] of the degree-p
    Lagrange basis on the unit simplex of dimension ``dim`` at x [N][dim]."""
    C = _lagrange_coef(p, dim)
    V, dV = _monomials(x, p)
    return V @ C, np.einsum("dnm,mb->dnb", dV, C)


# --------------------------------------------------------------------------
# collapsed Gauss-Jacobi quadrature
# --------------------------------------------------------------------------
def _gj01(q, alpha):
    """q-point Gauss rule on [0, 1] for the weight (1 - t)^alpha."""
    x, w = roots_jacobi(q, alpha, 0.0)
    return (x + 1.0) / 2.0, w / 2.0 ** (alpha + 1)


def tet_rule(q):
    """Points [q^3][3] and weights on the unit tetrahedron (volume 1/6),
    exact for total degree 2q-1: x = a(1-b)(1-c), y = b(1-c), z = c."""
    a, wa = _gj01(q, 0.0)
    b, wb = _gj01(q, 1.0)
    c, wc = _gj01(q, 2.0)
    pts, wts = [], []
    for k in range(q):
        for j in range(q):
            for i in range(q):
                pts.append([a[i] * (1 - b[j]) * (1 - c[k]), b[j] * (1 - c[k]), c[k]])
                wts.append(wa[i] * wb[j] * wc[k])
    return np.array(pts), np.array(wts)


def tri_rule(q):
    """Points [q^2][2] and weights on the unit triangle (area 1/2), exact for
    total degree 2q-1: s = a(1-b), t = b."""
    a, wa = _gj01(q, 0.0)
    b, wb = _gj01(q, 1.0)
    pts, wts = [], []
    for j in range(q):
        for i in range(q):
            pts.append([a[i] * (1 - b[j]), b[j]])
            wts.append(wa[i] * wb[j])
    return np.array(pts), np.array(wts)


# --------------------------------------------------------------------------
# reference tables of one macro-element
# --------------------------------------------------------------------------
def _subtet_nodes(p, T, idx):
    """Macro node index of each local node of sub-tet T (half-units)."""
    L = T * p                      # lattice units of the degree-2p lattice
    out = []
    for (al, be, ga) in lattice3(p):
        pos = L[0] * p + al * (L[1] - L[0]) + be * (L[2] - L[0]) + ga * (L[3] - L[0])
        out.append(idx[tuple(int(x) for x in pos // p)])
    return np.array(out, dtype=np.int64)


def _eval_in_subtet(p, T, xi, n, idx):
    """Macro basis values [N][n] and reference gradients [3][N][n] at points
    xi [N][3] of sub-tet T."""
    W = T / 2.0
    B = (W[1:] - W[0]).T                    # columns: edges of the sub-tet
    eta = np.linalg.solve(B, (xi - W[0]).T).T
    val, grad = lagrange(eta, p, 3)         # gradients in eta
    gx = np.einsum("ie,enb->inb", np.linalg.inv(B).T, grad)
    nodes = _subtet_nodes(p, T, idx)
    Phi = np.zeros((xi.shape[0], n))
    dPhi = np.zeros((3, xi.shape[0], n))
    Phi[:, nodes] = val
    dPhi[:, :, nodes] = gx
    return Phi, dPhi


def _containing_subtet(xi, tol=1e-12):
    """Index of a sub-tet whose closure holds the point xi [3]."""
    for s, T in enumerate(subtets()):
        W = T / 2.0
        lam = np.linalg.solve((W[1:] - W[0]).T, xi - W[0])
        if lam.min() >= -tol and lam.sum() <= 1.0 + tol:
            return s
    raise ValueError("point outside the reference macro-element")


@functools.lru_cache(maxsize=None)
def reference_tables(p: int):
    """Dense tables of the reference macro-tetrahedron.

    vol_xi [G][3], vol_w [G] (reference weights, summing to 1/6),
    vol_phi [G][n], vol_dphi [3][G][n] (d/dxi_i), vol_sub [G] (sub-tet of
    each point);
    per face f (0..3): face_xi [4][S][3], face_w [4][S] (weights of the
    face parameter triangle, summing to 1/2), face_phi [4][S][n] (macro
    basis on the face), face_psi [4][S][nf] (trace basis), face_nodes
    [4][nf] (macro node at each trace node).
    """
    m = 2 * p
    n, nf = n_nodes(p), nf_nodes(p)
    idx3, idx2 = _index3(m), _index2(m)
    lat = lattice3(m)
    q = p + 1

    tp, tw = tet_rule(q)
    xs, ws, ph, dph, sub = [], [], [], [], []
    for s, T in enumerate(subtets()):
        W = T / 2.0
        B = (W[1:] - W[0]).T
        xi = W[0] + tp @ B.T
        P_, D_ = _eval_in_subtet(p, T, xi, n, idx3)
        xs.append(xi)
        ws.append(tw * abs(np.linalg.det(B)))
        ph.append(P_)
        dph.append(D_)
        sub.append(np.full(tp.shape[0], s))
    vol_xi = np.concatenate(xs)
    vol_w = np.concatenate(ws)
    vol_phi = np.concatenate(ph)
    vol_dphi = np.concatenate(dph, axis=1)
    vol_sub = np.concatenate(sub)

    fp, fw = tri_rule(q)
    face_xi, face_w, face_phi, face_psi, face_nodes = [], [], [], [], []
    for f in range(4):
        P0, P1, P2 = (VERTS[v] for v in face_vertices(f))
        L0, L1, L2 = (np.rint(VERTS[v] * m).astype(np.int64) for v in face_vertices(f))
        fn = []
        for (i, j) in lattice2(m):
            pos = L0 * m + i * (L1 - L0) + j * (L2 - L0)
            fn.append(idx3[tuple(int(x) for x in pos // m)])
        fn = np.array(fn, dtype=np.int64)
        X, Wt, Ph, Ps = [], [], [], []
        for tri in subtris():
            A = tri / 2.0
            E = (A[1:] - A[0]).T                          # 2x2
            st = A[0] + fp @ E.T                          # face parameters
            xi = P0 + st[:, :1] * (P1 - P0) + st[:, 1:2] * (P2 - P0)
            # trace basis: degree-p Lagrange on the sub-triangle
            loc, _ = lagrange(fp, p, 2)
            psi = np.zeros((fp.shape[0], nf))
            La = tri * p
            for b, (al, be) in enumerate(lattice2(p)):
                pos = La[0] * p + al * (La[1] - La[0]) + be * (La[2] - La[0])
                psi[:, idx2[tuple(int(x) for x in pos // p)]] = loc[:, b]
            # macro basis: evaluated in the sub-tet holding the sub-triangle
            s = _containing_subtet(xi.mean(axis=0))
            Pv, _ = _eval_in_subtet(p, subtets()[s], xi, n, idx3)
            X.append(xi)
            Wt.append(fw * abs(np.linalg.det(E)))
            Ph.append(Pv)
            Ps.append(psi)
        face_xi.append(np.concatenate(X))
        face_w.append(np.concatenate(Wt))
        face_phi.append(np.concatenate(Ph))
        face_psi.append(np.concatenate(Ps))
        face_nodes.append(fn)
    return dict(n=n, nf=nf, lattice=lat, vol_xi=vol_xi, vol_w=vol_w, vol_phi=vol_phi,
                vol_dphi=vol_dphi, vol_sub=vol_sub, face_xi=np.stack(face_xi),
                face_w=np.stack(face_w), face_phi=np.stack(face_phi),
                face_psi=np.stack(face_psi), face_nodes=np.stack(face_nodes))


# --------------------------------------------------------------------------
# physical macro-elements
# --------------------------------------------------------------------------
class TetGeometry:
    """Affine tetrahedral macro-elements X [M][4][3] (vertex coordinates).

    Provides the table interface of ``forms``: phi, dphi, wv, and per face
    face_phi, face_psi, ws, normal."""

    nfaces = 4

    def __init__(self, p, X):
        self.p = p
        self.t = reference_tables(p)
        X = np.asarray(X, dtype=np.float64)
        if X.ndim != 3 or X.shape[1:] != (4, 3):
            raise ValueError("X must be [M][4][3]")
        self.X = X
        self.M = X.shape[0]
        self.n, self.nf = self.t["n"], self.t["nf"]
        J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)  # columns
        self.detJ = np.linalg.det(J)
        if np.any(np.abs(self.detJ) < 1e-300):
            raise ValueError("degenerate macro-element")
        self.invJT = np.linalg.inv(J).transpose(0, 2, 1)
        self.phi = self.t["vol_phi"]
        self.wv = np.abs(self.detJ)[:, None] * self.t["vol_w"][None, :]
        # dphi[m, j, g, a] = sum_i (J^-1)_{ij} d phi_a / d xi_i
        self.dphi = np.einsum("mji,iga->mjga", self.invJT, self.t["vol_dphi"])
        self._area, self._normal = [], []
        for f in range(4):
            P0, P1, P2 = face_vertices(f)
            cr = np.cross(X[:, P1] - X[:, P0], X[:, P2] - X[:, P0])
            a = np.linalg.norm(cr, axis=1)
            nrm = cr / a[:, None]
            out = np.einsum("mi,mi->m", nrm, X[:, P0] - X[:, f]) > 0.0
            self._normal.append(np.where(out[:, None], nrm, -nrm))
            self._area.append(a)

    def face_phi(self, f):
        return self.t["face_phi"][f]

    def face_psi(self, f):
        return self.t["face_psi"][f]

    def ws(self, f):
        """Physical face weights [M][S]."""
        return self._area[f][:, None] * self.t["face_w"][f][None, :]

    def normal(self, f):
        """Outward unit normal [M][3] of face f."""
        return self._normal[f]
