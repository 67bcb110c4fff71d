"""Seeded synthetic inputs for the macro-element HDG local work.

This module is the one place where inputs are made.  Both the FP64 CPU
oracle (``oracle/``) and the HIP library receive exactly the arrays built
here; the module computes nothing of the method itself (no inverse map
u(v), no fluxes, no quadrature, no algebra).  It only

* lays out structured boxes of hexahedral macro-elements, each split into
  2x2x2 sub-elements of degree p (the layout of the nodal arrays below),
* samples the paper's analytic initial states at the node positions:
  the advected isentropic vortex (Sec. 7.1, eq. S601) and the
  Taylor-Green vortex (Sec. 7.2, eq. TGV0),
* writes those states in the unknowns' own variables, the entropy
  variables of eq. (s222) -- this is the definition of the input, the hot
  path only ever evaluates the inverse map,
* adds seeded uniform noise so that every interface has a non-zero jump,
* turns a workload's physical constants into the numeric parameter set
  that both sides consume (Sec. 2.1 eq. C6, Sec. 3.2 viscous penalty,
  Sec. 5.3 time term).

Array layouts (all float64, C order):

* ``v``      [n_macro][5][n]        nodal entropy variables, node index
  a = i + n1d*(j + n1d*k), n1d = 2p+1, n = n1d**3;
* ``vhat``   [n_macro][6][5][n1d*n1d] per-macro gathered trace, faces
  ordered (-x, +x, -y, +y, -z, +z), face node c = c1 + n1d*c2 with
  (c1, c2) the node indices along the two tangential axes in increasing
  axis order;
* ``v_old``  [n_macro][5][n]        state the time term is taken against;
* ``origin``, ``h`` [n_macro][3]   lower corner and sub-element edge
  lengths (a macro-element spans 2*h per axis).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

N_VAR = 5

# Positions of the Gauss-Lobatto-Legendre points on [-1, 1] for the degrees
# used here.  They fix where the nodal values of the arrays above sit; they
# are the layout convention of the input, not part of any computation.
_GLL_CLOSED_FORM = {
    1: [-1.0, 1.0],
    2: [-1.0, 0.0, 1.0],
    3: [-1.0, -1.0 / math.sqrt(5.0), 1.0 / math.sqrt(5.0), 1.0],
    4: [-1.0, -math.sqrt(3.0 / 7.0), 0.0, math.sqrt(3.0 / 7.0), 1.0],
}


def node_positions_1d(p: int) -> np.ndarray:
    """Reference positions in [0, 2] of the 2p+1 nodes along one macro axis.

    Two sub-intervals [0,1] and [1,2], each carrying the p+1 GLL points; the
    middle node is shared (C0 continuity inside the macro-element).
    """
    g = np.asarray(_GLL_CLOSED_FORM[p])
    left = (g + 1.0) / 2.0
    return np.concatenate([left, 1.0 + left[1:]])


def sizes(p: int) -> dict:
    n1d = 2 * p + 1
    n = n1d ** 3
    nf = n1d * n1d
    return dict(n1d=n1d, n=n, nf=nf, N_V=5 * n, N_Q=15 * n, N_VH=30 * nf)


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Mesh:
    shape: tuple            # macros per axis (nx, ny, nz)
    lo: np.ndarray          # [3]
    hi: np.ndarray          # [3]
    origin: np.ndarray      # [n_macro][3]
    h: np.ndarray           # [n_macro][3] sub-element size
    ijk: np.ndarray         # [n_macro][3] integer macro coordinates

    @property
    def n_macro(self) -> int:
        return int(self.origin.shape[0])


def box_mesh(shape, lo, hi) -> Mesh:
    shape = tuple(int(s) for s in shape)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    size = (hi - lo) / np.asarray(shape, dtype=np.float64)
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)  # x fastest
    origin = lo[None, :] + ijk * size[None, :]
    h = np.broadcast_to(size / 2.0, origin.shape).copy()
    return Mesh(shape, lo, hi, origin, h, ijk)


def node_coords(mesh: Mesh, p: int) -> np.ndarray:
    """Physical coordinates [n_macro][3][n] of the nodes."""
    xi = node_positions_1d(p)
    n1d = xi.size
    a = np.arange(n1d ** 3)
    idx = np.stack([a % n1d, (a // n1d) % n1d, a // (n1d * n1d)], axis=0)  # [3][n]
    return mesh.origin[:, :, None] + mesh.h[:, :, None] * xi[idx][None, :, :]


FACE_AXIS = (0, 0, 1, 1, 2, 2)
FACE_SIDE = (0, 1, 0, 1, 0, 1)


def face_tangent_axes(f: int):
    d = FACE_AXIS[f]
    return tuple(ax for ax in range(3) if ax != d)


def face_node_coords(mesh: Mesh, p: int) -> np.ndarray:
    """Physical coordinates [n_macro][6][3][nf] of the trace nodes."""
    xi = node_positions_1d(p)
    n1d = xi.size
    c = np.arange(n1d * n1d)
    c1, c2 = c % n1d, c // n1d
    out = np.empty((mesh.n_macro, 6, 3, n1d * n1d))
    for f in range(6):
        d = FACE_AXIS[f]
        t1, t2 = face_tangent_axes(f)
        ref = np.empty((3, n1d * n1d))
        ref[d] = 2.0 * FACE_SIDE[f]
        ref[t1] = xi[c1]
        ref[t2] = xi[c2]
        out[:, f] = mesh.origin[:, :, None] + mesh.h[:, :, None] * ref[None]
    return out


def global_face_ids(mesh: Mesh) -> np.ndarray:
    """Index [n_macro][6] of the global (periodic) macro-face each local face is.

    Faces normal to axis d are numbered by the macro on their + side, so the
    +d face of macro (i,j,k) is the same global face as the -d face of its
    periodic neighbour.
    """
    nx, ny, nz = mesh.shape
    n = np.array(mesh.shape)
    out = np.empty((mesh.n_macro, 6), dtype=np.int64)
    per_axis = nx * ny * nz
    for f in range(6):
        d = FACE_AXIS[f]
        ijk = mesh.ijk.copy()
        if FACE_SIDE[f] == 1:
            ijk[:, d] = (ijk[:, d] + 1) % n[d]
        flat = ijk[:, 0] + nx * (ijk[:, 1] + ny * ijk[:, 2])
        out[:, f] = d * per_axis + flat
    return out


# --------------------------------------------------------------------------
# analytic states (primitive variables) and their entropy-variable form
# --------------------------------------------------------------------------
def tgv_primitive(x, M0, gamma):
    """Taylor-Green vortex initial state, Sec. 7.2 eq. (TGV0), L = rho0 = 1.

    p0 = 1/gamma (so c0 = 1), V0 = M0 c0, isothermal: P/rho = P0/rho0.
    """
    X, Y, Z = x[..., 0, :], x[..., 1, :], x[..., 2, :]
    V0 = M0
    u = V0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    w = -V0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    z = np.zeros_like(u)
    P = 1.0 / gamma + V0 ** 2 / 16.0 * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    rho = gamma * P
    return rho, np.stack([u, w, z], axis=-2), P


def vortex_primitive(x, t, eps, Minf, gamma, x0=5.0, y0=5.0, Vinf=1.0, alpha=0.0):
    """Advected isentropic vortex, Sec. 7.1 eq. (S601), rho_inf = 1.

    P_inf = 1/(gamma Minf^2) makes the free-stream Mach number Minf at Vinf = 1.
    """
    X, Y = x[..., 0, :], x[..., 1, :]
    dx = X - x0 - Vinf * math.cos(alpha) * t
    dy = Y - y0 - Vinf * math.sin(alpha) * t
    r2 = dx * dx + dy * dy
    Pinf = 1.0 / (gamma * Minf * Minf)
    rho = (1.0 - eps * eps * (gamma - 1.0) * Minf * Minf / (8.0 * math.pi ** 2)
           * np.exp(1.0 - r2)) ** (1.0 / (gamma - 1.0))
    e = np.exp((1.0 - r2) / 2.0)
    u = Vinf * (math.cos(alpha) - eps * dy / (2.0 * math.pi) * e)
    w = Vinf * (math.sin(alpha) + eps * dx / (2.0 * math.pi) * e)
    z = np.zeros_like(u)
    P = Pinf * rho ** gamma
    return rho, np.stack([u, w, z], axis=-2), P


def entropy_variables(rho, V, P, gamma):
    """Entropy variables of a primitive state, eq. (s222):
    v = [(gamma - s)/(gamma-1) - beta |V|^2/2, beta V, -beta], beta = rho/P,
    s = log(P / rho^gamma).  V carries the velocity components on axis -2.
    """
    beta = rho / P
    s = np.log(P) - gamma * np.log(rho)
    V2 = np.sum(V * V, axis=-2)
    v1 = (gamma - s) / (gamma - 1.0) - beta * V2 / 2.0
    comps = [v1] + [beta * V[..., i, :] for i in range(3)] + [-beta]
    return np.stack(comps, axis=-2)


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
FLUX_EC, FLUX_ES, FLUX_KEPES = 0, 1, 2
FLUX_NAMES = {"EC": FLUX_EC, "ES": FLUX_ES, "KEPES": FLUX_KEPES}


def dirk33_diagonal() -> float:
    """Diagonal coefficient of Alexander's L-stable three-stage DIRK(3,3):
    the root in (1/6, 1/2) of x^3 - 3x^2 + 3x/2 - 1/6."""
    r = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
    r = [float(x.real) for x in r if abs(x.imag) < 1e-12 and 1.0 / 6.0 < x.real < 0.5]
    return r[0]


def make_params(*, gamma=1.4, viscous=False, Re=None, M0=None, Pr=0.71, dt=None,
                flux="ES", alpha_ps=1.0, logmean_eps=1e-4, T_wall=1.0) -> dict:
    """Numeric parameter set consumed by both the oracle and the library.

    * mu = mu/Re_c with mu = 1 and the acoustic Reynolds number
      Re_c = Re/M0 (eq. C6 with c0 = 1);
    * kappa multiplies grad T in the heat flux: mu/Re_c / (Pr (gamma-1));
    * lam = -2/3 (Stokes hypothesis);
    * sigma_vis = (1/Re) diag(0, 1, 1, 1, 1/((gamma-1) M0^2 Pr)) (Sec. 3.2);
    * alpha_t = 1/(a_11 dt): first DIRK(3,3) stage, time term
      alpha_t (u(v) - u(v_old)) (eq. C242);
    * alpha_ps: pseudo-time continuation, 1/tau_init with tau_init = 1
      (Sec. 6.1), added to the Jacobian only.
    """
    aii = dirk33_diagonal()
    prm = dict(gamma=float(gamma), mu=0.0, kappa=0.0, lam=-2.0 / 3.0,
               sigma_vis=[0.0] * 5, alpha_t=0.0 if dt is None else 1.0 / (aii * dt),
               alpha_ps=float(alpha_ps), logmean_eps=float(logmean_eps),
               flux=FLUX_NAMES[flux] if isinstance(flux, str) else int(flux),
               viscous=int(bool(viscous)), T_wall=float(T_wall))
    if viscous:
        mu = M0 / Re
        prm["mu"] = mu
        prm["kappa"] = mu / (Pr * (gamma - 1.0))
        prm["sigma_vis"] = [0.0, 1.0 / Re, 1.0 / Re, 1.0 / Re,
                            1.0 / (Re * (gamma - 1.0) * M0 * M0 * Pr)]
    return prm


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    p: int
    mesh: Mesh
    params: dict
    v: np.ndarray
    vhat: np.ndarray
    v_old: np.ndarray
    face_bc: np.ndarray      # [n_macro][6] uint8: 0 interior/periodic, 1 wall
    q: Optional[np.ndarray] = None

    @property
    def n_macro(self):
        return self.mesh.n_macro


def _noise(rng, shape, amp):
    return rng.uniform(-amp, amp, size=shape)


def _build(name, p, mesh, params, prim_fn, seed_v, seed_vh, amp=1e-3, noise_vhat=True):
    gamma = params["gamma"]
    xn = node_coords(mesh, p)
    v_clean = entropy_variables(*prim_fn(xn), gamma)
    xf = face_node_coords(mesh, p)                       # [M][6][3][nf]
    vh_clean = entropy_variables(*prim_fn(xf), gamma)    # [M][6][5][nf]
    v = v_clean.copy()
    if seed_v is not None:
        v += _noise(np.random.default_rng(seed_v), v.shape, amp)
    vhat = vh_clean.copy()
    if noise_vhat and seed_vh is not None:
        # one noise sample per global face node, shared by both sides
        gid = global_face_ids(mesh)
        nf = vhat.shape[-1]
        table = _noise(np.random.default_rng(seed_vh), (int(gid.max()) + 1, 5, nf), amp)
        vhat += table[gid]
    face_bc = np.zeros((mesh.n_macro, 6), dtype=np.uint8)
    return Workload(name, p, mesh, params, np.ascontiguousarray(v),
                    np.ascontiguousarray(vhat), np.ascontiguousarray(v_clean), face_bc)


def vortex_workload(shape=(2, 2, 2), p=2, eps=5.0, Minf=0.85, dt=1e-3, flux="EC",
                    seed_v=11, seed_vh=12, amp=1e-3, lo=(0.0, 0.0, 0.0), hi=(10.0, 10.0, 10.0)):
    """Euler, periodic cube [0,10]^3, isentropic vortex of strength eps."""
    gamma = 1.4
    mesh = box_mesh(shape, lo, hi)
    prm = make_params(gamma=gamma, viscous=False, dt=dt, flux=flux)
    return _build("vortex", p, mesh, prm,
                  lambda x: vortex_primitive(x, 0.0, eps, Minf, gamma),
                  seed_v, seed_vh, amp)


def tgv_workload(shape=(16, 16, 16), p=2, M0=0.1, Re=1600.0, Pr=0.71, viscous=True,
                 flux="ES", seed_v=21, seed_vh=22, amp=1e-3, noise_vhat=True):
    """Taylor-Green vortex on the periodic box [0, 2pi]^3, dt = 0.057 t_c."""
    gamma = 1.4
    mesh = box_mesh(shape, (0.0, 0.0, 0.0), (2 * math.pi,) * 3)
    dt = 0.057 / M0
    prm = make_params(gamma=gamma, viscous=viscous, Re=Re, M0=M0, Pr=Pr, dt=dt, flux=flux)
    return _build("tgv", p, mesh, prm, lambda x: tgv_primitive(x, M0, gamma),
                  seed_v, seed_vh, amp, noise_vhat)


def mixed_degree_tgv(shape=(16, 16, 16), degrees=(1, 2, 3), seed_p=41, M0=0.1, Re=1600.0, flux="ES",
                     seed_v=43, seed_vh=44, wall_frac=0.2, seed_wall=42):
    """Viscous Taylor-Green box whose macro-elements take degrees drawn
    uniformly (seeded) from ``degrees``, with the -z face of a seeded
    fraction ``wall_frac`` of the macros flagged as an isothermal wall.
    Returns (p [n_macro], face_bc [n_macro][6], parts) with parts[d] the
    workload of the macros of degree d (in macro order, face_bc included),
    each sampled from the box at its own degree."""
    mesh = box_mesh(shape, (0.0, 0.0, 0.0), (2 * math.pi,) * 3)
    deg = np.asarray(degrees, dtype=np.int64)
    p = deg[np.random.default_rng(seed_p).integers(0, deg.size, mesh.n_macro)]
    face_bc = np.zeros((mesh.n_macro, 6), dtype=np.uint8)
    face_bc[np.random.default_rng(seed_wall).permutation(mesh.n_macro)[:int(round(wall_frac * mesh.n_macro))], 4] = 1
    parts = {}
    for d in sorted(set(p.tolist())):
        w = tgv_workload(shape=shape, p=d, M0=M0, Re=Re, flux=flux, seed_v=seed_v, seed_vh=seed_vh)
        w.face_bc = face_bc
        parts[d] = subset(w, np.nonzero(p == d)[0])
    return p, face_bc, parts


def workload(config: int, shape=None):
    """The five workloads of the hot-path study, optionally on a smaller box."""
    if config == 1:
        return vortex_workload(shape=shape or (2, 2, 2))
    if config == 2:
        return tgv_workload(shape=shape or (16, 16, 16), p=2, M0=0.1, Re=1600.0, flux="ES",
                            seed_v=21, seed_vh=22)
    if config == 3:
        return tgv_workload(shape=shape or (8, 8, 8), p=2, M0=0.4, viscous=False, flux="ES",
                            seed_v=31, seed_vh=None, noise_vhat=False)
    if config == 5:
        return tgv_workload(shape=shape or (16, 16, 8), p=3, M0=0.3, Re=5000.0, flux="KEPES",
                            seed_v=51, seed_vh=52)
    raise ValueError(f"unknown workload {config}")


def subset(w: Workload, idx) -> Workload:
    """The same workload restricted to the macro-elements ``idx``."""
    idx = np.asarray(idx)
    m = w.mesh
    mesh = Mesh(m.shape, m.lo, m.hi, m.origin[idx], m.h[idx], m.ijk[idx])
    return Workload(w.name, w.p, mesh, w.params, np.ascontiguousarray(w.v[idx]),
                    np.ascontiguousarray(w.vhat[idx]), np.ascontiguousarray(w.v_old[idx]),
                    np.ascontiguousarray(w.face_bc[idx]),
                    None if w.q is None else np.ascontiguousarray(w.q[idx]))


# --------------------------------------------------------------------------
# tetrahedral macro-elements
# --------------------------------------------------------------------------
# Layout of a tetrahedral macro-element of degree p (the degree-2p lattice of
# its eight P_p sub-tetrahedra, Sec. 3.1):
#   * vertices X [4][3]; a point with reference coordinates xi (in the unit
#     tetrahedron (0,0,0), e_x, e_y, e_z) sits at X0 + sum_i xi_i (X_i - X0);
#   * node a at xi = (i, j, k)/(2p), i + j + k <= 2p, i fastest, then j, k:
#     n = (2p+1)(2p+2)(2p+3)/6 nodes;
#   * face f is opposite vertex f, with vertices (P0, P1, P2) the other three
#     in increasing order; face node c at P0 + (i (P1-P0) + j (P2-P0))/(2p),
#     i + j <= 2p, i fastest: nf = (2p+1)(2p+2)/2 nodes;
#   * ``vhat`` [n_macro][4][5][nf].

@dataclasses.dataclass
class TetMesh:
    shape: tuple            # cubes per axis
    lo: np.ndarray
    hi: np.ndarray
    X: np.ndarray           # [n_macro][4][3] vertex coordinates
    vid: np.ndarray         # [n_macro][4] periodic vertex ids

    @property
    def n_macro(self) -> int:
        return int(self.X.shape[0])


def tet_sizes(p: int) -> dict:
    m = 2 * p
    n = (m + 1) * (m + 2) * (m + 3) // 6
    nf = (m + 1) * (m + 2) // 2
    return dict(n=n, nf=nf, N_V=5 * n, N_Q=15 * n, N_VH=20 * nf)


def _lattice3(m):
    return np.array([(i, j, k) for k in range(m + 1) for j in range(m + 1 - k)
                     for i in range(m + 1 - j - k)], dtype=np.int64)


def _lattice2(m):
    return np.array([(i, j) for j in range(m + 1) for i in range(m + 1 - j)], dtype=np.int64)


def tet_box_mesh(shape, lo, hi) -> TetMesh:
    """Periodic box of cubes, each split into the six tetrahedra around its
    main diagonal (vertices c, c + e_a, c + e_a + e_b, c + (1,1,1) for the
    six orders (a, b) of the axes); conforming across cubes."""
    shape = tuple(int(s) for s in shape)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    size = (hi - lo) / np.asarray(shape, dtype=np.float64)
    nx, ny, nz = shape
    Xs, ids = [], []
    E = np.eye(3, dtype=np.int64)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = np.array([i, j, k], dtype=np.int64)
                for (a, b, _) in perms:
                    corners = [c, c + E[a], c + E[a] + E[b], c + 1]
                    Xs.append([lo + size * cc for cc in corners])
                    ids.append([int(cc[0] % nx + nx * (cc[1] % ny + ny * (cc[2] % nz))) for cc in corners])
    return TetMesh(shape, lo, hi, np.array(Xs, dtype=np.float64), np.array(ids, dtype=np.int64))


def tet_face_vertices(f: int):
    return tuple(v for v in range(4) if v != f)


def tet_node_coords(mesh: TetMesh, p: int) -> np.ndarray:
    """Physical coordinates [n_macro][3][n] of the macro nodes."""
    xi = _lattice3(2 * p) / (2.0 * p)                   # [n][3]
    X = mesh.X
    E = X[:, 1:] - X[:, :1]                             # [M][3 edges][3]
    return (X[:, 0, :, None] + np.einsum("ne,mec->mcn", xi, E))


def tet_face_node_coords(mesh: TetMesh, p: int) -> np.ndarray:
    """Physical coordinates [n_macro][4][3][nf] of the trace nodes."""
    ij = _lattice2(2 * p) / (2.0 * p)
    out = np.empty((mesh.n_macro, 4, 3, ij.shape[0]))
    for f in range(4):
        P0, P1, P2 = tet_face_vertices(f)
        X = mesh.X
        out[:, f] = (X[:, P0, :, None] + ij[None, None, :, 0] * (X[:, P1] - X[:, P0])[:, :, None]
                     + ij[None, None, :, 1] * (X[:, P2] - X[:, P0])[:, :, None])
    return out


def tet_global_faces(mesh: TetMesh, p: int):
    """(face id [n_macro][4], node id [n_macro][4][nf]): the global macro-face
    each local face is, and the global index of each of its trace nodes in a
    numbering shared by both sides of the face.  A trace node is named by its
    lattice weights on the face's three (periodic) vertex ids, sorted; this
    naming is one-to-one only with at least three cubes per axis."""
    if min(mesh.shape) < 3:
        raise ValueError("periodic face numbering needs at least 3 cubes per axis")
    m = 2 * p
    ij = _lattice2(m)
    keys, fid = {}, np.empty((mesh.n_macro, 4), dtype=np.int64)
    nodes = np.empty((mesh.n_macro, 4, ij.shape[0]), dtype=np.int64)
    for t in range(mesh.n_macro):
        for f in range(4):
            vs = [int(mesh.vid[t, v]) for v in tet_face_vertices(f)]
            key = tuple(sorted(vs))
            fid[t, f] = keys.setdefault(key, len(keys))
            for c, (i, j) in enumerate(ij):
                wts = {vs[0]: m - i - j, vs[1]: i, vs[2]: j}
                w_sorted = [wts[g] for g in key]        # weights on sorted vertices
                # index of (w1, w2) in the same lattice order
                a, b = w_sorted[1], w_sorted[2]
                nodes[t, f, c] = fid[t, f] * ij.shape[0] + int(b * (m + 1) - b * (b - 1) // 2 + a)
    return fid, nodes


@dataclasses.dataclass
class TetWorkload:
    name: str
    p: int
    mesh: TetMesh
    params: dict
    v: np.ndarray            # [n_macro][5][n]
    vhat: np.ndarray         # [n_macro][4][5][nf]
    v_old: np.ndarray
    face_bc: np.ndarray      # [n_macro][4]

    @property
    def n_macro(self):
        return self.mesh.n_macro


def tet_tgv_workload(shape=(2, 2, 2), p=2, M0=0.1, Re=1600.0, Pr=0.71, viscous=True, flux="ES",
                     seed_v=61, seed_vh=62, amp=1e-3):
    """Taylor-Green vortex on the periodic box [0, 2pi]^3 of tetrahedral
    macro-elements (six per cube, as in the paper's tetrahedral meshes of
    Sec. 7.2), dt = 0.057 t_c."""
    gamma = 1.4
    mesh = tet_box_mesh(shape, (0.0, 0.0, 0.0), (2 * math.pi,) * 3)
    prm = make_params(gamma=gamma, viscous=viscous, Re=Re, M0=M0, Pr=Pr, dt=0.057 / M0, flux=flux)
    prim = lambda x: tgv_primitive(x, M0, gamma)
    v_clean = entropy_variables(*prim(tet_node_coords(mesh, p)), gamma)
    vhat = entropy_variables(*prim(tet_face_node_coords(mesh, p)), gamma)   # [M][4][5][nf]
    v = v_clean.copy()
    if seed_v is not None:
        v += _noise(np.random.default_rng(seed_v), v.shape, amp)
    if seed_vh is not None and min(mesh.shape) >= 3:
        # one noise sample per global trace node, shared by both sides
        _, nodes = tet_global_faces(mesh, p)
        table = _noise(np.random.default_rng(seed_vh), (int(nodes.max()) + 1, 5), amp)
        vhat += table[nodes].transpose(0, 1, 3, 2)
    elif seed_vh is not None:
        # boxes too small for the periodic naming: independent noise per side
        vhat += _noise(np.random.default_rng(seed_vh), vhat.shape, amp)
    return TetWorkload("tet_tgv", p, mesh, prm, np.ascontiguousarray(v), np.ascontiguousarray(vhat),
                       np.ascontiguousarray(v_clean), np.zeros((mesh.n_macro, 4), dtype=np.uint8))
