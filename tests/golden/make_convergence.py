"""Writes tests/golden/convergence.txt: L2 errors of the oracle's discrete
solution against closed-form Euler solutions on periodic meshes of
macro-elements, for the p+1 convergence pin (Sec. 7.1 reports optimal
order p+1 for the advected isentropic vortex).

Calls only the oracle (global trace solve + DIRK(3,3)) and the closed-form
input fields.  Cases:
  wave    advected density wave rho = 1 + 0.2 sin(2 pi (x + y)), V = (0.5, 0.25, 0),
          P = 1, on [0,1]^2 x [0, 1/N] with N x N x 1 macros (smooth and periodic,
          so tiny meshes are already in the asymptotic range);
  vortex  isentropic vortex eps = 2.5, Minf = 0.5 advected at unit speed on
          [0,10]^2 x [0, 10/N] with N x N x 1 macros.
Entropy-stable flux (eq. Flux_En_Inv; the central entropy-conservative flux
leaves the global trace system singular), dt proportional to h.  Run:
    python -m tests.golden.make_convergence [wave|vortex|all]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

from oracle import basis, global_solve, local, physics
from paper_2507_22195_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GAMMA = 1.4


def wave_primitive(x, t):
    V1, V2 = 0.5, 0.25
    X, Y = x[..., 0, :], x[..., 1, :]
    rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * ((X - V1 * t) + (Y - V2 * t)))
    V = np.stack([np.full_like(X, V1), np.full_like(X, V2), np.zeros_like(X)], axis=-2)
    P = np.ones_like(X)
    return rho, V, P


def vortex_primitive(x, t):
    return W.vortex_primitive(x, t, 2.5, 0.5, GAMMA)


CASES = {
    # kind: (primitive, domain length in x/y, final time, dt at N = 1)
    "wave": (wave_primitive, 1.0, 0.2, 0.1),
    "vortex": (vortex_primitive, 10.0, 1.0, 0.5),
}


def setup(kind, p, N):
    """Mesh, parameters, initial state (nodal interpolant) and time steps of one case."""
    prim, L, T, dt1 = CASES[kind]
    mesh = W.box_mesh((N, N, 1), (0.0, 0.0, 0.0), (L, L, L / N))
    prm = W.make_params(gamma=GAMMA, flux="ES", dt=1.0, alpha_ps=0.0)
    xn = W.node_coords(mesh, p)
    v = W.entropy_variables(*prim(xn, 0.0), GAMMA)
    ids, nfaces = global_solve.periodic_face_ids(mesh.shape, mesh.ijk)
    xf = W.face_node_coords(mesh, p)                          # [M][6][3][nf]
    vh_loc = W.entropy_variables(*prim(xf, 0.0), GAMMA)       # [M][6][5][nf]
    vh_g = np.zeros((nfaces, 5, vh_loc.shape[-1]))
    vh_g[ids.reshape(-1)] = vh_loc.reshape(-1, 5, vh_loc.shape[-1])
    steps = int(round(T / (dt1 / N)))
    return dict(mesh=mesh, prm=prm, v=v, vh_g=vh_g, ids=ids, nfaces=nfaces, steps=steps, dt=T / steps,
                prim=prim, T=T)


def l2_error(kind, p, mesh, v):
    """L2 error of the density at the volume Gauss points at the final time."""
    prim, T = CASES[kind][0], CASES[kind][2]
    geo = local.Geometry(p, mesh.h)
    vg = np.einsum("ga,mka->mkg", geo.t["vol_phi"], v)
    rho_h = physics.conservative_from_entropy([vg[:, k] for k in range(5)], GAMMA)[0]
    # physical volume points: g = g1 + nq (g2 + nq g3), 1-D points on [0, 2] times h
    xq = basis.tables_1d(p)["xq"]
    nq = xq.size
    gidx = np.arange(nq ** 3)
    ref = np.stack([xq[gidx % nq], xq[(gidx // nq) % nq], xq[gidx // (nq * nq)]])
    xg = mesh.origin[:, :, None] + mesh.h[:, :, None] * ref[None]          # [M][3][G]
    rho_ex = prim(xg, T)[0]
    return float(np.sqrt(np.sum(geo.w_vol() * (rho_h - rho_ex) ** 2)))


def run(kind, p, N):
    """Returns (h, L2 error of rho at the final time, Newton iterations)."""
    c = setup(kind, p, N)
    v, vh_g = c["v"], c["vh_g"]
    its = []
    for _ in range(c["steps"]):
        v, vh_g, it = global_solve.dirk33_step(p, c["mesh"].h, c["ids"], c["nfaces"], v, vh_g, c["prm"], c["dt"])
        its += it
    return float(c["mesh"].h[0, 0]), l2_error(kind, p, c["mesh"], v), its


def study(kind, p, Ns):
    rows = []
    for N in Ns:
        t0 = time.perf_counter()
        h, e, its = run(kind, p, N)
        rate = np.nan if not rows else np.log(rows[-1][3] / e) / np.log(rows[-1][2] / h)
        rows.append((p, N, h, e, rate, max(its)))
        print(f"{kind} p={p} N={N} h={h:.5g} err={e:.6e} rate={rate:.3f} newton<= {max(its)} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    return rows


PLAN = {"wave": [(1, (2, 4, 8)), (2, (1, 2, 4))], "vortex": [(1, (2, 4, 8)), (2, (2, 4))]}


def main(which):
    kinds = list(PLAN) if which == "all" else [which]
    for kind in kinds:
        lines = ["# kind p N h L2_err_rho rate max_newton_iterations",
                 f"# written by tests/golden/make_convergence.py ({kind}); see its docstring"]
        for p, Ns in PLAN[kind]:
            for r in study(kind, p, Ns):
                lines.append(f"{kind} {r[0]} {r[1]} {r[2]:.17g} {r[3]:.17g} {r[4]:.6f} {r[5]}")
        with open(os.path.join(HERE, f"convergence_{kind}.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
