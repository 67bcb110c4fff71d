"""Global trace solve and DIRK(3,3) time stepping on periodic box meshes of
macro-elements (oracle, FP64).

Oracle test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import this package.  Used by the
convergence pins; nothing on the GPU path depends on it.

* Trace unknowns are single-valued per global face (Sec. 3.1 trace space M);
  every macro gathers its six faces.  Axis-aligned boxes of one orientation
  order the nodes of a shared face the same way from both sides.
* One Newton step (Sec. 6.2, Algorithm 1): every macro condenses its local
  system to Ahat dvhat = bhat (eq. R5); the global trace system is the sum
  of the local ones over the faces, K dVhat = F with K = sum_m P_m^T Ahat_m P_m
  and F = sum_m P_m^T bhat_m -- the linearisation of sum_m R_Vhat,m = 0, the
  conservation condition on every face; then every macro recovers dv, dq
  (eq. R2, R6).  K is sparse (a face couples with the faces of its two
  macros) and is solved directly.  q stays the weak gradient of (v, vhat).
* Time: Alexander's L-stable three-stage DIRK(3,3), stiffly accurate
  (Sec. 5.3 uses DIRK(3,3)).  Stage i solves
      alpha_i ((u(V_i), phi) - old_i) + R_sp(V_i) = 0,
      alpha_i = 1 / (a_ii dt),  old_i = (u(v^n), phi) + dt sum_{j<i} a_ij f_j,
  with f_j = -R_sp(V_j) = alpha_j ((u(V_j), phi) - old_j) from the
  converged stage j; v^{n+1} = V_3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import local


def dirk33_tableau():
    """Butcher matrix of Alexander's DIRK(3,3): a_ii = g, the root in (1/6, 1/2)
    of g^3 - 3 g^2 + 3 g / 2 - 1/6 (so that the method has order 3 and is
    L-stable), a21 = (1 - g)/2, a31 = -(6g^2 - 16g + 1)/4, a32 = (6g^2 - 20g + 5)/4."""
    roots = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
    g = float([r.real for r in roots if abs(r.imag) < 1e-12 and 1 / 6 < r.real < 0.5][0])
    A = np.zeros((3, 3))
    A[0, 0] = g
    A[1, 0], A[1, 1] = (1.0 - g) / 2.0, g
    A[2, 0] = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0
    A[2, 1] = (6.0 * g * g - 20.0 * g + 5.0) / 4.0
    A[2, 2] = g
    return A


def periodic_face_ids(shape, ijk):
    """Global face of each (macro, local face) on a periodic N1 x N2 x N3 box
    of macros: the face of axis d on side s of macro (i, j, k) is interface
    (idx_d + s) mod N_d of axis d.  Returns ids [M][6], number of faces."""
    N = np.asarray(shape, dtype=np.int64)
    ijk = np.asarray(ijk, dtype=np.int64)
    total = int(N.prod())
    ids = np.empty((ijk.shape[0], 6), dtype=np.int64)
    for f in range(6):
        d, s = f // 2, f % 2
        idx = ijk.copy()
        idx[:, d] = (idx[:, d] + s) % N[d]
        ids[:, f] = d * total + idx[:, 0] + N[0] * (idx[:, 1] + N[1] * idx[:, 2])
    return ids, 3 * total


def _dof_map(face_ids, nf):
    """Global trace dof of every local trace dof (f*5 + k)*nf + c -> [M][6*5*nf]."""
    M = face_ids.shape[0]
    loc = np.arange(5 * nf)
    return (face_ids[:, :, None] * (5 * nf) + loc[None, None, :]).reshape(M, 6 * 5 * nf)


def trace_system(cond, face_ids, nfaces, nf):
    """Global K (sparse, CSC) and F of the condensed local systems in ``cond``
    (local.condense output): K = sum_m P_m^T Ahat_m P_m, F = sum_m P_m^T bhat_m."""
    dmap = _dof_map(face_ids, nf)
    ndof = nfaces * 5 * nf
    rows = np.repeat(dmap[:, :, None], dmap.shape[1], axis=2).reshape(-1)
    cols = np.repeat(dmap[:, None, :], dmap.shape[1], axis=1).reshape(-1)
    K = sp.csc_matrix((cond["Ahat"].reshape(-1), (rows, cols)), shape=(ndof, ndof))
    F = np.zeros(ndof)
    np.add.at(F, dmap.reshape(-1), cond["bhat"].reshape(-1))
    return K, F


def gather(vh_g, face_ids):
    """Per-macro trace [M][6][5][nf] from the global one [faces][5][nf]."""
    return vh_g[face_ids]


def newton_stage(p, h, face_ids, nfaces, v, vh_g, old, prm, tol=1e-11, maxit=15):
    """Newton iterations for one implicit stage; returns v, vh_g, iterations,
    final max-norm of the residual (interior and assembled trace)."""
    nf = (2 * p + 1) ** 2
    dmap = _dof_map(face_ids, nf)
    ndof = nfaces * 5 * nf
    v = v.copy()
    vh_g = vh_g.copy()
    res = np.inf
    for it in range(maxit + 1):
        vhat = gather(vh_g, face_ids)
        c = local.condense(p, h, v, vhat, v, prm, old=old)
        Rg = np.zeros(ndof)
        np.add.at(Rg, dmap.reshape(-1), c["R_vhat"].reshape(-1))
        res = max(np.abs(c["R_v"]).max(), np.abs(Rg).max())
        if res < tol or it == maxit:
            return v, vh_g, it, res
        M = v.shape[0]
        K, F = trace_system(c, face_ids, nfaces, nf)
        dV = spla.spsolve(K, F)
        dv, _ = local.recover(c, dV[dmap].reshape(M, 6, 5, nf))
        v += dv
        vh_g += dV.reshape(nfaces, 5, nf)
    return v, vh_g, maxit, res


def dirk33_step(p, h, face_ids, nfaces, v, vh_g, prm, dt, tol=1e-11):
    """One DIRK(3,3) step of size dt; returns v^{n+1}, vh_g and the Newton
    iteration counts of the three stages."""
    A = dirk33_tableau()
    T0 = local.time_functional(p, h, v, prm)
    f = []
    V, VH = v, vh_g
    its = []
    for i in range(3):
        alpha = 1.0 / (A[i, i] * dt)
        old = T0 + dt * sum(A[i, j] * f[j] for j in range(i))
        prm_i = dict(prm, alpha_t=alpha, alpha_ps=0.0)
        V, VH, it, _ = newton_stage(p, h, face_ids, nfaces, V, VH, old, prm_i, tol=tol)
        its.append(it)
        f.append(alpha * (local.time_functional(p, h, V, prm) - old))
    return V, VH, its
