"""Jacobian-vector and vector-Jacobian products of the macro-element
residual (oracle, FP64).

Oracle test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import this package.  Nothing on the GPU
path depends on it.

The residual R = [R_Q, R_V, R_Vhat] of Sec. 4.1 (eq. s32a-c with the stage
time term of eq. C242) is a function of (q, v, vhat).  Its exact Jacobian
is the block matrix of Sec. 6.2 (eq. R1), taken here from local.jacobian:

    J = [[A_qq, A_qv, A_qvh],
         [A_vq, A_vv, A_vvh],
         [A_hq, A_hv, A_hh ]]      (A_vv includes the pseudo-time term).

Two forms of each product:

* full: J x for x = (dq, dv, dvhat), and J^T w for w = (w_q, w_v, w_vhat);
* reduced: q is the weak gradient of (v, vhat), the solution of R_Q = 0
  (eq. s32a).  R_Q is linear, so q = L_v v + L_h vhat with
  L_v = -A_qq^-1 A_qv, L_h = -A_qq^-1 A_qvh, and the residual of (v, vhat)
  alone has the Jacobian
      J_r = [[A_vv + A_vq L_v, A_vvh + A_vq L_h],
             [A_hv + A_hq L_v, A_hh + A_hq L_h]],
  the operator a Jacobian-free Newton-Krylov method on the (v, vhat)
  unknowns of Algorithm 1 multiplies by.

``face_bc`` (wall faces) is passed to local.jacobian.
"""
from __future__ import annotations

import numpy as np

from . import local


def _blocks(p, h, v, vhat, v_old, prm, q=None, face_bc=None):
    return local.jacobian(p, h, v, vhat, v_old, prm, q=q, face_bc=face_bc)


def reduced_jacobian(J):
    """Per-macro J_r [M][N_V + N_VH][N_V + N_VH] from the full blocks."""
    M_ = J["A_vv"].shape[0]
    out = []
    for m in range(M_):
        Aqq = np.kron(np.eye(15), J["mass"][m])
        Lv = -np.linalg.solve(Aqq, J["A_qv"][m])
        Lh = -np.linalg.solve(Aqq, J["A_qvh"][m])
        out.append(np.block([[J["A_vv"][m] + J["A_vq"][m] @ Lv, J["A_vvh"][m] + J["A_vq"][m] @ Lh],
                             [J["A_hv"][m] + J["A_hq"][m] @ Lv, J["A_hh"][m] + J["A_hq"][m] @ Lh]]))
    return np.stack(out)


def jvp(p, h, v, vhat, v_old, prm, dv, dvhat, dq=None, q=None, face_bc=None):
    """J x at the state (q, v, vhat); q None means the weak gradient.

    With dq given: the full product, returns (JR_q, JR_v, JR_vhat) shaped like
    (q, v, vhat).  With dq None: dq is the weak gradient of (dv, dvhat), so
    JR_q vanishes; returns (zeros, JR_v, JR_vhat) from J_r."""
    J = _blocks(p, h, v, vhat, v_old, prm, q=q, face_bc=face_bc)
    M_ = v.shape[0]
    NV, NH = J["A_vv"].shape[1], J["A_hh"].shape[1]
    if dq is None:
        Jr = reduced_jacobian(J)
        x = np.concatenate([dv.reshape(M_, NV), dvhat.reshape(M_, NH)], axis=1)
        y = np.einsum("mij,mj->mi", Jr, x)
        return (np.zeros((M_, 5, 3, NV // 5)), y[:, :NV].reshape(dv.shape), y[:, NV:].reshape(dvhat.shape))
    x = np.concatenate([dq.reshape(M_, -1), dv.reshape(M_, NV), dvhat.reshape(M_, NH)], axis=1)
    out = []
    for m in range(M_):
        Jf = np.block([[J["A_qq"][m], J["A_qv"][m], J["A_qvh"][m]],
                       [J["A_vq"][m], J["A_vv"][m], J["A_vvh"][m]],
                       [J["A_hq"][m], J["A_hv"][m], J["A_hh"][m]]])
        out.append(Jf @ x[m])
    y = np.stack(out)
    NQ = 3 * NV
    return (y[:, :NQ].reshape(dq.shape), y[:, NQ:NQ + NV].reshape(dv.shape), y[:, NQ + NV:].reshape(dvhat.shape))


def vjp(p, h, v, vhat, v_old, prm, w_v, w_vhat, w_q=None, q=None, full=False, face_bc=None):
    """J^T w at the state (q, v, vhat); q None means the weak gradient.

    full: gradient of w_q.R_Q + w_v.R_V + w_vhat.R_Vhat in (q, v, vhat),
    returns (g_q, g_v, g_vhat).  Reduced (full False, w_q None): gradient of
    w_v.R_V + w_vhat.R_Vhat in (v, vhat) through the weak gradient, returns
    (g_v, g_vhat) from J_r^T."""
    J = _blocks(p, h, v, vhat, v_old, prm, q=q, face_bc=face_bc)
    M_ = v.shape[0]
    NV, NH = J["A_vv"].shape[1], J["A_hh"].shape[1]
    if not full:
        if w_q is not None:
            raise ValueError("the reduced product takes no w_q")
        Jr = reduced_jacobian(J)
        wv = np.concatenate([w_v.reshape(M_, NV), w_vhat.reshape(M_, NH)], axis=1)
        g = np.einsum("mji,mj->mi", Jr, wv)
        return g[:, :NV].reshape(w_v.shape), g[:, NV:].reshape(w_vhat.shape)
    wv = np.concatenate([w_q.reshape(M_, -1), w_v.reshape(M_, NV), w_vhat.reshape(M_, NH)], axis=1)
    out = []
    for m in range(M_):
        Jf = np.block([[J["A_qq"][m], J["A_qv"][m], J["A_qvh"][m]],
                       [J["A_vq"][m], J["A_vv"][m], J["A_vvh"][m]],
                       [J["A_hq"][m], J["A_hv"][m], J["A_hh"][m]]])
        out.append(Jf.T @ wv[m])
    g = np.stack(out)
    NQ = 3 * NV
    return g[:, :NQ].reshape(w_q.shape), g[:, NQ:NQ + NV].reshape(w_v.shape), g[:, NQ + NV:].reshape(w_vhat.shape)
