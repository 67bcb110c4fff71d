"""Local work of one Newton step on a batch of macro-elements (oracle, FP64).

Oracle test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import this package.  It shares no code
with the HIP library; both receive the same seeded inputs.

What it computes, per macro-element K (Sec. 4.1 eq. s32a-c with the stage
time term of eq. C242, Sec. 6.1-6.2 eq. R1-R6):

* the residual R = [R_Q, R_V, R_Vhat] by quadrature,
    R_Q[k,j,a]  = (q_kj, phi_a) + (v_k, d_j phi_a) - <vhat_k, phi_a n_j>,
    R_V[k,a]    = alpha_t (u_k(v) - u_k(v_old), phi_a) - (F_kj + G_kj, d_j phi_a)
                  + <Fhat_k + Ghat_k, phi_a>,
    R_Vhat[f,k,c] = <Fhat_k + Ghat_k, psi_c>_f,
* the per-macro face entropy production sum_s w ([[v]]^T Fhat - [[Psi_n]]),
* the exact Jacobian blocks of that residual (pointwise dual numbers plus
  the linear chain rule through the quadrature), with the pseudo-time term
  alpha_ps (A0(v) dv, w) added to A_vv,
* static condensation: S (R3), Y, X, A', r_V, r_hat, then
  Ahat = A' + X S^-1 Y (R5a) and bhat = r_hat - X S^-1 r_V (R5b),
* recovery: dV = S^-1 (r_V + Y dVhat) (R2) and
  dQ = A_qq^-1 (-R_Q - A_qv dV - A_qvhat dVhat) (R6).

Orderings: V index k*n + a; Q index (k*3 + j)*n + a; Vhat index
(f*5 + k)*nf + c.
"""
from __future__ import annotations

import numpy as np

from . import ad
from . import basis
from . import physics as ph


class Geometry:
    """Reference tables scaled to the macros of a batch."""

    def __init__(self, p, h):
        self.p = p
        self.t = basis.reference_tables(p)
        self.h = np.asarray(h, dtype=np.float64)
        self.volfac, self.invh, self.facefac = basis.physical(self.h)
        self.n = self.t["n1d"] ** 3
        self.nf = self.t["n1d"] ** 2
        self.G = self.t["vol_w"].size
        self.S = self.t["face_w"].shape[1]

    def w_vol(self):                       # [M][G]
        return self.volfac[:, None] * self.t["vol_w"][None, :]

    def w_face(self, f):                   # [M][S]
        return self.facefac[:, f, None] * self.t["face_w"][f][None, :]

    # constant blocks of R_Q --------------------------------------------------
    def mass(self):
        """M[a,b] = sum_g w phi_a phi_b  -> [M][n][n]."""
        P = self.t["vol_phi"]
        base = P.T @ (self.t["vol_w"][:, None] * P)
        return self.volfac[:, None, None] * base[None]

    def grad_coupling(self):
        """C_j[a,b] = sum_g w d_j phi_a phi_b -> [M][3][n][n]."""
        P = self.t["vol_phi"]
        out = []
        for j in range(3):
            base = self.t["vol_dphi"][j].T @ (self.t["vol_w"][:, None] * P)
            out.append((self.volfac * self.invh[:, j])[:, None, None] * base[None])
        return np.stack(out, axis=1)

    def trace_coupling(self):
        """Chat_j[a, (f,c)] = sum_{s in f} w phi_a n_j psi_c -> [M][3][n][6*nf]."""
        M = self.h.shape[0]
        out = np.zeros((M, 3, self.n, 6 * self.nf))
        for f in range(6):
            n = basis.face_normal(f)
            base = self.t["face_phi"][f].T @ (self.t["face_w"][f][:, None] * self.t["face_psi"][f])
            for j in range(3):
                if n[j] != 0.0:
                    out[:, j, :, f * self.nf:(f + 1) * self.nf] = \
                        (self.facefac[:, f] * n[j])[:, None, None] * base[None]
        return out


def _walls(face_bc, M_):
    """[M][6] bool: the faces with the isothermal wall operator."""
    if face_bc is None:
        return np.zeros((M_, 6), dtype=bool)
    return np.asarray(face_bc).reshape(M_, 6) != 0


def _comp(x, axis):
    """Split an array into a list of components along ``axis``."""
    return [np.take(x, i, axis=axis) for i in range(x.shape[axis])]


def lift_q(geo, v, vhat):
    """q that makes R_Q vanish: q_kj = M^-1 (Chat_j vhat_k - C_j v_k)."""
    Mm = geo.mass()
    C = geo.grad_coupling()
    Ch = geo.trace_coupling()
    M_ = v.shape[0]
    vh = vhat.transpose(0, 2, 1, 3).reshape(M_, 5, -1)       # [M][k][(f,c)]
    q = np.empty((M_, 5, 3, geo.n))
    for j in range(3):
        rhs = np.einsum("mab,mkb->mka", Ch[:, j], vh) - np.einsum("mab,mkb->mka", C[:, j], v)
        q[:, :, j, :] = np.linalg.solve(Mm[:, None], rhs[..., None])[..., 0]
    return q


def _points(geo, v, q, vhat, v_old):
    t = geo.t
    vg = np.einsum("ga,mka->mkg", t["vol_phi"], v)
    qg = np.einsum("ga,mkja->mkjg", t["vol_phi"], q)
    vog = np.einsum("ga,mka->mkg", t["vol_phi"], v_old)
    faces = []
    for f in range(6):
        vs = np.einsum("sa,mka->mks", t["face_phi"][f], v)
        qs = np.einsum("sa,mkja->mkjs", t["face_phi"][f], q)
        vhs = np.einsum("sc,mkc->mks", t["face_psi"][f], vhat[:, f])
        faces.append((vs, qs, vhs))
    return vg, qg, vog, faces


def _q_lists(qg):
    return [[qg[:, l, j] for j in range(3)] for l in range(5)]


def _face_flux(vhs, vs, qs, n, prm):
    Fh = ph.inviscid_trace_flux(vhs, vs, n, prm)
    if prm["viscous"]:
        Gh = ph.viscous_trace_flux(vhs, vs, qs, n, prm)
        return [Fh[k] + Gh[k] for k in range(5)], Fh
    return list(Fh), Fh


def residual(p, h, v, vhat, v_old, prm, q=None, face_bc=None, old=None):
    """Residual blocks and face entropy production of a batch of macros.

    With ``old`` [M][5][n] given, the time term is alpha_t ((u(v), phi_a) - old)
    instead of alpha_t (u(v) - u(v_old), phi_a): the stage form of a DIRK
    step, whose old term is a combination of earlier stages (Sec. 5.3).

    ``face_bc`` [M][6] (nonzero: isothermal no-slip wall): on a wall face the
    trace equations use the boundary operator
        B = [(Fhat + Ghat)_1, vhat_2, vhat_3, vhat_4, vhat_5 + gamma / T_wall]
    (no mass flux, zero velocity since vhat_2..4 = beta V, and T = T_wall since
    vhat_5 = -gamma / T), tested against the trace basis like the flux; the
    element equations keep Fhat + Ghat.

    Returns dict R_q [M][5][3][n], R_v [M][5][n], R_vhat [M][6][5][nf],
    entropy [M], q [M][5][3][n] (the q used).
    """
    geo = Geometry(p, h)
    t = geo.t
    gamma = prm["gamma"]
    if q is None:
        q = lift_q(geo, v, vhat)
    vg, qg, vog, faces = _points(geo, v, q, vhat, v_old)
    wv = geo.w_vol()
    M_ = v.shape[0]

    # R_Q (eq. s32a)
    Mm = geo.mass()
    C = geo.grad_coupling()
    Ch = geo.trace_coupling()
    vh = vhat.transpose(0, 2, 1, 3).reshape(M_, 5, -1)
    R_q = np.empty((M_, 5, 3, geo.n))
    for j in range(3):
        # (q_kj, phi_a) + (v_k, d_j phi_a) - <vhat_k, phi_a n_j>
        R_q[:, :, j, :] = (np.einsum("mab,mkb->mka", Mm, q[:, :, j, :])
                           + np.einsum("mab,mkb->mka", C[:, j], v)
                           - np.einsum("mab,mkb->mka", Ch[:, j], vh))

    # R_V volume part (eq. s32b with the time term of C242)
    vl = _comp(vg, 1)
    u = ph.conservative_from_entropy(vl, gamma)
    u_old = ph.conservative_from_entropy(_comp(vog, 1), gamma)
    F = ph.inviscid_flux(vl, gamma)
    if prm["viscous"]:
        Gv = ph.viscous_flux(vl, _q_lists(qg), prm)
        Fv = [[F[j][k] + Gv[j][k] for k in range(5)] for j in range(3)]
    else:
        Fv = F
    R_v = np.zeros((M_, 5, geo.n))
    for k in range(5):
        if old is None:
            R_v[:, k] += prm["alpha_t"] * ((wv * (u[k] - u_old[k])) @ t["vol_phi"])
        else:
            R_v[:, k] += prm["alpha_t"] * ((wv * u[k]) @ t["vol_phi"] - old[:, k])
        for j in range(3):
            R_v[:, k] -= ((wv * geo.invh[:, j, None]) * Fv[j][k]) @ t["vol_dphi"][j]

    # face terms
    R_vh = np.zeros((M_, 6, 5, geo.nf))
    ent = np.zeros(M_)
    for f in range(6):
        vs, qs, vhs = faces[f]
        n = basis.face_normal(f)
        ws = geo.w_face(f)
        tot, Finv = _face_flux(_comp(vhs, 1), _comp(vs, 1), _q_lists(qs), n, prm)
        for k in range(5):
            R_v[:, k] += (ws * tot[k]) @ t["face_phi"][f]
            R_vh[:, f, k] = (ws * tot[k]) @ t["face_psi"][f]
        wall = _walls(face_bc, M_)[:, f]
        if wall.any():
            for k in range(1, 5):
                Bk = vhs[:, k] + (gamma / prm["T_wall"] if k == 4 else 0.0)
                R_vh[wall, f, k] = ((ws * Bk) @ t["face_psi"][f])[wall]
        integrand = ph.entropy_production_integrand(_comp(vhs, 1), _comp(vs, 1), Finv, n, gamma)
        ent += np.sum(ws * integrand, axis=1)
    return dict(R_q=R_q, R_v=R_v, R_vhat=R_vh, entropy=ent, q=q)


def time_functional(p, h, v, prm):
    """(u(v), phi_a) per macro -> [M][5][n] (the mass term of the time derivative)."""
    geo = Geometry(p, h)
    vg = np.einsum("ga,mka->mkg", geo.t["vol_phi"], v)
    u = ph.conservative_from_entropy(_comp(vg, 1), prm["gamma"])
    wv = geo.w_vol()
    return np.stack([(wv * u[k]) @ geo.t["vol_phi"] for k in range(5)], axis=1)


# --------------------------------------------------------------------------
# Jacobian blocks
# --------------------------------------------------------------------------
def _assemble(test, coef, trial):
    """sum_g test[g,a] coef[m,g,K,L] trial[g,b] -> [m][K][a][L][b]."""
    M_, G, K, L = coef.shape
    nb = trial.shape[1]
    T = coef[..., None] * trial[None, :, None, None, :]        # m,g,K,L,b
    out = np.matmul(test.T[None], T.reshape(M_, G, K * L * nb))   # m,a,(K L b)
    return out.reshape(M_, test.shape[1], K, L, nb).transpose(0, 2, 1, 3, 4)


def jacobian(p, h, v, vhat, v_old, prm, q=None, face_bc=None):
    """All Jacobian blocks of the residual at (q, v, vhat), dense per macro
    (``face_bc``: see residual)."""
    geo = Geometry(p, h)
    t = geo.t
    gamma = prm["gamma"]
    if q is None:
        q = lift_q(geo, v, vhat)
    vg, qg, vog, faces = _points(geo, v, q, vhat, v_old)
    M_, n, nf = v.shape[0], geo.n, geo.nf
    NV, NQ, NH = 5 * n, 15 * n, 30 * nf
    wv = geo.w_vol()
    visc = bool(prm["viscous"])

    A_vv = np.zeros((M_, 5, n, 5, n))
    A_vq = np.zeros((M_, 5, n, 15, n))
    A_vvh = np.zeros((M_, 5, n, 6, 5, nf))
    A_hv = np.zeros((M_, 6, 5, nf, 5, n))
    A_hq = np.zeros((M_, 6, 5, nf, 15, n))
    A_hh = np.zeros((M_, 6, 5, nf, 6, 5, nf))

    # volume: derivatives in v (5 directions) ...........................
    vd = ad.seed(_comp(vg, 1), 5, 0)
    u = ph.conservative_from_entropy(vd, gamma)
    A0 = ad.jac(u)                                           # m,g,k,l
    A_vv += _assemble(t["vol_phi"], (prm["alpha_t"] + prm["alpha_ps"]) * wv[..., None, None] * A0,
                      t["vol_phi"])
    F = ph.inviscid_flux(vd, gamma)
    if visc:
        qc = [[ad.const([qg[:, l, j]], 5)[0] for j in range(3)] for l in range(5)]
        Gv = ph.viscous_flux(vd, qc, prm)
    for j in range(3):
        comps = [F[j][k] + Gv[j][k] for k in range(5)] if visc else F[j]
        dF = np.stack([c.d if isinstance(c, ad.Dual) else np.zeros(vg.shape[:1] + vg.shape[2:] + (5,))
                       for c in comps], axis=-2)
        A_vv -= _assemble(t["vol_dphi"][j], (wv * geo.invh[:, j, None])[..., None, None] * dF,
                          t["vol_phi"])
    # volume: derivatives in q (15 directions) ...........................
    if visc:
        vc = ad.const(_comp(vg, 1), 15)
        qd_flat = ad.seed([qg[:, l, j] for l in range(5) for j in range(3)], 15, 0)
        qd = [[qd_flat[l * 3 + j] for j in range(3)] for l in range(5)]
        Gq = ph.viscous_flux(vc, qd, prm)
        for i in range(3):
            dG = np.stack([c.d if isinstance(c, ad.Dual) else np.zeros(vg.shape[:1] + vg.shape[2:] + (15,))
                           for c in Gq[i]], axis=-2)      # m,g,k,(l,j)
            A_vq -= _assemble(t["vol_dphi"][i], (wv * geo.invh[:, i, None])[..., None, None] * dG,
                              t["vol_phi"])

    # faces ...............................................................
    for f in range(6):
        vs, qs, vhs = faces[f]
        nrm = basis.face_normal(f)
        ws = geo.w_face(f)[..., None, None]
        phi, psi = t["face_phi"][f], t["face_psi"][f]
        # seeds: vhat in 0..4, v in 5..9
        vhd = ad.seed(_comp(vhs, 1), 10, 0)
        vdd = ad.seed(_comp(vs, 1), 10, 5)
        if visc:
            qc = [[ad.const([qs[:, l, j]], 10)[0] for j in range(3)] for l in range(5)]
        else:
            qc = None
        tot, _ = _face_flux(vhd, vdd, qc, nrm, prm)
        J = ad.jac(tot)                                       # m,s,k,10
        dh, dv = ws * J[..., 0:5], ws * J[..., 5:10]
        A_vv += _assemble(phi, dv, phi)
        A_vvh[:, :, :, f] += _assemble(phi, dh, psi)
        A_hv[:, f] += _assemble(psi, dv, phi)
        A_hh[:, f, :, :, f] += _assemble(psi, dh, psi)
        if visc:
            vhc = ad.const(_comp(vhs, 1), 15)
            vc = ad.const(_comp(vs, 1), 15)
            qd_flat = ad.seed([qs[:, l, j] for l in range(5) for j in range(3)], 15, 0)
            qd = [[qd_flat[l * 3 + j] for j in range(3)] for l in range(5)]
            Gh = ph.viscous_trace_flux(vhc, vc, qd, nrm, prm)
            dq = ws * ad.jac(Gh)                              # m,s,k,15
            A_vq += _assemble(phi, dq, phi)
            A_hq[:, f] += _assemble(psi, dq, phi)
        # wall faces: rows 2..5 of the trace equations are vhat_k (+ const)
        wall = _walls(face_bc, M_)[:, f]
        if wall.any():
            A_hv[wall, f, 1:] = 0.0
            A_hq[wall, f, 1:] = 0.0
            A_hh[wall, f, 1:] = 0.0
            Mf = np.einsum("ms,sc,sd->mcd", geo.w_face(f), psi, psi)
            for k in range(1, 5):
                A_hh[wall, f, k, :, f, k, :] = Mf[wall]

    # constant blocks of R_Q (eq. s32a) ...................................
    Mm = geo.mass()
    C = geo.grad_coupling()
    Ch = geo.trace_coupling()
    A_qq = np.zeros((M_, 5, 3, n, 5, 3, n))
    A_qv = np.zeros((M_, 5, 3, n, 5, n))
    A_qvh = np.zeros((M_, 5, 3, n, 6, 5, nf))
    for k in range(5):
        for j in range(3):
            A_qq[:, k, j, :, k, j, :] = Mm
            A_qv[:, k, j, :, k, :] = C[:, j]
            A_qvh[:, k, j, :, :, k, :] = -Ch[:, j].reshape(M_, n, 6, nf)

    return dict(
        A_qq=A_qq.reshape(M_, NQ, NQ), A_qv=A_qv.reshape(M_, NQ, NV),
        A_qvh=A_qvh.reshape(M_, NQ, NH),
        A_vq=A_vq.reshape(M_, NV, NQ), A_vv=A_vv.reshape(M_, NV, NV),
        A_vvh=A_vvh.reshape(M_, NV, NH),
        A_hq=A_hq.reshape(M_, NH, NQ), A_hv=A_hv.reshape(M_, NH, NV),
        A_hh=A_hh.reshape(M_, NH, NH), mass=Mm, q=q)


# --------------------------------------------------------------------------
# static condensation and recovery (Sec. 6.2)
# --------------------------------------------------------------------------
def _apply_Aqq_inv(Mm, X):
    """(I_15 (x) M)^-1 X for X with rows in Q ordering: [NQ] or [NQ][c]."""
    n = Mm.shape[0]
    vec = X.ndim == 1
    Y = X.reshape(15, n, -1)
    out = np.linalg.solve(Mm[None], Y)
    return out.reshape(X.shape) if not vec else out.reshape(-1)


def condense(p, h, v, vhat, v_old, prm, q=None, want_cond=False, old=None, face_bc=None):
    """Residual, blocks and condensed system of each macro.

    Returns dict with R_q, R_v, R_vhat, entropy, Ahat [M][NH][NH],
    bhat [M][NH], and the pieces needed for recovery.  ``old``, ``face_bc``:
    see residual.
    """
    res = residual(p, h, v, vhat, v_old, prm, q=q, old=old, face_bc=face_bc)
    J = jacobian(p, h, v, vhat, v_old, prm, q=res["q"], face_bc=face_bc)
    return condense_blocks(res, J, want_cond=want_cond)


def condense_blocks(res, J, want_cond=False):
    """The condensed system of each macro from its residual ``res`` and its
    Jacobian blocks ``J`` (any macro shape: the algebra of eq. R3, R5a-b
    only needs A_qq = I_15 (x) mass)."""
    M_ = res["R_v"].shape[0]
    out = dict(res)
    keys = ["S", "X", "Y", "Ap", "r_v", "r_hat", "Ahat", "bhat"]
    for kname in keys:
        out[kname] = []
    if want_cond:
        out["cond_S"] = []
    for m in range(M_):
        Mm = J["mass"][m]
        R_q = res["R_q"][m].reshape(-1)
        R_v = res["R_v"][m].reshape(-1)
        R_h = res["R_vhat"][m].reshape(-1)
        Aqv_s = _apply_Aqq_inv(Mm, J["A_qv"][m])
        Aqh_s = _apply_Aqq_inv(Mm, J["A_qvh"][m])
        Rq_s = _apply_Aqq_inv(Mm, R_q)
        S = J["A_vv"][m] - J["A_vq"][m] @ Aqv_s                  # eq. R3
        Y = -J["A_vvh"][m] + J["A_vq"][m] @ Aqh_s
        X = J["A_hv"][m] - J["A_hq"][m] @ Aqv_s
        Ap = J["A_hh"][m] - J["A_hq"][m] @ Aqh_s
        r_v = -R_v + J["A_vq"][m] @ Rq_s
        r_h = -R_h + J["A_hq"][m] @ Rq_s
        Ahat = Ap + X @ np.linalg.solve(S, Y)                    # eq. R5a
        bhat = r_h - X @ np.linalg.solve(S, r_v)                 # eq. R5b
        for kname, val in zip(keys, [S, X, Y, Ap, r_v, r_h, Ahat, bhat]):
            out[kname].append(val)
        if want_cond:
            out["cond_S"].append(np.linalg.cond(S))
    for kname in keys + (["cond_S"] if want_cond else []):
        out[kname] = np.stack(out[kname])
    out["J"] = J
    return out


def recover(cond, dvhat):
    """Interior update of each macro from its trace update (eq. R2, R6).

    dvhat [M][6][5][nf] -> dv [M][5][n], dq [M][5][3][n].
    """
    J = cond["J"]
    M_ = dvhat.shape[0]
    n = J["mass"].shape[1]
    dv = np.empty((M_, 5, n))
    dq = np.empty((M_, 5, 3, n))
    for m in range(M_):
        dh = dvhat[m].reshape(-1)
        dV = np.linalg.solve(cond["S"][m], cond["r_v"][m] + cond["Y"][m] @ dh)
        rhs = -cond["R_q"][m].reshape(-1) - J["A_qv"][m] @ dV - J["A_qvh"][m] @ dh
        dQ = _apply_Aqq_inv(J["mass"][m], rhs)
        dv[m] = dV.reshape(5, n)
        dq[m] = dQ.reshape(5, 3, n)
    return dv, dq
