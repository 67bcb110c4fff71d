"""The macro-element residual, its Jacobian and static condensation on any
macro-element shape given as quadrature tables (oracle, FP64).

Oracle test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import this package.  Nothing on the GPU
path depends on it.

The weak form is that of Sec. 4.1 eq. s32a-c with the stage time term of
eq. C242 and the wall operator of the boundary condition, exactly as in
``local`` (which writes it for axis-aligned hexahedral macros with
tensor-product tables); here every geometric quantity comes from a
geometry object with

    M, n, nf, nfaces                sizes
    phi   [G][n]                    macro basis at the volume points
    dphi  [M][3][G][n]              physical gradients d/dx_j of the basis
    wv    [M][G]                    physical volume weights
    face_phi(f) [S][n]              macro basis at the points of face f
    face_psi(f) [S][nf]             trace basis at the points of face f
    ws(f) [M][S]                    physical face weights
    normal(f) [M][3]                outward unit normal (constant per face)

so that tetrahedral macro-elements (``tet.TetGeometry``) and hexahedral
ones (``HexGeometry`` below) share one statement of the residual.  The
orderings follow ``local``: V index k*n + a; Q index (k*3 + j)*n + a;
Vhat index (f*5 + k)*nf + c.
"""
from __future__ import annotations

import numpy as np

from . import ad
from . import basis
from . import local
from . import physics as ph


class HexGeometry:
    """The tables of ``basis`` for axis-aligned hexahedral macros h [M][3],
    in the interface above."""

    nfaces = 6

    def __init__(self, p, h):
        self.p = p
        t = basis.reference_tables(p)
        self.t = t
        h = np.asarray(h, dtype=np.float64)
        self.M = h.shape[0]
        volfac, invh, facefac = basis.physical(h)
        self.n, self.nf = t["n1d"] ** 3, t["n1d"] ** 2
        self.phi = t["vol_phi"]
        self.wv = volfac[:, None] * t["vol_w"][None, :]
        self.dphi = invh[:, :, None, None] * t["vol_dphi"][None]
        self._facefac = facefac

    def face_phi(self, f):
        return self.t["face_phi"][f]

    def face_psi(self, f):
        return self.t["face_psi"][f]

    def ws(self, f):
        return self._facefac[:, f, None] * self.t["face_w"][f][None, :]

    def normal(self, f):
        return np.broadcast_to(basis.face_normal(f), (self.M, 3))


def _comp(x, axis):
    return [np.take(x, i, axis=axis) for i in range(x.shape[axis])]


def _walls(face_bc, M_, nfaces):
    if face_bc is None:
        return np.zeros((M_, nfaces), dtype=bool)
    return np.asarray(face_bc).reshape(M_, nfaces) != 0


# --------------------------------------------------------------------------
# the constant blocks of R_Q (eq. s32a)
# --------------------------------------------------------------------------
def mass(geo):
    """M[m,a,b] = sum_g w phi_a phi_b."""
    return np.einsum("mg,ga,gb->mab", geo.wv, geo.phi, geo.phi)


def grad_coupling(geo):
    """C[m,j,a,b] = sum_g w d_j phi_a phi_b."""
    return np.einsum("mg,mjga,gb->mjab", geo.wv, geo.dphi, geo.phi)


def trace_coupling(geo):
    """Chat[m,j,a,(f,c)] = sum_{s in f} w n_j phi_a psi_c."""
    out = np.zeros((geo.M, 3, geo.n, geo.nfaces * geo.nf))
    for f in range(geo.nfaces):
        base = np.einsum("ms,sa,sc->mac", geo.ws(f), geo.face_phi(f), geo.face_psi(f))
        out[:, :, :, f * geo.nf:(f + 1) * geo.nf] = geo.normal(f)[:, :, None, None] * base[:, None]
    return out


def lift_q(geo, v, vhat):
    """The q that makes R_Q vanish (weak gradient of (v, vhat))."""
    Mm, C, Ch = mass(geo), grad_coupling(geo), trace_coupling(geo)
    vh = vhat.transpose(0, 2, 1, 3).reshape(geo.M, 5, -1)
    q = np.empty((geo.M, 5, 3, geo.n))
    for j in range(3):
        rhs = np.einsum("mab,mkb->mka", Ch[:, j], vh) - np.einsum("mab,mkb->mka", C[:, j], v)
        q[:, :, j, :] = np.linalg.solve(Mm[:, None], rhs[..., None])[..., 0]
    return q


def _q_lists(qg):
    return [[qg[:, l, j] for j in range(3)] for l in range(5)]


def _face_flux_m(vhs, vs, qs, nrm, prm):
    """Fhat + Ghat and Fhat at the points of one face of one macro: the
    physics routines take one normal, so macros are handled one by one."""
    Fh = ph.inviscid_trace_flux(vhs, vs, nrm, prm)
    if prm["viscous"]:
        Gh = ph.viscous_trace_flux(vhs, vs, qs, nrm, prm)
        return [Fh[k] + Gh[k] for k in range(5)], Fh
    return list(Fh), Fh


# --------------------------------------------------------------------------
# residual
# --------------------------------------------------------------------------
def residual(geo, v, vhat, v_old, prm, q=None, face_bc=None):
    """R_q [M][5][3][n], R_v [M][5][n], R_vhat [M][nfaces][5][nf],
    entropy [M] (face entropy production), q [M][5][3][n]."""
    gamma = prm["gamma"]
    M_, n, nf, NF = geo.M, geo.n, geo.nf, geo.nfaces
    if q is None:
        q = lift_q(geo, v, vhat)
    phi, wv = geo.phi, geo.wv
    vg = np.einsum("ga,mka->mkg", phi, v)
    qg = np.einsum("ga,mkja->mkjg", phi, q)
    vog = np.einsum("ga,mka->mkg", phi, v_old)

    # R_Q (eq. s32a): (q_kj, phi_a) + (v_k, d_j phi_a) - <vhat_k, phi_a n_j>
    Mm, C, Ch = mass(geo), grad_coupling(geo), trace_coupling(geo)
    vh = vhat.transpose(0, 2, 1, 3).reshape(M_, 5, -1)
    R_q = np.empty((M_, 5, 3, n))
    for j in range(3):
        R_q[:, :, j, :] = (np.einsum("mab,mkb->mka", Mm, q[:, :, j, :])
                           + np.einsum("mab,mkb->mka", C[:, j], v)
                           - np.einsum("mab,mkb->mka", Ch[:, j], vh))

    # R_V volume part (eq. s32b, time term of eq. C242)
    vl = _comp(vg, 1)
    u = ph.conservative_from_entropy(vl, gamma)
    u_old = ph.conservative_from_entropy(_comp(vog, 1), gamma)
    F = ph.inviscid_flux(vl, gamma)
    if prm["viscous"]:
        Gv = ph.viscous_flux(vl, _q_lists(qg), prm)
        Fv = [[F[j][k] + Gv[j][k] for k in range(5)] for j in range(3)]
    else:
        Fv = F
    R_v = np.zeros((M_, 5, n))
    for k in range(5):
        R_v[:, k] += prm["alpha_t"] * ((wv * (u[k] - u_old[k])) @ phi)
        for j in range(3):
            R_v[:, k] -= np.einsum("mg,mga->ma", wv * Fv[j][k], geo.dphi[:, j])

    # faces (eq. s32b-c)
    R_vh = np.zeros((M_, NF, 5, nf))
    ent = np.zeros(M_)
    wall = _walls(face_bc, M_, NF)
    for f in range(NF):
        fphi, fpsi, ws = geo.face_phi(f), geo.face_psi(f), geo.ws(f)
        vs = np.einsum("sa,mka->mks", fphi, v)
        qs = np.einsum("sa,mkja->mkjs", fphi, q)
        vhs = np.einsum("sc,mkc->mks", fpsi, vhat[:, f])
        for m in range(M_):
            nrm = geo.normal(f)[m]
            qm = [[qs[m, l, j] for j in range(3)] for l in range(5)]
            tot, Finv = _face_flux_m(_comp(vhs[m], 0), _comp(vs[m], 0), qm, nrm, prm)
            for k in range(5):
                R_v[m, k] += (ws[m] * tot[k]) @ fphi
                R_vh[m, f, k] = (ws[m] * tot[k]) @ fpsi
            if wall[m, f]:
                for k in range(1, 5):
                    Bk = vhs[m, k] + (gamma / prm["T_wall"] if k == 4 else 0.0)
                    R_vh[m, f, k] = (ws[m] * Bk) @ fpsi
            integrand = ph.entropy_production_integrand(_comp(vhs[m], 0), _comp(vs[m], 0), Finv, nrm, gamma)
            ent[m] += np.sum(ws[m] * integrand)
    return dict(R_q=R_q, R_v=R_v, R_vhat=R_vh, entropy=ent, q=q)


# --------------------------------------------------------------------------
# Jacobian blocks
# --------------------------------------------------------------------------
def _assemble(test, coef, trial):
    """sum_g test[(m,)g,a] coef[m,g,K,L] trial[g,b] -> [m][K][a][L][b]; test
    is shared ([G][a]) or per macro ([M][G][a])."""
    if test.ndim == 2:
        return np.einsum("ga,mgKL,gb->mKaLb", test, coef, trial, optimize=True)
    return np.einsum("mga,mgKL,gb->mKaLb", test, coef, trial, optimize=True)


def _dual_jac(comps, shape, nd):
    return np.stack([c.d if isinstance(c, ad.Dual) else np.zeros(shape + (nd,)) for c in comps], axis=-2)


def jacobian(geo, v, vhat, v_old, prm, q=None, face_bc=None):
    """All Jacobian blocks of ``residual`` at (q, v, vhat), dense per macro,
    with the pseudo-time term alpha_ps (A0(v) dv, w) in A_vv."""
    gamma = prm["gamma"]
    M_, n, nf, NF = geo.M, geo.n, geo.nf, geo.nfaces
    if q is None:
        q = lift_q(geo, v, vhat)
    phi, wv = geo.phi, geo.wv
    vg = np.einsum("ga,mka->mkg", phi, v)
    qg = np.einsum("ga,mkja->mkjg", phi, q)
    NV, NQ, NH = 5 * n, 15 * n, 5 * NF * nf
    visc = bool(prm["viscous"])
    pshape = vg.shape[:1] + vg.shape[2:]

    A_vv = np.zeros((M_, 5, n, 5, n))
    A_vq = np.zeros((M_, 5, n, 15, n))
    A_vvh = np.zeros((M_, 5, n, NF, 5, nf))
    A_hv = np.zeros((M_, NF, 5, nf, 5, n))
    A_hq = np.zeros((M_, NF, 5, nf, 15, n))
    A_hh = np.zeros((M_, NF, 5, nf, NF, 5, nf))

    # volume, derivatives in v
    vd = ad.seed(_comp(vg, 1), 5, 0)
    A0 = ad.jac(ph.conservative_from_entropy(vd, gamma))            # m,g,k,l
    A_vv += _assemble(phi, (prm["alpha_t"] + prm["alpha_ps"]) * wv[..., None, None] * A0, phi)
    F = ph.inviscid_flux(vd, gamma)
    if visc:
        qc = [[ad.const([qg[:, l, j]], 5)[0] for j in range(3)] for l in range(5)]
        Gv = ph.viscous_flux(vd, qc, prm)
    for j in range(3):
        comps = [F[j][k] + Gv[j][k] for k in range(5)] if visc else F[j]
        dF = _dual_jac(comps, pshape, 5)
        A_vv -= _assemble(geo.dphi[:, j], wv[..., None, None] * dF, phi)
    # volume, derivatives in q
    if visc:
        vc = ad.const(_comp(vg, 1), 15)
        qd_flat = ad.seed([qg[:, l, j] for l in range(5) for j in range(3)], 15, 0)
        qd = [[qd_flat[l * 3 + j] for j in range(3)] for l in range(5)]
        Gq = ph.viscous_flux(vc, qd, prm)
        for i in range(3):
            dG = _dual_jac(Gq[i], pshape, 15)
            A_vq -= _assemble(geo.dphi[:, i], wv[..., None, None] * dG, phi)

    # faces
    wall = _walls(face_bc, M_, NF)
    for f in range(NF):
        fphi, fpsi, ws = geo.face_phi(f), geo.face_psi(f), geo.ws(f)
        vs = np.einsum("sa,mka->mks", fphi, v)
        qs = np.einsum("sa,mkja->mkjs", fphi, q)
        vhs = np.einsum("sc,mkc->mks", fpsi, vhat[:, f])
        S = fphi.shape[0]
        Jh = np.zeros((M_, S, 5, 10))
        Jq = np.zeros((M_, S, 5, 15))
        for m in range(M_):
            nrm = geo.normal(f)[m]
            vhd = ad.seed(_comp(vhs[m], 0), 10, 0)
            vdd = ad.seed(_comp(vs[m], 0), 10, 5)
            qc = ([[ad.const([qs[m, l, j]], 10)[0] for j in range(3)] for l in range(5)] if visc else None)
            tot, _ = _face_flux_m(vhd, vdd, qc, nrm, prm)
            Jh[m] = ad.jac(tot)
            if visc:
                qd_flat = ad.seed([qs[m, l, j] for l in range(5) for j in range(3)], 15, 0)
                qd = [[qd_flat[l * 3 + j] for j in range(3)] for l in range(5)]
                Gh = ph.viscous_trace_flux(ad.const(_comp(vhs[m], 0), 15), ad.const(_comp(vs[m], 0), 15),
                                           qd, nrm, prm)
                Jq[m] = ad.jac(Gh)
        w4 = ws[..., None, None]
        dh, dv = w4 * Jh[..., 0:5], w4 * Jh[..., 5:10]
        A_vv += _assemble(fphi, dv, fphi)
        A_vvh[:, :, :, f] += _assemble(fphi, dh, fpsi)
        A_hv[:, f] += _assemble(fpsi, dv, fphi)
        A_hh[:, f, :, :, f] += _assemble(fpsi, dh, fpsi)
        if visc:
            dq = w4 * Jq
            A_vq += _assemble(fphi, dq, fphi)
            A_hq[:, f] += _assemble(fpsi, dq, fphi)
        if wall[:, f].any():
            w_ = wall[:, f]
            A_hv[w_, f, 1:] = 0.0
            A_hq[w_, f, 1:] = 0.0
            A_hh[w_, f, 1:] = 0.0
            Mf = np.einsum("ms,sc,sd->mcd", ws, fpsi, fpsi)
            for k in range(1, 5):
                A_hh[w_, f, k, :, f, k, :] = Mf[w_]

    # R_Q blocks
    Mm, C, Ch = mass(geo), grad_coupling(geo), trace_coupling(geo)
    A_qq = np.zeros((M_, 5, 3, n, 5, 3, n))
    A_qv = np.zeros((M_, 5, 3, n, 5, n))
    A_qvh = np.zeros((M_, 5, 3, n, NF, 5, nf))
    for k in range(5):
        for j in range(3):
            A_qq[:, k, j, :, k, j, :] = Mm
            A_qv[:, k, j, :, k, :] = C[:, j]
            A_qvh[:, k, j, :, :, k, :] = -Ch[:, j].reshape(M_, n, NF, nf)
    return dict(
        A_qq=A_qq.reshape(M_, NQ, NQ), A_qv=A_qv.reshape(M_, NQ, NV), A_qvh=A_qvh.reshape(M_, NQ, NH),
        A_vq=A_vq.reshape(M_, NV, NQ), A_vv=A_vv.reshape(M_, NV, NV), A_vvh=A_vvh.reshape(M_, NV, NH),
        A_hq=A_hq.reshape(M_, NH, NQ), A_hv=A_hv.reshape(M_, NH, NV), A_hh=A_hh.reshape(M_, NH, NH),
        mass=Mm, q=q)


def condense(geo, v, vhat, v_old, prm, q=None, face_bc=None):
    """Residual, Jacobian blocks and the condensed system (eq. R3, R5a-b) of
    each macro; ``local.recover`` applies to the result."""
    res = residual(geo, v, vhat, v_old, prm, q=q, face_bc=face_bc)
    J = jacobian(geo, v, vhat, v_old, prm, q=res["q"], face_bc=face_bc)
    return local.condense_blocks(res, J)
