"""Pins of the oracle's Jacobian-vector and vector-Jacobian products
(oracle.linearized) against the residual itself.

* reduced JVP (q the weak gradient of (v, vhat), eq. s32a) against a central
  difference of the residual evaluated with q = weak gradient;
* full and reduced VJP through the directional identity
  <J^T w, x> = d/dt w.R(state + t x), the derivative by central differences
  of the residual -- independent of how the blocks are transposed;
* reduced VJP against the brute-force gradient of w.R, one central
  difference per input component, on one p = 1 macro;
* the R_Q part of the reduced JVP is zero and the full JVP with
  dq = weak gradient of (dv, dvhat) equals the reduced one.
The pseudo-time term is set to zero (it is Jacobian-only, not a derivative
of the residual).
"""
import numpy as np
import pytest

from oracle import linearized as lin
from oracle import local
from paper_2507_22195_amd import workloads as W

FD_H = 1e-6


def _cases():
    w1 = W.subset(W.workload(1), [0, 5])                                   # Euler, EC, p=2
    w2 = W.subset(W.workload(2, shape=(4, 4, 4)), [0, 21])                 # NS, ES, p=2
    w3 = W.subset(W.tgv_workload(shape=(3, 3, 3), p=1, M0=0.3, Re=500.0, flux="KEPES", seed_v=5, seed_vh=6,
                                 amp=3e-2), [0, 13])                      # NS, KEPES, p=1
    return [w1, w2, w3]


def _prm(w):
    return dict(w.params, alpha_ps=0.0)


def _R(w, prm, v, vh, q=None):
    r = local.residual(w.p, w.mesh.h, v, vh, w.v_old, prm, q=q)
    return r["R_q"], r["R_v"], r["R_vhat"]


@pytest.mark.parametrize("case", [0, 1, 2])
def test_reduced_jvp_matches_fd(case):
    w = _cases()[case]
    prm = _prm(w)
    rng = np.random.default_rng(1)
    dv = rng.standard_normal(w.v.shape)
    dh = rng.standard_normal(w.vhat.shape)
    Jq, Jv, Jh = lin.jvp(w.p, w.mesh.h, w.v, w.vhat, w.v_old, prm, dv, dh)
    _, pv, ph = _R(w, prm, w.v + FD_H * dv, w.vhat + FD_H * dh)
    _, mv, mh = _R(w, prm, w.v - FD_H * dv, w.vhat - FD_H * dh)
    for got, fd in ((Jv, (pv - mv) / (2 * FD_H)), (Jh, (ph - mh) / (2 * FD_H))):
        for m in range(w.n_macro):
            assert np.linalg.norm(got[m] - fd[m]) < 1e-7 * np.linalg.norm(fd[m])
    assert not Jq.any()


@pytest.mark.parametrize("case", [0, 1, 2])
def test_full_jvp_with_lifted_dq_equals_reduced(case):
    w = _cases()[case]
    prm = _prm(w)
    rng = np.random.default_rng(2)
    dv = rng.standard_normal(w.v.shape)
    dh = rng.standard_normal(w.vhat.shape)
    geo = local.Geometry(w.p, w.mesh.h)
    q = local.lift_q(geo, w.v, w.vhat)
    dq = local.lift_q(geo, dv, dh)
    Jq, Jv, Jh = lin.jvp(w.p, w.mesh.h, w.v, w.vhat, w.v_old, prm, dv, dh, dq=dq, q=q)
    _, Rv, Rh = lin.jvp(w.p, w.mesh.h, w.v, w.vhat, w.v_old, prm, dv, dh)
    assert np.linalg.norm(Jq) < 1e-12 * np.linalg.norm(Jv)
    assert np.linalg.norm(Jv - Rv) < 1e-12 * np.linalg.norm(Rv)
    assert np.linalg.norm(Jh - Rh) < 1e-12 * np.linalg.norm(Rh)


@pytest.mark.parametrize("case", [0, 1, 2])
def test_vjp_directional_identity(case):
    """<J^T w, x> = d/dt w.R(state + t x) for the full and the reduced product."""
    w = _cases()[case]
    prm = _prm(w)
    rng = np.random.default_rng(3)
    geo = local.Geometry(w.p, w.mesh.h)
    q = local.lift_q(geo, w.v, w.vhat) + 1e-3 * rng.standard_normal((w.n_macro, 5, 3, geo.n))
    wq = rng.standard_normal(q.shape)
    wv = rng.standard_normal(w.v.shape)
    wh = rng.standard_normal(w.vhat.shape)
    gq, gv, gh = lin.vjp(w.p, w.mesh.h, w.v, w.vhat, w.v_old, prm, wv, wh, w_q=wq, q=q, full=True)
    rv, rh = lin.vjp(w.p, w.mesh.h, w.v, w.vhat, w.v_old, prm, wv, wh)
    for _ in range(2):
        xq = rng.standard_normal(q.shape)
        xv = rng.standard_normal(w.v.shape)
        xh = rng.standard_normal(w.vhat.shape)

        def phi_full(t):
            Rq, Rv, Rh = _R(w, prm, w.v + t * xv, w.vhat + t * xh, q=q + t * xq)
            return np.array([np.sum(wq[m] * Rq[m]) + np.sum(wv[m] * Rv[m]) + np.sum(wh[m] * Rh[m])
                             for m in range(w.n_macro)])

        def phi_red(t):
            _, Rv, Rh = _R(w, prm, w.v + t * xv, w.vhat + t * xh)
            return np.array([np.sum(wv[m] * Rv[m]) + np.sum(wh[m] * Rh[m]) for m in range(w.n_macro)])

        fd_f = (phi_full(FD_H) - phi_full(-FD_H)) / (2 * FD_H)
        fd_r = (phi_red(FD_H) - phi_red(-FD_H)) / (2 * FD_H)
        for m in range(w.n_macro):
            a_f = np.sum(gq[m] * xq[m]) + np.sum(gv[m] * xv[m]) + np.sum(gh[m] * xh[m])
            a_r = np.sum(rv[m] * xv[m]) + np.sum(rh[m] * xh[m])
            scale_f = np.linalg.norm(np.concatenate([gq[m].ravel(), gv[m].ravel(), gh[m].ravel()])) * \
                np.linalg.norm(np.concatenate([xq[m].ravel(), xv[m].ravel(), xh[m].ravel()]))
            scale_r = np.linalg.norm(np.concatenate([rv[m].ravel(), rh[m].ravel()])) * \
                np.linalg.norm(np.concatenate([xv[m].ravel(), xh[m].ravel()]))
            assert abs(a_f - fd_f[m]) < 1e-7 * scale_f, (a_f, fd_f[m])
            assert abs(a_r - fd_r[m]) < 1e-7 * scale_r, (a_r, fd_r[m])


def test_reduced_vjp_brute_force_gradient():
    """Every component of the reduced VJP against its own central difference
    (one p = 1 viscous KEPES macro: 135 + 270 inputs)."""
    w = W.subset(_cases()[2], [1])
    prm = _prm(w)
    rng = np.random.default_rng(4)
    wv = rng.standard_normal(w.v.shape)
    wh = rng.standard_normal(w.vhat.shape)
    gv, gh = lin.vjp(w.p, w.mesh.h, w.v, w.vhat, w.v_old, prm, wv, wh)

    def phi(v, vh):
        _, Rv, Rh = _R(w, prm, v, vh)
        return np.sum(wv * Rv) + np.sum(wh * Rh)

    for x, g, other_first in ((w.v, gv, True), (w.vhat, gh, False)):
        fd = np.empty(x.size)
        for i in range(x.size):
            e = np.zeros(x.size)
            e[i] = FD_H
            e = e.reshape(x.shape)
            if other_first:
                fd[i] = (phi(w.v + e, w.vhat) - phi(w.v - e, w.vhat)) / (2 * FD_H)
            else:
                fd[i] = (phi(w.v, w.vhat + e) - phi(w.v, w.vhat - e)) / (2 * FD_H)
        assert np.linalg.norm(g.ravel() - fd) < 1e-7 * np.linalg.norm(fd)
