"""GPU residual of tetrahedral macro-elements (mehdg_tet_residual) against
the oracle (oracle.forms on oracle.tet geometry).

* p = 1, 2, 3 on the Taylor-Green box of Kuhn tetrahedra (12 macros, every
  flux, viscous and inviscid), per macro normwise relative <= 1e-12 for R_V
  and R_Vhat; R_Q with q lifted vanishes to round-off, checked against the
  size of its terms; with q given (seeded), R_Q itself to 1e-12;
* distorted macros (random affine vertices): general face normals;
* wall faces (isothermal no-slip) on a seeded set of faces;
* the entropy production to 1e-12 of the size of the face terms;
* a macro with a non-physical state gets NaN outputs and ENONPHYSICAL while
  the others are unaffected;
* mehdg_tet_jvp: the oracle's dense Jacobian (forms.jacobian, with the
  pseudo-time term) times the direction, full (dq given) and reduced (dq the
  weak gradient of (dv, dvhat)), per macro normwise relative <= 1e-12, with
  walls; and at p = 3 against a central difference of the GPU residual
  (EC flux, viscous, alpha_ps = 0, step 1e-6, relative 1e-7);
* the local work of a Newton step (mehdg_tet_assemble, _condense, _recover)
  against oracle.forms.condense and oracle.local.recover: Ahat, bhat, dv,
  dq per macro normwise relative <= 1e-12, p = 1, 2, 3, walls; and the call
  order (ESTATE);
* mehdg_tet_vjp (J_r^T w from the assembled bordered matrices) against the
  oracle's reduced Jacobian transposed, and the adjoint identity
  <w, J_r x> = <J_r^T w, x> against mehdg_tet_jvp, per macro at 1e-12;
* mehdg_tet_condense_rhs: with (-R_V, -R_Vhat) it reproduces bhat of the
  condensation; with a seeded right-hand side, bhat and the recovered dV
  against the oracle's S, X, Y at 1e-12;
* more macros than one column launch holds (66654 at p = 1), macros on both
  sides of the launch boundary;
* the benchmark's tetrahedral workloads at full size (1296-macro step, 10368-
  macro residual), sampled macros against the oracle; the Mach 0.1 residual
  R_V is bounded by max(1e-12, 10x the oracle's own change under one-ulp
  input noise), measured in the test (about 6e-13).
"""
import numpy as np
import pytest

from oracle import forms, tet
from paper_2507_22195_amd import workloads as W
from tests.gpu_util import banner, dev, empty, host, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _run(w, X, q=None, face_bc=None, prm=None):
    from paper_2507_22195_amd import mehdg
    prm = prm or w.params
    ctx = mehdg.TetContext(w.p, X, prm, face_bc=face_bc)
    S = ctx.shapes()
    R_q, R_v, R_vh, ent = empty(S["R_q"]), empty(S["R_v"]), empty(S["R_vhat"]), empty(S["entropy"])
    ctx.residual(dev(w.v), dev(w.vhat), None if q is None else dev(q), dev(w.v_old), R_q, R_v, R_vh, ent)
    rc, st = ctx.status()
    ctx.close()
    return rc, st, dict(R_q=host(R_q), R_v=host(R_v), R_vhat=host(R_vh), entropy=host(ent))


def _check(w, X, q=None, face_bc=None, prm=None, label=""):
    prm = prm or w.params
    banner(f"tet residual {label}: p={w.p} macros={w.n_macro} flux={prm['flux']} viscous={prm['viscous']}")
    rc, st, got = _run(w, X, q=q, face_bc=face_bc, prm=prm)
    assert rc == 0, st
    ref = forms.residual(tet.TetGeometry(w.p, X), w.v, w.vhat, w.v_old, prm, q=q, face_bc=face_bc)
    errs = dict(R_v=rel_err(got["R_v"], ref["R_v"]), R_vhat=rel_err(got["R_vhat"], ref["R_vhat"]))
    if q is None:
        # R_Q vanishes: compare with the size of its terms, |M q|
        geo = tet.TetGeometry(w.p, X)
        Mq = np.einsum("mab,mkjb->mkja", forms.mass(geo), ref["q"])
        errs["R_q"] = float(np.max(np.abs(got["R_q"]) / np.abs(Mq).max()))
    else:
        errs["R_q"] = rel_err(got["R_q"], ref["R_q"])
    escale = np.abs(ref["R_vhat"]).max() * np.abs(w.vhat).max()
    errs["entropy"] = float(np.max(np.abs(got["entropy"] - ref["entropy"])) / escale)
    banner(f"  errors {errs}")
    for k, e in errs.items():
        assert e <= TOL, (k, e)


def _tgv(p, flux="ES", viscous=True, shape=(2, 1, 1), seed=61):
    return W.tet_tgv_workload(shape=shape, p=p, M0=0.3, Re=500.0, flux=flux, viscous=viscous,
                              seed_v=seed, seed_vh=seed + 1, amp=1e-2)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tet_residual_matches_oracle(p):
    w = _tgv(p)
    _check(w, w.mesh.X, label="tgv ES viscous")


@pytest.mark.parametrize("flux,viscous", [("EC", False), ("ES", False), ("KEPES", True)])
def test_tet_residual_fluxes(flux, viscous):
    w = _tgv(2, flux, viscous, seed=71)
    _check(w, w.mesh.X, label=f"tgv {flux}")


def test_tet_residual_given_q_and_distorted_macros():
    w = _tgv(2, "KEPES", True, seed=81)
    rng = np.random.default_rng(5)
    X = w.mesh.X + 0.15 * rng.standard_normal(w.mesh.X.shape)
    q = 0.1 * rng.standard_normal((w.n_macro, 5, 3, w.v.shape[2]))
    _check(w, X, q=q, label="distorted, q given")
    _check(w, X, label="distorted, q lifted")


def test_tet_residual_walls():
    w = _tgv(3, "ES", True, seed=91)
    rng = np.random.default_rng(7)
    bc = (rng.random((w.n_macro, 4)) < 0.3).astype(np.uint8)
    prm = dict(w.params, T_wall=1.05)
    _check(w, w.mesh.X, face_bc=bc, prm=prm, label="walls")


def test_tet_nonphysical_macro_is_flagged():
    w = _tgv(1)
    bad = 3
    w.v[bad, 4, :] = 0.5                     # beta = -v5 < 0 at every point of the macro
    banner("tet residual: non-physical state in macro 3")
    rc, st, got = _run(w, w.mesh.X)
    assert rc == 5 and st[bad] == 5 and np.count_nonzero(st) == 1, st
    assert np.all(np.isnan(got["R_v"][bad])) and np.all(np.isnan(got["R_vhat"][bad]))
    ok = [m for m in range(w.n_macro) if m != bad]
    ref = forms.residual(tet.TetGeometry(1, w.mesh.X[ok]), w.v[ok], w.vhat[ok], w.v_old[ok], w.params)
    assert rel_err(got["R_v"][ok], ref["R_v"]) <= TOL


def _oracle_jvp(w, X, prm, dv, dh, dq=None, face_bc=None):
    geo = tet.TetGeometry(w.p, X)
    J = forms.jacobian(geo, w.v, w.vhat, w.v_old, prm, face_bc=face_bc)
    if dq is None:
        dq = forms.lift_q(geo, dv, dh)
    M_ = w.n_macro
    x = np.concatenate([dq.reshape(M_, -1), dv.reshape(M_, -1), dh.reshape(M_, -1)], axis=1)
    out = []
    for m in range(M_):
        Jf = np.block([[J["A_qq"][m], J["A_qv"][m], J["A_qvh"][m]],
                       [J["A_vq"][m], J["A_vv"][m], J["A_vvh"][m]],
                       [J["A_hq"][m], J["A_hv"][m], J["A_hh"][m]]])
        out.append(Jf @ x[m])
    y = np.stack(out)
    NQ, NV = dq[0].size, dv[0].size
    return y[:, :NQ].reshape(dq.shape), y[:, NQ:NQ + NV].reshape(dv.shape), y[:, NQ + NV:].reshape(dh.shape)


def _gpu_jvp(w, X, prm, dv, dh, dq=None, face_bc=None):
    from paper_2507_22195_amd import mehdg
    ctx = mehdg.TetContext(w.p, X, prm, face_bc=face_bc)
    S = ctx.shapes()
    Jq, Jv, Jh = empty(S["R_q"]), empty(S["R_v"]), empty(S["R_vhat"])
    ctx.jvp(dev(w.v), dev(w.vhat), None, dev(dv), dev(dh), None if dq is None else dev(dq), Jq, Jv, Jh)
    rc, st = ctx.status()
    ctx.close()
    assert rc == 0, st
    return host(Jq), host(Jv), host(Jh)


@pytest.mark.parametrize("p,flux,walls", [(1, "KEPES", False), (2, "ES", True), (2, "EC", False)])
def test_tet_jvp_matches_oracle(p, flux, walls):
    w = _tgv(p, flux, flux != "EC", shape=(1, 1, 1), seed=101)
    prm = dict(w.params, T_wall=1.05)
    bc = None
    if walls:
        bc = (np.random.default_rng(3).random((w.n_macro, 4)) < 0.3).astype(np.uint8)
    rng = np.random.default_rng(4)
    dv, dh = rng.standard_normal(w.v.shape), rng.standard_normal(w.vhat.shape)
    dq = rng.standard_normal((w.n_macro, 5, 3, w.v.shape[2]))
    for label, dqq in (("full", dq), ("reduced", None)):
        banner(f"tet jvp {label}: p={p} flux={flux} walls={walls}")
        got = _gpu_jvp(w, w.mesh.X, prm, dv, dh, dq=dqq, face_bc=bc)
        ref = _oracle_jvp(w, w.mesh.X, prm, dv, dh, dq=dqq, face_bc=bc)
        errs = dict(JR_v=rel_err(got[1], ref[1]), JR_vhat=rel_err(got[2], ref[2]))
        if dqq is not None:
            errs["JR_q"] = rel_err(got[0], ref[0])
        banner(f"  errors {errs}")
        for k, e in errs.items():
            assert e <= TOL, (k, e)


def test_tet_jvp_p3_against_central_difference_of_the_gpu_residual():
    # EC flux: no |.| anywhere in the trace flux, so the residual is smooth
    # (the ES and KEPES dissipation has |Vhat.n|, which this state comes within
    # 6e-6 of at some face point); the other fluxes are covered exactly above
    w = _tgv(3, "EC", True, seed=111)
    prm = dict(w.params, alpha_ps=0.0)
    rng = np.random.default_rng(6)
    dv, dh = rng.standard_normal(w.v.shape), rng.standard_normal(w.vhat.shape)
    banner("tet jvp p3 vs central difference of the residual")
    got = _gpu_jvp(w, w.mesh.X, prm, dv, dh)
    eps = 1e-6
    outs = []
    for sgn in (1.0, -1.0):
        ws = W.TetWorkload(w.name, w.p, w.mesh, prm, w.v + sgn * eps * dv, w.vhat + sgn * eps * dh, w.v_old,
                           w.face_bc)
        rc, st, r = _run(ws, w.mesh.X, prm=prm)
        assert rc == 0, st
        outs.append(r)
    for key, g in (("R_v", got[1]), ("R_vhat", got[2])):
        fd = (outs[0][key] - outs[1][key]) / (2 * eps)
        e = rel_err(g, fd)
        banner(f"  {key}: {e:.2e}")
        assert e <= 1e-7, (key, e)


def _step(w, prm, face_bc, dvh):
    from paper_2507_22195_amd import mehdg
    ctx = mehdg.TetContext(w.p, w.mesh.X, prm, face_bc=face_bc)
    S = ctx.shapes()
    e = {k: empty(S[k]) for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
    ctx.assemble(dev(w.v), dev(w.vhat), dev(w.v_old), e["R_q"], e["R_v"], e["R_vhat"], e["entropy"])
    ctx.condense(e["Ahat"], e["bhat"])
    ctx.recover(e["R_q"], dev(dvh), e["dv"], e["dq"])
    rc, st = ctx.status()
    ctx.close()
    assert rc == 0, st
    return {k: host(x) for k, x in e.items()}


@pytest.mark.parametrize("p,flux,walls", [(1, "KEPES", True), (2, "ES", False), (3, "ES", True)])
def test_tet_step_matches_oracle(p, flux, walls):
    from oracle import local
    w = _tgv(p, flux, True, shape=(1, 1, 1), seed=121)
    if p == 3:
        w = W.TetWorkload(w.name, w.p, w.mesh, w.params, w.v[:3], w.vhat[:3], w.v_old[:3], w.face_bc[:3])
        w.mesh = W.TetMesh(w.mesh.shape, w.mesh.lo, w.mesh.hi, w.mesh.X[:3], w.mesh.vid[:3])
    prm = dict(w.params, T_wall=1.05)
    bc = None
    if walls:
        bc = (np.random.default_rng(5).random((w.n_macro, 4)) < 0.3).astype(np.uint8)
    dvh = 1e-2 * np.random.default_rng(6).standard_normal(w.vhat.shape)
    banner(f"tet step: p={p} flux={flux} walls={walls} macros={w.n_macro}")
    got = _step(w, prm, bc, dvh)
    ref = forms.condense(tet.TetGeometry(w.p, w.mesh.X), w.v, w.vhat, w.v_old, prm, face_bc=bc)
    rdv, rdq = local.recover(ref, dvh)
    errs = dict(R_v=rel_err(got["R_v"], ref["R_v"]), Ahat=rel_err(got["Ahat"], ref["Ahat"]),
                bhat=rel_err(got["bhat"], ref["bhat"]), dv=rel_err(got["dv"], rdv), dq=rel_err(got["dq"], rdq))
    banner(f"  errors {errs}")
    for k, e in errs.items():
        assert e <= TOL, (k, e)


def test_tet_step_call_order():
    from paper_2507_22195_amd import mehdg
    w = _tgv(1, shape=(1, 1, 1))
    ctx = mehdg.TetContext(w.p, w.mesh.X, w.params)
    S = ctx.shapes()
    with pytest.raises(mehdg.MehdgError) as ex:
        ctx.condense(empty(S["Ahat"]), empty(S["bhat"]))
    assert ex.value.code == 4
    with pytest.raises(mehdg.MehdgError) as ex:
        ctx.recover(empty(S["R_q"]), empty(S["vhat"]), empty(S["dv"]), empty(S["dq"]))
    assert ex.value.code == 4
    ctx.close()


def test_tet_full_size_sampled_against_oracle():
    """The benchmark's tetrahedral workloads at full size, in the launch shapes
    bench.py times: the step on 6^3 cubes x 6 = 1296 p = 3 macros and the
    residual on 12^3 cubes x 6 = 10368 macros, two sampled macros of each
    against the oracle (plus finite, flag-free outputs everywhere)."""
    from oracle import local
    from paper_2507_22195_amd import mehdg
    w = W.tet_tgv_workload(shape=(6, 6, 6), p=3, M0=0.1, Re=1600.0, flux="KEPES", seed_v=61, seed_vh=62)
    dvh = 1e-2 * np.random.default_rng(9).standard_normal(w.vhat.shape)
    banner(f"tet step full size: {w.n_macro} macros, p=3, KEPES")
    got = _step(w, w.params, None, dvh)
    for k in ("Ahat", "bhat", "dv", "dq"):
        assert np.all(np.isfinite(got[k])), k
    idx = [17, 1201]
    ref = forms.condense(tet.TetGeometry(3, w.mesh.X[idx]), w.v[idx], w.vhat[idx], w.v_old[idx], w.params)
    rdv, rdq = local.recover(ref, dvh[idx])
    errs = dict(Ahat=rel_err(got["Ahat"][idx], ref["Ahat"]), bhat=rel_err(got["bhat"][idx], ref["bhat"]),
                dv=rel_err(got["dv"][idx], rdv), dq=rel_err(got["dq"][idx], rdq))
    banner(f"  sampled errors {errs}")
    for k, e in errs.items():
        assert e <= TOL, (k, e)
    wr = W.tet_tgv_workload(shape=(12, 12, 12), p=3, M0=0.1, Re=1600.0, flux="KEPES", seed_v=61, seed_vh=62)
    banner(f"tet residual full size: {wr.n_macro} macros")
    rc, st, r = _run(wr, wr.mesh.X)
    assert rc == 0, st
    idx = [5, 9999]
    geo = tet.TetGeometry(3, wr.mesh.X[idx])
    v, vh, vo = wr.v[idx], wr.vhat[idx], wr.v_old[idx]
    ref = forms.residual(geo, v, vh, vo, wr.params)
    # At Mach 0.1 R_V is a small difference of large flux terms: the oracle's
    # own R_V moves by ~6e-13 (relative) under one-ulp noise on (v, vhat).
    # The bound is max(1e-12, 10x that measured change), per macro.
    rng = np.random.default_rng(13)
    floor = {k: np.zeros(2) for k in ("R_v", "R_vhat")}
    for _ in range(2):
        ulp = lambda x: x * (1.0 + 2.2e-16 * rng.choice([-1.0, 1.0], x.shape))
        r2 = forms.residual(geo, ulp(v), ulp(vh), vo, wr.params)
        for k in floor:
            d = np.linalg.norm((r2[k] - ref[k]).reshape(2, -1), axis=1)
            floor[k] = np.maximum(floor[k], 10.0 * d)
    for k in ("R_v", "R_vhat"):
        assert np.all(np.isfinite(r[k])), k
        num = np.linalg.norm((r[k][idx] - ref[k]).reshape(2, -1), axis=1)
        den = np.linalg.norm(ref[k].reshape(2, -1), axis=1)
        bound = np.maximum(TOL * den, floor[k])
        banner(f"  {k}: errors {num / den}, bounds {bound / den}")
        assert np.all(num <= bound), (k, num / den, bound / den)


@pytest.mark.parametrize("p,flux", [(1, "KEPES"), (2, "ES")])
def test_tet_vjp(p, flux):
    from oracle import linearized
    from paper_2507_22195_amd import mehdg
    w = _tgv(p, flux, True, shape=(1, 1, 1), seed=131)
    ctx = mehdg.TetContext(w.p, w.mesh.X, w.params)
    S = ctx.shapes()
    e = {k: empty(S[k]) for k in ("R_q", "R_v", "R_vhat", "entropy")}
    rng = np.random.default_rng(8)
    wv, wh = rng.standard_normal(w.v.shape), rng.standard_normal(w.vhat.shape)
    xv, xh = rng.standard_normal(w.v.shape), rng.standard_normal(w.vhat.shape)
    banner(f"tet vjp: p={p} flux={flux}")
    ctx.assemble(dev(w.v), dev(w.vhat), dev(w.v_old), e["R_q"], e["R_v"], e["R_vhat"], e["entropy"])
    gv, gh = empty(S["v"]), empty(S["vhat"])
    ctx.vjp(dev(wv), dev(wh), gv, gh)
    Jq, Jv, Jh = empty(S["R_q"]), empty(S["R_v"]), empty(S["R_vhat"])
    ctx.jvp(dev(w.v), dev(w.vhat), None, dev(xv), dev(xh), None, Jq, Jv, Jh)
    rc, st = ctx.status()
    ctx.close()
    assert rc == 0, st
    gv, gh, Jv, Jh = host(gv), host(gh), host(Jv), host(Jh)
    J = forms.jacobian(tet.TetGeometry(w.p, w.mesh.X), w.v, w.vhat, w.v_old, w.params)
    Jr = linearized.reduced_jacobian(J)
    M_ = w.n_macro
    wvec = np.concatenate([wv.reshape(M_, -1), wh.reshape(M_, -1)], axis=1)
    ref = np.einsum("mji,mj->mi", Jr, wvec)
    got = np.concatenate([gv.reshape(M_, -1), gh.reshape(M_, -1)], axis=1)
    err = rel_err(got, ref)
    lhs = np.einsum("mi,mi->m", wvec, np.concatenate([Jv.reshape(M_, -1), Jh.reshape(M_, -1)], axis=1))
    rhs = np.einsum("mi,mi->m", got, np.concatenate([xv.reshape(M_, -1), xh.reshape(M_, -1)], axis=1))
    adj = float(np.max(np.abs(lhs - rhs) / np.abs(lhs)))
    banner(f"  vjp error {err:.2e}, adjoint identity {adj:.2e}")
    assert err <= TOL and adj <= TOL, (err, adj)
    # after the condensation the assembled matrices are gone
    ctx = mehdg.TetContext(w.p, w.mesh.X, w.params)
    with pytest.raises(mehdg.MehdgError) as ex:
        ctx.vjp(dev(wv), dev(wh), empty(S["v"]), empty(S["vhat"]))
    assert ex.value.code == 4
    ctx.close()


def test_tet_step_beyond_one_launch_of_macros():
    """More macros than one column launch holds (65535 along the grid's y):
    23 x 23 x 21 cubes x 6 = 66654 p = 1 macros; macros on both sides of the
    launch boundary against the oracle."""
    import torch
    from oracle import local
    from paper_2507_22195_amd import mehdg
    w = W.tet_tgv_workload(shape=(23, 23, 21), p=1, M0=0.3, Re=500.0, flux="ES", seed_v=141, seed_vh=142)
    assert w.n_macro > 65535
    banner(f"tet step: {w.n_macro} p=1 macros (two column launches)")
    ctx = mehdg.TetContext(w.p, w.mesh.X, w.params)
    S = ctx.shapes()
    e = {k: empty(S[k]) for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
    dvh = 1e-2 * np.random.default_rng(10).standard_normal(w.vhat.shape)
    ctx.assemble(dev(w.v), dev(w.vhat), dev(w.v_old), e["R_q"], e["R_v"], e["R_vhat"], e["entropy"])
    ctx.condense(e["Ahat"], e["bhat"])
    ctx.recover(e["R_q"], dev(dvh), e["dv"], e["dq"])
    rc, st = ctx.status()
    assert rc == 0, st
    idx = [0, 65534, 65535, w.n_macro - 1]
    got = {k: host(e[k][torch.tensor(idx, device="cuda")]) for k in ("Ahat", "bhat", "dv", "dq")}
    ctx.close()
    ref = forms.condense(tet.TetGeometry(1, w.mesh.X[idx]), w.v[idx], w.vhat[idx], w.v_old[idx], w.params)
    rdv, rdq = local.recover(ref, dvh[idx])
    errs = dict(Ahat=rel_err(got["Ahat"], ref["Ahat"]), bhat=rel_err(got["bhat"], ref["bhat"]),
                dv=rel_err(got["dv"], rdv), dq=rel_err(got["dq"], rdq))
    banner(f"  errors {errs}")
    for k, x in errs.items():
        assert x <= TOL, (k, x)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tet_condense_rhs(p):
    from paper_2507_22195_amd import mehdg
    w = _tgv(p, "ES", True, shape=(1, 1, 1), seed=151)
    ctx = mehdg.TetContext(w.p, w.mesh.X, w.params)
    S = ctx.shapes()
    e = {k: empty(S[k]) for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
    banner(f"tet condense_rhs: p={p}")
    ctx.assemble(dev(w.v), dev(w.vhat), dev(w.v_old), e["R_q"], e["R_v"], e["R_vhat"], e["entropy"])
    ctx.condense(e["Ahat"], e["bhat"])
    b1 = empty(S["bhat"])
    ctx.condense_rhs(-e["R_v"], (-e["R_vhat"]).reshape(S["bhat"]).contiguous(), b1)
    same = rel_err(host(b1), host(e["bhat"]))
    rng = np.random.default_rng(17)
    rv, rh = rng.standard_normal(w.v.shape), rng.standard_normal(S["bhat"])
    b2 = empty(S["bhat"])
    ctx.condense_rhs(dev(rv), dev(rh), b2)
    dvh = rng.standard_normal(w.vhat.shape)
    ctx.recover(e["R_q"], dev(dvh), e["dv"], e["dq"])
    rc, st = ctx.status()
    ctx.close()
    assert rc == 0, st
    ref = forms.condense(tet.TetGeometry(p, w.mesh.X), w.v, w.vhat, w.v_old, w.params)
    M_ = w.n_macro
    rb, rdv = [], []
    for m in range(M_):
        Ssol = np.linalg.solve(ref["S"][m], np.column_stack([rv[m].ravel(), ref["Y"][m] @ dvh[m].ravel()]))
        rb.append(rh[m] - ref["X"][m] @ Ssol[:, 0])
        rdv.append(Ssol[:, 0] + Ssol[:, 1])
    errs = dict(same=same, bhat=rel_err(host(b2), np.stack(rb)),
                dv=rel_err(host(e["dv"]).reshape(M_, -1), np.stack(rdv)))
    banner(f"  errors {errs}")
    for k, x in errs.items():
        assert x <= TOL, (k, x)
