"""GPU parity of mehdg_assemble (residual part) against the FP64 oracle.

Bar: per macro, |gpu - oracle| <= max(1e-12 |oracle|, 10 * s), where s is
the oracle's own change under a one-ulp relative perturbation of its inputs
(the rounding floor: the time term alpha_t (u(v) - u(v_old)) subtracts two
nearly equal states, which amplifies input rounding).  R_Q is compared
relative to the size of its mass term |(q, phi)|, since it is zero up to
rounding when q is the weak gradient; the entropy production relative to
the sum of the magnitudes it is formed from.
"""
import numpy as np
import pytest

from oracle import local
from paper_2507_22195_amd import workloads as W
from tests.gpu_util import banner, dev, empty, host, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12


def run_gpu(w, q=None):
    from paper_2507_22195_amd import mehdg
    ctx = mehdg.Context(w.p, w.mesh.h, w.params)
    S = ctx.shapes()
    out = dict(R_q=empty(S["R_q"]), R_v=empty(S["R_v"]), R_vhat=empty(S["R_vhat"]),
               entropy=empty(S["entropy"]))
    ctx.assemble(dev(w.v), dev(w.vhat), None if q is None else dev(q), dev(w.v_old),
                 out["R_q"], out["R_v"], out["R_vhat"], out["entropy"])
    rc, st = ctx.status()
    res = {k: host(t) for k, t in out.items()}
    ctx.close()
    return res, rc, st


def rounding_floor(w, q, key, trials=3):
    """10x the largest per-macro change of the oracle's output ``key`` under
    one-ulp relative perturbations of v, vhat (and q)."""
    rng = np.random.default_rng(123)
    base = local.residual(w.p, w.mesh.h, w.v, w.vhat, w.v_old, w.params, q=q)[key]
    worst = np.zeros(w.n_macro)
    for _ in range(trials):
        pert = lambda x: x * (1 + 2.2e-16 * rng.uniform(-1, 1, x.shape))
        r = local.residual(w.p, w.mesh.h, pert(w.v), pert(w.vhat), w.v_old, w.params,
                           q=None if q is None else pert(q))[key]
        worst = np.maximum(worst, np.linalg.norm((r - base).reshape(w.n_macro, -1), axis=1))
    return 10 * worst


def compare(w, q=None):
    banner(f"residual {w.name} p={w.p} M={w.n_macro} flux={w.params['flux']} visc={w.params['viscous']}"
           f" q={'given' if q is not None else 'lifted'}")
    got, rc, st = run_gpu(w, q)
    assert rc == 0 and not st.any()
    ref = local.residual(w.p, w.mesh.h, w.v, w.vhat, w.v_old, w.params, q=q)
    geo = local.Geometry(w.p, w.mesh.h)
    Mq = np.einsum("mab,mkjb->mkja", geo.mass(), ref["q"])
    e_rq = rel_err(got["R_q"], ref["R_q"], floor=np.linalg.norm(Mq.reshape(w.n_macro, -1), axis=1))
    fl = rounding_floor(w, q, "R_v")
    e_rv = rel_err(got["R_v"], ref["R_v"], floor=fl / TOL)
    e_rh = rel_err(got["R_vhat"], ref["R_vhat"])
    banner(f"  R_v rounding floor / |R_v| = {np.max(fl / np.linalg.norm(ref['R_v'].reshape(w.n_macro, -1), axis=1)):.2e}")
    ent_scale = np.sum(np.abs(ref["R_vhat"]), axis=(1, 2, 3)) * np.max(np.abs(w.vhat))
    e_en = float(np.max(np.abs(got["entropy"] - ref["entropy"]) / ent_scale))
    banner(f"  errors R_q {e_rq:.2e} R_v {e_rv:.2e} R_vhat {e_rh:.2e} entropy {e_en:.2e}")
    assert e_rq < TOL and e_rv < TOL and e_rh < TOL and e_en < TOL
    return got, ref


def test_residual_vortex_ec():
    got, ref = compare(W.workload(1))
    # entropy conservation carries over to the device result
    assert np.max(np.abs(got["entropy"])) < 1e-13


def test_residual_tgv_viscous_es():
    compare(W.workload(2, shape=(4, 4, 2)))


def test_residual_tgv_inviscid_all_fluxes():
    for flux in (0, 1, 2):
        w = W.workload(3, shape=(2, 2, 2))
        w.params = dict(w.params, flux=flux)
        compare(w)


def test_residual_kepes_viscous_p3():
    w = W.subset(W.workload(5, shape=(2, 2, 1)), [0, 3])
    compare(w)


def test_residual_p1_given_q():
    w = W.tgv_workload(shape=(3, 2, 2), p=1, M0=0.3, Re=400.0, flux="KEPES", seed_v=3, seed_vh=4)
    rng = np.random.default_rng(9)
    geo = local.Geometry(w.p, w.mesh.h)
    q = local.lift_q(geo, w.v, w.vhat) + 1e-2 * rng.standard_normal((w.n_macro, 5, 3, geo.n))
    compare(w, q=q)


def test_residual_full_config2_sampled():
    """Full 16^3 p=2 workload in one launch; sampled macros against the oracle."""
    w = W.workload(2)
    got, rc, st = run_gpu(w)
    assert rc == 0 and not st.any()
    idx = np.array([0, 1, 1234, 2047, 4095])
    ws = W.subset(w, idx)
    ref = local.residual(ws.p, ws.mesh.h, ws.v, ws.vhat, ws.v_old, ws.params)
    e_rv = rel_err(got["R_v"][idx], ref["R_v"], floor=rounding_floor(ws, None, "R_v") / TOL)
    e_rh = rel_err(got["R_vhat"][idx], ref["R_vhat"])
    banner(f"  full config-2 sampled errors R_v {e_rv:.2e} R_vhat {e_rh:.2e}")
    assert e_rv < TOL and e_rh < TOL
