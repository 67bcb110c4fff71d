"""Parity of the hexahedral Newton step at the benchmark's full sizes, in the
launch configuration the benchmark times (Sec. 6.2 eq. R2-R6).

* The headline workload: viscous Taylor-Green vortex on 16^3 macro-elements of
  2x2x2 p = 2 hexahedra (4096 macros, N_V = 625, N_VH = 750), ES flux,
  Re 1600, Mach 0.1.
* The degree-3 workload: 16x16x8 macros of 2x2x2 p = 3 hexahedra (2048 macros,
  N_V = 1715, N_VH = 1470), KEPES flux, Re 5000, Mach 0.3.
* Degree 4 on two macros (the largest degree of the mixed-degree batches).
* The mixed-degree batch of 4096 macros (degrees 1..4, walls) through the
  batch calls, sampled per degree.

The whole batch runs assemble + condense + recover on the GPU; the oracle
computes a seeded sample of macros one by one.  The sample covers every
residue of the macro index mod 8 (the launches deal consecutive macros to
the eight XCDs in turn), the first and the last macro.  Compared per sampled
macro: the bordered blocks S, Y, X, A' (copied before the condensation),
Ahat, bhat, dV, dQ, at the 1e-12 bar of the FP64 path.  Outputs that carry
r_V = -R_V (a small difference of large flux terms at low Mach) take the
oracle's own one-ulp floor, propagated through the exact solve, as in the
small-mesh tests.  For KEPES the blocks Y, X, A' take the oracle's own
one-ulp block sensitivity (the pressure switch theta = sqrt|(P - P_hat)/(P +
P_hat)| of eq. KEPES5 has an unbounded derivative where P = P_hat); the
number of face points close to that switch is printed beside it.  At degree 3
(kappa(S) ~ 8e3) Ahat inherits that sensitivity through S^-1: for KEPES it
takes its own measured floor too (about 2e-12 relative); the ES workload
keeps the plain bar for every output.
"""
import numpy as np
import pytest

from oracle import local
from oracle import physics as ph
from paper_2507_22195_amd import workloads as W
from tests.gpu_util import banner, dev, empty, host, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _sample(n_macro, seed, lanes=range(8)):
    """The first and the last macro, and one seeded macro per listed residue mod 8."""
    rng = np.random.default_rng(seed)
    picks = {0, n_macro - 1}
    for lane in lanes:
        picks.add(int(rng.choice(np.arange(lane, n_macro, 8))))
    return sorted(picks)


def _near_switch(w, idx):
    """Face quadrature points of the sampled macros with |P - P_hat|/(P + P_hat)
    below 1e-4 and 1e-6 (of all face points)."""
    ws = W.subset(w, idx)
    geo = local.Geometry(ws.p, ws.mesh.h)
    q = local.lift_q(geo, ws.v, ws.vhat)
    _, _, _, faces = local._points(geo, ws.v, q, ws.vhat, ws.v_old)
    xs = []
    for vs, _, vhs in faces:
        _, _, P, _ = ph.primitive_from_entropy([vs[:, k] for k in range(5)], ws.params["gamma"])
        _, _, Ph, _ = ph.primitive_from_entropy([vhs[:, k] for k in range(5)], ws.params["gamma"])
        xs.append(np.abs(P - Ph) / (P + Ph))
    x = np.concatenate([a.ravel() for a in xs])
    return int(np.sum(x < 1e-4)), int(np.sum(x < 1e-6)), x.size


def _oracle_floors(ws, dvhat, with_blocks):
    """Per-macro one-ulp change of the oracle's r_V, and (with_blocks) of its
    blocks, Frobenius norms times 10."""
    rng = np.random.default_rng(7)
    base = local.condense(ws.p, ws.mesh.h, ws.v, ws.vhat, ws.v_old, ws.params, face_bc=ws.face_bc)
    base["dv"], base["dq"] = local.recover(base, dvhat)
    keys = ("r_v", "S", "Y", "X", "Ap", "Ahat") if with_blocks else ("r_v",)
    worst = {k: np.zeros(ws.n_macro) for k in keys}
    for _ in range(2):
        pert = lambda x: x * (1 + 2.2e-16 * rng.uniform(-1, 1, x.shape))
        if with_blocks:
            c = local.condense(ws.p, ws.mesh.h, pert(ws.v), pert(ws.vhat), ws.v_old, ws.params,
                               face_bc=ws.face_bc)
        else:
            c = dict(r_v=-local.residual(ws.p, ws.mesh.h, pert(ws.v), pert(ws.vhat), ws.v_old,
                                         ws.params, face_bc=ws.face_bc)["R_v"].reshape(ws.n_macro, -1))
        for k in keys:
            d = np.linalg.norm((c[k] - base[k]).reshape(ws.n_macro, -1), axis=1)
            worst[k] = np.maximum(worst[k], d)
    return base, {k: 10.0 * v for k, v in worst.items()}


def _run(w, idx, kepes):
    import torch
    from paper_2507_22195_amd import mehdg
    banner(f"full size: {w.name} p={w.p} M={w.n_macro} flux={w.params['flux']} samples={idx}")
    rng = np.random.default_rng(5)
    dvhat_s = 1e-2 * rng.standard_normal((len(idx),) + w.vhat.shape[1:])
    torch.cuda.empty_cache()
    ctx = mehdg.Context(w.p, w.mesh.h, w.params)
    S = ctx.shapes()
    R_q, R_v, R_vh, ent = empty(S["R_q"]), empty(S["R_v"]), empty(S["R_vhat"]), empty(S["entropy"])
    ctx.assemble(dev(w.v), dev(w.vhat), None, dev(w.v_old), R_q, R_v, R_vh, ent, want_blocks=True)
    bord = {m: ctx.bordered(m) for m in idx}
    Ahat, bhat = empty(S["Ahat"]), empty(S["bhat"])
    ctx.condense(Ahat, bhat)
    dvhat = torch.zeros(S["vhat"], dtype=torch.float64, device="cuda")
    dvhat[torch.tensor(idx, device="cuda")] = dev(dvhat_s)
    dv, dq = empty(S["dv"]), empty(S["dq"])
    ctx.recover(R_q, dvhat, dv, dq)
    rc, st = ctx.status()
    ii = torch.tensor(idx, device="cuda")
    got = dict(Ahat=host(Ahat[ii]), bhat=host(bhat[ii]), dv=host(dv[ii]), dq=host(dq[ii]))
    ctx.close()
    del Ahat, bhat, dv, dq, R_q, R_v, R_vh, ent, dvhat
    torch.cuda.empty_cache()
    assert rc == 0 and not st.any(), (rc, np.flatnonzero(st)[:10])
    banner("  GPU step done; oracle on the sample")

    ws = W.subset(w, idx)
    ref, fl = _oracle_floors(ws, dvhat_s, with_blocks=kepes)
    ref_dv, ref_dq = local.recover(ref, dvhat_s)
    NV, NH = ref["S"].shape[1], ref["Ap"].shape[1]
    if kepes:
        n4, n6, nall = _near_switch(w, idx)
        banner(f"  face points near the KEPES switch: {n4} below 1e-4, {n6} below 1e-6 (of {nall})")
    for i, m in enumerate(idx):
        Bm = bord[m]
        bfl = (lambda k: fl[k][i:i + 1] / TOL) if kepes else (lambda k: 0.0)
        e = dict(S=rel_err(Bm[None, :NV, :NV], ref["S"][i:i + 1], floor=bfl("S")),
                 Y=rel_err(-Bm[None, :NV, NV:NV + NH], ref["Y"][i:i + 1], floor=bfl("Y")),
                 X=rel_err(Bm[None, NV:, :NV], ref["X"][i:i + 1], floor=bfl("X")),
                 Ap=rel_err(Bm[None, NV:, NV:NV + NH], ref["Ap"][i:i + 1], floor=bfl("Ap")),
                 r_v=rel_err(Bm[None, :NV, NV + NH], ref["r_v"][i:i + 1], floor=fl["r_v"][i:i + 1] / TOL),
                 r_hat=rel_err(Bm[None, NV:, NV + NH], ref["r_hat"][i:i + 1]))
        banner(f"  macro {m}: " + " ".join(f"{k} {v:.2e}" for k, v in e.items()))
        assert all(v < TOL for v in e.values()), (m, e)
    if kepes:
        banner("  block floors (relative): " + " ".join(
            f"{k} {np.max(fl[k] / np.linalg.norm(ref[k].reshape(len(idx), -1), axis=1)):.1e}"
            for k in ("S", "Y", "X", "Ap", "Ahat")))
    Sinv = np.array([np.linalg.norm(np.linalg.inv(ref["S"][i]), 2) for i in range(len(idx))])
    Xn = np.array([np.linalg.norm(ref["X"][i], 2) for i in range(len(idx))])
    e_A = rel_err(got["Ahat"], ref["Ahat"], floor=fl["Ahat"] / TOL if kepes else 0.0)
    e_b = rel_err(got["bhat"], ref["bhat"], floor=10 * Xn * Sinv * fl["r_v"] / TOL)
    e_dv = rel_err(got["dv"], ref_dv, floor=10 * Sinv * fl["r_v"] / TOL)
    e_dq = rel_err(got["dq"], ref_dq, floor=10 * Sinv * fl["r_v"] / TOL)
    banner(f"  Ahat {e_A:.2e} bhat {e_b:.2e} dV {e_dv:.2e} dQ {e_dq:.2e}")
    assert e_A < TOL and e_b < TOL and e_dv < TOL and e_dq < TOL


def test_full_size_tgv16_p2_es():
    w = W.workload(2)
    assert w.n_macro == 4096 and w.p == 2
    _run(w, _sample(w.n_macro, 2024), kepes=False)


def test_full_size_tgv16x16x8_p3_kepes():
    w = W.workload(5)
    assert w.n_macro == 2048 and w.p == 3
    _run(w, _sample(w.n_macro, 2025, lanes=(3, 5)), kepes=True)


def test_degree4_macros_against_the_oracle():
    """Degree 4 (N_V 3645, N_VH 2430): two viscous Taylor-Green macros, ES
    flux, every block and output at the 1e-12 bar (the r_V floor as above)."""
    w = W.tgv_workload(shape=(2, 1, 1), p=4, M0=0.1, Re=1600.0, flux="ES", seed_v=21, seed_vh=22)
    _run(w, [0, 1], kepes=False)


def test_full_size_mixed_degree_batch_sampled():
    """The batching workload as the benchmark runs it: 4096 macros of degree
    drawn from {1, 2, 3, 4}, 20% with an isothermal wall, one batch call per
    phase (the degree-4 group streamed in waves when the workspace budget asks
    for it).  Per degree, the first and the last macro of its group and one
    seeded macro with a wall: Ahat, bhat, dV, dQ against the oracle at 1e-12
    (r_V's one-ulp floor as above)."""
    import torch
    from paper_2507_22195_amd.batch import MixedBatch
    p, bc, parts = W.mixed_degree_tgv(shape=(16, 16, 16), degrees=(1, 2, 3, 4), seed_p=41, wall_frac=0.2,
                                      seed_wall=42)
    h = np.empty((p.size, 3))
    for d, w in parts.items():
        h[np.nonzero(p == d)[0]] = w.mesh.h
    torch.cuda.empty_cache()
    b = MixedBatch(p, h, parts[1].params, face_bc=bc)
    banner(f"full-size batch: degrees {dict(zip(*np.unique(p, return_counts=True)))}, waves {b.waves}, "
           f"{int(bc.sum())} wall faces")
    rng = np.random.default_rng(11)
    dvh_parts = {d: 1e-2 * rng.standard_normal(w.vhat.shape) for d, w in parts.items()}
    v = dev(b.pack("v", {d: w.v for d, w in parts.items()}))
    vh = dev(b.pack("vhat", {d: w.vhat for d, w in parts.items()}))
    vo = dev(b.pack("v", {d: w.v_old for d, w in parts.items()}))
    dvh = dev(b.pack("vhat", dvh_parts))
    out = {k: b.alloc(k) for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
    b.step(v, vh, vo, out["R_q"], out["R_v"], out["R_vhat"], out["entropy"], out["Ahat"], out["bhat"], dvh,
           out["dv"], out["dq"])
    torch.cuda.synchronize()
    rc, st = b.status()
    assert rc == 0 and not st.any(), (rc, np.flatnonzero(st)[:10])
    picks, got = {}, {}
    for gi, (d, first, cnt, _) in enumerate(b.groups):
        walls = np.flatnonzero(parts[d].face_bc.any(axis=1))
        idx = sorted({0, cnt - 1, int(rng.choice(walls))})
        picks[d] = idx
        ii = torch.tensor(idx, device="cuda")
        got[d] = {k: host(b.view(out[k], k, gi)[ii]) for k in ("Ahat", "bhat", "dv", "dq")}
    b.close()
    del out, v, vh, vo, dvh
    torch.cuda.empty_cache()
    banner("  GPU step done; oracle on the sample")
    for d, idx in picks.items():
        ws = W.subset(parts[d], idx)
        ref, fl = _oracle_floors(ws, dvh_parts[d][idx], with_blocks=False)
        ref_dv, ref_dq = local.recover(ref, dvh_parts[d][idx])
        Sinv = np.array([np.linalg.norm(np.linalg.inv(ref["S"][i]), 2) for i in range(len(idx))])
        Xn = np.array([np.linalg.norm(ref["X"][i], 2) for i in range(len(idx))])
        g = got[d]
        e_A = rel_err(g["Ahat"], ref["Ahat"])
        e_b = rel_err(g["bhat"], ref["bhat"], floor=10 * Xn * Sinv * fl["r_v"] / TOL)
        e_dv = rel_err(g["dv"], ref_dv, floor=10 * Sinv * fl["r_v"] / TOL)
        e_dq = rel_err(g["dq"], ref_dq, floor=10 * Sinv * fl["r_v"] / TOL)
        banner(f"  degree {d}, group positions {idx} ({int(ws.face_bc.sum())} wall faces): "
               f"Ahat {e_A:.2e} bhat {e_b:.2e} dV {e_dv:.2e} dQ {e_dq:.2e}")
        assert e_A < TOL and e_b < TOL and e_dv < TOL and e_dq < TOL, d
