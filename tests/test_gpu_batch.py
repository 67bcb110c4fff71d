"""Macro-elements of mixed degree in one step (the library's mehdg_batch_*
calls through paper_2507_22195_amd.batch).

On a 3x2x2 viscous Taylor-Green box with degrees drawn from {1, 2, 3} and
isothermal walls on the -z face of a third of the macros: every
output of the batched step (residual, entropy production, Ahat, bhat, dV,
dQ) equals, bit for bit, what a single-degree context computes for the same
macros (the same kernels on the same data), in FP64 and in the FP32 mode with
FP64 refinement; one macro of each degree has its Ahat compared with the
oracle (1e-12); the batched FP64 step captured in one HIP graph (three degree
groups on three forked streams) replays to the same bits.
"""
import numpy as np
import pytest

from oracle import local
from paper_2507_22195_amd import workloads as W
from tests.gpu_util import banner, dev, empty, host, rel_err

pytestmark = pytest.mark.gpu


def test_mixed_degree_batch():
    import torch
    from paper_2507_22195_amd import mehdg
    from paper_2507_22195_amd.batch import MixedBatch
    p, bc, parts = W.mixed_degree_tgv(shape=(3, 2, 2), degrees=(1, 2, 3), seed_p=41, wall_frac=0.34)
    banner(f"batch: degrees {dict(zip(*np.unique(p, return_counts=True)))}, {int(bc.sum())} wall faces")
    h = np.empty((p.size, 3))
    for d, w in parts.items():
        h[np.nonzero(p == d)[0]] = w.mesh.h
    prm = parts[1].params
    b = MixedBatch(p, h, prm, face_bc=bc)
    rng = np.random.default_rng(7)
    dvh_parts = {d: 1e-2 * rng.standard_normal(w.vhat.shape) for d, w in parts.items()}
    v = dev(b.pack("v", {d: w.v for d, w in parts.items()}))
    vh = dev(b.pack("vhat", {d: w.vhat for d, w in parts.items()}))
    vo = dev(b.pack("v", {d: w.v_old for d, w in parts.items()}))
    dvh = dev(b.pack("vhat", dvh_parts))
    out = {k: b.alloc(k) for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
    args = (v, vh, vo, out["R_q"], out["R_v"], out["R_vhat"], out["entropy"], out["Ahat"], out["bhat"], dvh,
            out["dv"], out["dq"])
    b.step(*args, prec="fp32")
    torch.cuda.synchronize()
    rc, st = b.status()
    assert rc == 0 and not st.any()
    ref32 = {k: t.clone() for k, t in out.items()}
    b.step(*args)
    torch.cuda.synchronize()
    rc, st = b.status()
    assert rc == 0 and not st.any()
    ref = {k: t.clone() for k, t in out.items()}
    assert sorted(b.order.tolist()) == list(range(p.size)) and np.all(np.diff(p[b.order]) >= 0)

    for gi, (d, first, cnt, _) in enumerate(b.groups):
        w = parts[d]
        ctx = mehdg.Context(d, w.mesh.h, prm, face_bc=w.face_bc)
        S = ctx.shapes()
        o = {k: empty(S[k]) for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
        ctx.assemble(dev(w.v), dev(w.vhat), None, dev(w.v_old), o["R_q"], o["R_v"], o["R_vhat"], o["entropy"],
                     want_blocks=True)
        ctx.condense(o["Ahat"], o["bhat"])
        ctx.recover(o["R_q"], dev(dvh_parts[d]), o["dv"], o["dq"])
        torch.cuda.synchronize()
        for k, t in o.items():
            assert torch.equal(b.view(ref[k], k, gi), t), f"degree {d}: {k} differs from a single-degree context"
        ctx.assemble(dev(w.v), dev(w.vhat), None, dev(w.v_old), o["R_q"], o["R_v"], o["R_vhat"], o["entropy"],
                     want_blocks=True)
        ctx.condense(o["Ahat"], o["bhat"], prec="fp32")
        ctx.recover(o["R_q"], dev(dvh_parts[d]), o["dv"], o["dq"])
        torch.cuda.synchronize()
        for k, t in o.items():
            assert torch.equal(b.view(ref32[k], k, gi), t), f"degree {d}: fp32 {k} differs from a single context"
        ctx.close()
        ws = W.subset(w, [0])
        e = rel_err(host(b.view(ref["Ahat"], "Ahat", gi))[:1],
                    local.condense(ws.p, ws.mesh.h, ws.v, ws.vhat, ws.v_old, ws.params,
                                   face_bc=ws.face_bc)["Ahat"])
        banner(f"  degree {d}: {cnt} macros equal the single-degree context; Ahat vs oracle {e:.1e}")
        assert e < 1e-12

    # one graph for the whole mixed step
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.step(*args)
    for _ in range(2):
        for t in out.values():
            t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for k in out:
            assert torch.equal(out[k], ref[k]), f"graph replay differs in {k}"
    banner("  graph replays equal the eager batched step")
    del g
    b.close()
