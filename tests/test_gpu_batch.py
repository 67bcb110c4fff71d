"""Macro-elements of mixed degree in one step (the library's mehdg_batch_*
calls through paper_2507_22195_amd.batch).

On a 3x2x2 viscous Taylor-Green box with degrees drawn from {1, 2, 3, 4} and
isothermal walls on the -z face of a third of the macros:

* every output of the batched step (residual, entropy production, Ahat, bhat,
  dV, dQ) equals, bit for bit, what a single-degree context computes for the
  same macros (the same kernels on the same data), in FP64 and, for degrees
  1..3, in the FP32 mode with FP64 refinement; one macro of each degree has
  its Ahat compared with the oracle (1e-12);
* the batched FP64 step captured in one HIP graph (four degree groups on four
  forked streams) replays to the same bits;
* with a workspace budget too small for any group, every group is streamed
  one macro per wave (the recovery assembling and factoring each wave
  again): the same bits again, eager and graph-replayed;
* the residual pass of the whole groups, one persistent launch over a
  degree-sorted queue by default, gives the same bits as one launch per
  degree (residual_per_degree).
"""
import numpy as np
import pytest

from oracle import local
from paper_2507_22195_amd import workloads as W
from tests.gpu_util import banner, dev, empty, host, rel_err

pytestmark = pytest.mark.gpu

KEYS = ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")


def _setup():
    p, bc, parts = W.mixed_degree_tgv(shape=(3, 2, 2), degrees=(1, 2, 3, 4), seed_p=41, wall_frac=0.34)
    h = np.empty((p.size, 3))
    for d, w in parts.items():
        h[np.nonzero(p == d)[0]] = w.mesh.h
    rng = np.random.default_rng(7)
    dvh_parts = {d: 1e-2 * rng.standard_normal(w.vhat.shape) for d, w in parts.items()}
    return p, bc, parts, h, dvh_parts


def _inputs(b, parts, dvh_parts):
    v = dev(b.pack("v", {d: w.v for d, w in parts.items()}))
    vh = dev(b.pack("vhat", {d: w.vhat for d, w in parts.items()}))
    vo = dev(b.pack("v", {d: w.v_old for d, w in parts.items()}))
    dvh = dev(b.pack("vhat", dvh_parts))
    out = {k: b.alloc(k) for k in KEYS}
    args = (v, vh, vo, out["R_q"], out["R_v"], out["R_vhat"], out["entropy"], out["Ahat"], out["bhat"], dvh,
            out["dv"], out["dq"])
    return out, args


def _graph_replays(b, args, out, ref):
    import torch
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
    del g


def test_mixed_degree_batch():
    import torch
    from paper_2507_22195_amd import mehdg
    from paper_2507_22195_amd.batch import MixedBatch
    p, bc, parts, h, dvh_parts = _setup()
    banner(f"batch: degrees {dict(zip(*np.unique(p, return_counts=True)))}, {int(bc.sum())} wall faces")
    prm = parts[1].params
    b = MixedBatch(p, h, prm, face_bc=bc)
    assert all(b.waves[d] == c for (d, _, c, _) in b.groups)          # nothing streamed
    out, args = _inputs(b, parts, dvh_parts)
    assert sorted(b.order.tolist()) == list(range(p.size)) and np.all(np.diff(p[b.order]) >= 0)

    # FP64 step, then the FP32 mode on the groups of degree <= 3
    b.step(*args)
    torch.cuda.synchronize()
    rc, st = b.status()
    assert rc == 0 and not st.any()
    ref = {k: t.clone() for k, t in out.items()}

    for gi, (d, first, cnt, _) in enumerate(b.groups):
        w = parts[d]
        ctx = mehdg.Context(d, w.mesh.h, prm, face_bc=w.face_bc)
        S = ctx.shapes()
        o = {k: empty(S[k]) for k in KEYS}
        ctx.assemble(dev(w.v), dev(w.vhat), None, dev(w.v_old), o["R_q"], o["R_v"], o["R_vhat"], o["entropy"],
                     want_blocks=True)
        ctx.condense(o["Ahat"], o["bhat"])
        ctx.recover(o["R_q"], dev(dvh_parts[d]), o["dv"], o["dq"])
        torch.cuda.synchronize()
        for k, t in o.items():
            assert torch.equal(b.view(ref[k], k, gi), t), f"degree {d}: {k} differs from a single-degree context"
        ctx.close()
        ws = W.subset(w, [0])
        e = rel_err(host(b.view(ref["Ahat"], "Ahat", gi))[:1],
                    local.condense(ws.p, ws.mesh.h, ws.v, ws.vhat, ws.v_old, ws.params,
                                   face_bc=ws.face_bc)["Ahat"])
        banner(f"  degree {d}: {cnt} macros equal the single-degree context; Ahat vs oracle {e:.1e}")
        assert e < 1e-12
    _graph_replays(b, args, out, ref)
    banner("  graph replays equal the eager batched step")
    b.close()

    # the FP32 mode (degrees 1..3: the mixed-precision modes stop at degree 3)
    keep = p <= 3
    sub = {d: w for d, w in parts.items() if d <= 3}
    b = MixedBatch(p[keep], h[keep], prm, face_bc=bc[keep])
    out, args = _inputs(b, sub, {d: dvh_parts[d] for d in sub})
    b.step(*args, prec="fp32")
    torch.cuda.synchronize()
    rc, st = b.status()
    assert rc == 0 and not st.any()
    for gi, (d, first, cnt, _) in enumerate(b.groups):
        w = parts[d]
        ctx = mehdg.Context(d, w.mesh.h, prm, face_bc=w.face_bc)
        S = ctx.shapes()
        o = {k: empty(S[k]) for k in KEYS}
        ctx.assemble(dev(w.v), dev(w.vhat), None, dev(w.v_old), o["R_q"], o["R_v"], o["R_vhat"], o["entropy"],
                     want_blocks=True)
        ctx.condense(o["Ahat"], o["bhat"], prec="fp32")
        ctx.recover(o["R_q"], dev(dvh_parts[d]), o["dv"], o["dq"])
        torch.cuda.synchronize()
        for k, t in o.items():
            assert torch.equal(b.view(out[k], k, gi), t), f"degree {d}: fp32 {k} differs from a single context"
        ctx.close()
    banner("  fp32 mode equals the single-degree contexts")
    b.close()


def test_streamed_groups_give_the_same_bits():
    import torch
    from paper_2507_22195_amd.batch import MixedBatch
    p, bc, parts, h, dvh_parts = _setup()
    prm = parts[1].params
    full = MixedBatch(p, h, prm, face_bc=bc)
    out, args = _inputs(full, parts, dvh_parts)
    full.step(*args)
    torch.cuda.synchronize()
    ref = {k: t.clone() for k, t in out.items()}
    full.close()
    del out, args

    b = MixedBatch(p, h, prm, face_bc=bc, max_workspace_bytes=1)
    banner(f"streamed batch: waves {b.waves}")
    assert all(b.waves[d] == 1 for (d, _, _, _) in b.groups)
    out, args = _inputs(b, parts, dvh_parts)
    b.step(*args)
    torch.cuda.synchronize()
    rc, st = b.status()
    assert rc == 0 and not st.any()
    for k in out:
        assert torch.equal(out[k], ref[k]), f"streamed batch differs in {k}"
    _graph_replays(b, args, out, ref)
    banner("  one macro per wave: eager and graph replays equal the whole-group batch")
    b.close()
    del out, args

    # one residual launch per degree instead of the persistent one: the same bits
    b = MixedBatch(p, h, prm, face_bc=bc, residual_per_degree=True)
    out, args = _inputs(b, parts, dvh_parts)
    b.step(*args)
    torch.cuda.synchronize()
    rc, st = b.status()
    assert rc == 0 and not st.any()
    for k in out:
        assert torch.equal(out[k], ref[k]), f"per-degree residual launches differ in {k}"
    banner("  per-degree residual launches equal the persistent one")
    b.close()
