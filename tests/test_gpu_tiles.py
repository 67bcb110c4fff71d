"""Tile variants of the batched FP64 products (mehdg_set_tile).

Every tile shape adds the products of one output element in the same order,
so on a p = 2 and a p = 3 Taylor-Green batch (several tiles per macro, a
ragged last tile) every variant at either call site gives Ahat, bhat, dV
and dQ bit for bit equal to variant 0's; variant 0 is compared with the
oracle on one macro (1e-12).
"""
import numpy as np
import pytest

from oracle import local
from paper_2507_22195_amd import workloads as W
from tests.gpu_util import banner, dev, empty, host, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p,shape", [(2, (3, 2, 2)), (3, (2, 2, 1))])
def test_every_tile_variant_gives_the_same_bits(p, shape):
    import torch
    from paper_2507_22195_amd import mehdg
    w = W.tgv_workload(shape=shape, p=p, M0=0.1, Re=1600.0, flux="ES", seed_v=21, seed_vh=22)
    variants = mehdg.tile_variants()
    ctx = mehdg.Context(p, w.mesh.h, w.params)
    S = ctx.shapes()
    banner(f"tiles: p={p} M={ctx.n_macro} variants={len(variants)} "
           f"table: update {ctx.get_tile('update')} schur {ctx.get_tile('schur')}")
    dvhat = dev(1e-2 * np.random.default_rng(3).standard_normal(S["vhat"]))

    def step():
        o = {k: empty(S[k]) for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
        ctx.assemble(dev(w.v), dev(w.vhat), None, dev(w.v_old), o["R_q"], o["R_v"], o["R_vhat"], o["entropy"],
                     want_blocks=True)
        ctx.condense(o["Ahat"], o["bhat"])
        ctx.recover(o["R_q"], dvhat, o["dv"], o["dq"])
        torch.cuda.synchronize()
        rc, st = ctx.status()
        assert rc == 0 and not st.any()
        return {k: o[k] for k in ("Ahat", "bhat", "dv", "dq")}

    ctx.set_tile("update", 0)
    ctx.set_tile("schur", 0)
    ref = step()
    ws = W.subset(w, [0])
    e = rel_err(host(ref["Ahat"][:1]), local.condense(ws.p, ws.mesh.h, ws.v, ws.vhat, ws.v_old, ws.params)["Ahat"])
    assert e < 1e-12, e
    for site in ("update", "schur"):
        for i, v in enumerate(variants):
            ctx.set_tile(site, i)
            got = step()
            for k in ref:
                assert torch.equal(got[k], ref[k]), f"{site} variant {i} ({v['TM']}x{v['TN']}): {k} differs"
        ctx.set_tile(site, 0)
    banner(f"  every variant at both sites equals variant 0; Ahat vs oracle {e:.1e}")
    ctx.set_tile("update", -1)
    ctx.set_tile("schur", -1)
    ctx.close()
