"""One Newton step's local work (mehdg_assemble + mehdg_condense + mehdg_recover)
captured in a HIP graph (torch.cuda.CUDAGraph around the library's launches on
the capture stream) and replayed.

Every replay is compared with the eager result on the same inputs, bit for
bit (the same kernels on the same data are deterministic): three replays with
eager library work on other inputs in between, then a replay after the
captured input tensors are overwritten in place with a new state.  The
context's workspaces are allocated by an eager call before the capture, so
the captured calls allocate nothing.
"""
import numpy as np
import pytest

from paper_2507_22195_amd import workloads as W
from tests.gpu_util import banner, dev, empty

pytestmark = pytest.mark.gpu


def test_step_graph_replays_equal_eager():
    import torch
    from paper_2507_22195_amd import mehdg
    w = W.workload(2, shape=(3, 2, 2))
    banner(f"graph: tgv p={w.p} M={w.n_macro}")
    ctx = mehdg.Context(w.p, w.mesh.h, w.params)
    S = ctx.shapes()
    rng = np.random.default_rng(3)
    v, vh, vo = dev(w.v), dev(w.vhat), dev(w.v_old)
    dvh = dev(1e-2 * rng.standard_normal(w.vhat.shape))
    R_q, R_v, R_vh, ent = empty(S["R_q"]), empty(S["R_v"]), empty(S["R_vhat"]), empty(S["entropy"])
    Ahat, bhat, dv, dq = empty(S["Ahat"]), empty(S["bhat"]), empty(S["dv"]), empty(S["dq"])
    outs = (R_v, R_vh, ent, Ahat, bhat, dv, dq)

    def step():
        ctx.assemble(v, vh, None, vo, R_q, R_v, R_vh, ent, want_blocks=True)
        ctx.condense(Ahat, bhat)
        ctx.recover(R_q, dvh, dv, dq)

    def snapshot():
        torch.cuda.synchronize()
        return [t.clone() for t in outs]

    step()
    ref = snapshot()
    # a second state for the in-place update, and its eager result
    v2 = (v + dev(1e-4 * rng.standard_normal(w.v.shape))).contiguous()
    v_keep = v.clone()
    v.copy_(v2)
    step()
    ref2 = snapshot()
    v.copy_(v_keep)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                       # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()

    other = W.workload(2, shape=(3, 2, 2))
    other_v = dev(other.v + 1e-4)
    for rep in range(3):
        g.replay()
        got = snapshot()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), f"replay {rep} differs from the eager step"
        # eager library work on other inputs between replays
        ctx.assemble(other_v, vh, None, vo, R_q, R_v, R_vh, ent, want_blocks=True)
        ctx.condense(Ahat, bhat)
        torch.cuda.synchronize()
    v.copy_(v2)
    g.replay()
    got = snapshot()
    for a, b in zip(got, ref2):
        assert torch.equal(a, b), "replay after an in-place input update differs from the eager step"
    rc, st = ctx.status()
    assert rc == 0
    banner("  4 replays equal the eager steps bit for bit")
    del g
    ctx.close()
