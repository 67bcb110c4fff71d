"""Stored factors applied to new right-hand sides (mehdg_condense_rhs) and the
Jacobian-free Newton-Krylov stepper (paper_2507_22195_amd.jfnk).

* condense_rhs with the assembled (r_V, r_hat) reproduces the condensation's
  own bhat and y (the right-hand-side column of the factors) to 1e-13;
  with random right-hand sides, bhat = r_hat - X S^-1 r_V and the recovered
  dV = S^-1 (r_V + Y dVhat) equal the oracle's to 1e-12 (per macro, normwise);
* one DIRK(3,3) step by JFNK (residual JVP as the Krylov operator, the
  stage's first assembled Newton solve as lagged preconditioner) equals the
  assembled Newton's step to 1e-9, and the first Newton iteration of every
  stage takes one or two Krylov iterations (the preconditioner is exact there);
* the p = 1 density-wave convergence study through JFNK reproduces the
  oracle's stored L2 errors to 1e-6 relative.
"""
import os

import numpy as np
import pytest

from oracle import local
from paper_2507_22195_amd import workloads as W
from tests.golden import make_convergence as mc
from tests.gpu_util import banner, dev, empty, host, rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name", ["tgv viscous ES p2", "vortex EC p2", "tgv viscous ES p3"])
def test_condense_rhs(name):
    from paper_2507_22195_amd import mehdg
    w = {"tgv viscous ES p2": lambda: W.subset(W.workload(2, shape=(4, 4, 4)), [0, 21, 40]),
         "vortex EC p2": lambda: W.subset(W.workload(1), [0, 5]),
         "tgv viscous ES p3": lambda: W.subset(W.tgv_workload(shape=(2, 1, 1), p=3, M0=0.3, Re=5000.0, flux="ES",
                                                              seed_v=51, seed_vh=52), [0, 1])}[name]()
    banner(f"condense_rhs: {name} M={w.n_macro}")
    ctx = mehdg.Context(w.p, w.mesh.h, w.params)
    S = ctx.shapes()
    NV, NH = ctx.sz["N_V"], ctx.sz["N_VH"]
    R_q, R_v, R_vh, ent = empty(S["R_q"]), empty(S["R_v"]), empty(S["R_vhat"]), empty(S["entropy"])
    ctx.assemble(dev(w.v), dev(w.vhat), None, dev(w.v_old), R_q, R_v, R_vh, ent, want_blocks=True)
    B0 = [ctx.bordered(m) for m in range(w.n_macro)]
    r_v = np.stack([b[:NV, NV + NH] for b in B0])
    r_h = np.stack([b[NV:NV + NH, NV + NH] for b in B0])
    Ahat, bhat0, bhat1 = empty(S["Ahat"]), empty(S["bhat"]), empty(S["bhat"])
    ctx.condense(Ahat, bhat0)
    y0 = np.stack([ctx.bordered(m)[:NV, NV + NH] for m in range(w.n_macro)])
    ctx.condense_rhs(dev(r_v.reshape(S["v"])), dev(r_h), bhat1)
    y1 = np.stack([ctx.bordered(m)[:NV, NV + NH] for m in range(w.n_macro)])
    e_same = (rel_err(host(bhat1), host(bhat0)), rel_err(y1, y0))
    banner(f"  assembled rhs: bhat {e_same[0]:.1e} y {e_same[1]:.1e}")
    assert max(e_same) < 1e-13

    rng = np.random.default_rng(6)
    a = rng.standard_normal((w.n_macro, NV))
    c = rng.standard_normal((w.n_macro, NH))
    dvh = rng.standard_normal(w.vhat.shape)
    ctx.condense_rhs(dev(a.reshape(S["v"])), dev(c), bhat1)
    dv, dq = empty(S["dv"]), empty(S["dq"])
    ctx.recover(dev(np.zeros(S["R_q"])), dev(dvh), dv, dq)
    ref = local.condense(w.p, w.mesh.h, w.v, w.vhat, w.v_old, w.params)
    rb = np.stack([c[m] - ref["X"][m] @ np.linalg.solve(ref["S"][m], a[m]) for m in range(w.n_macro)])
    rdv = np.stack([np.linalg.solve(ref["S"][m], a[m] + ref["Y"][m] @ dvh[m].ravel()) for m in range(w.n_macro)])
    e_new = (rel_err(host(bhat1), rb), rel_err(host(dv), rdv))
    banner(f"  random rhs: bhat {e_new[0]:.1e} dV {e_new[1]:.1e}")
    assert max(e_new) < 1e-12
    rc, st = ctx.status()
    assert rc == 0
    ctx.close()


def _step(cls, kind, p, N, steps=1, **kw):
    c = mc.setup(kind, p, N)
    st = cls(p, c["mesh"].h, c["prm"], c["dt"], c["ids"], c["nfaces"], **kw)
    v, vh = dev(c["v"]), dev(c["vh_g"])
    for _ in range(steps if steps is not None else c["steps"]):
        st.step(v, vh)
    out = host(v), host(vh), st
    st.close()
    return c, out


@pytest.mark.parametrize("p,N", [(1, 2), (2, 1)])
def test_jfnk_step_matches_assembled_newton(p, N):
    from paper_2507_22195_amd.dirk import DirkStepper
    from paper_2507_22195_amd.jfnk import JfnkStepper
    banner(f"jfnk: one step, wave p={p} N={N}")
    _, (va, vha, sa) = _step(DirkStepper, "wave", p, N)
    _, (vj, vhj, sj) = _step(JfnkStepper, "wave", p, N)
    banner(f"  Newton iterations assembled {sa.iterations}, JFNK {sj.iterations}; Krylov per Newton {sj.krylov}")
    assert rel_err(vj.reshape(1, -1), va.reshape(1, -1)) < 1e-9
    assert rel_err(vhj.reshape(1, -1), vha.reshape(1, -1)) < 1e-9
    for kry in sj.krylov:
        assert len(kry) >= 1 and kry[0] <= 2, sj.krylov


def test_jfnk_convergence_matches_stored_table():
    from paper_2507_22195_amd.jfnk import JfnkStepper
    rows = {}
    for ln in open(os.path.join(GOLDEN, "convergence_wave.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        k, pp, N, h, e, rate, it = ln.split()
        rows[(int(pp), int(N))] = float(e)
    for N in sorted(N for (pp, N) in rows if pp == 1):
        c, (v, vh, st) = _step(JfnkStepper, "wave", 1, N, steps=None)
        e = mc.l2_error("wave", 1, c["mesh"], v)
        banner(f"jfnk: wave p=1 N={N} GPU error {e:.9e}, oracle {rows[(1, N)]:.9e}")
        assert abs(e - rows[(1, N)]) <= 1e-6 * rows[(1, N)]
