"""Newton + DIRK(3,3) time stepping on the GPU (paper_2507_22195_amd.dirk)
against the oracle's global solve (oracle.global_solve).

* One time step on the advected density wave (p = 1 on 2x2x1 macros, p = 2
  on one macro): the new state and trace equal the oracle's to 1e-9
  relative (both Newton iterations stop at residual ~1e-11; the local
  systems agree to 1e-12 and the trace systems are conditioned ~1e3).
* The whole convergence study of the density wave (tests/golden/
  convergence_wave.txt, written by the oracle) re-run on the GPU: every L2
  error equals the stored one to 1e-6 relative, and the finest pair of
  meshes converges at order p+1 (within 0.3).
"""
import os

import numpy as np
import pytest

from oracle import global_solve
from tests.golden import make_convergence as mc
from tests.gpu_util import banner, dev, host, rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gpu_run(kind, p, N, steps=None):
    from paper_2507_22195_amd.dirk import DirkStepper
    c = mc.setup(kind, p, N)
    st = DirkStepper(p, c["mesh"].h, c["prm"], c["dt"], c["ids"], c["nfaces"])
    v, vh = dev(c["v"]), dev(c["vh_g"])
    for _ in range(c["steps"] if steps is None else steps):
        st.step(v, vh)
    out = host(v), host(vh), st.iterations
    st.close()
    return c, out


@pytest.mark.parametrize("p,N", [(1, 2), (2, 1)])
def test_one_step_matches_oracle(p, N):
    banner(f"dirk: one step, wave p={p} N={N}")
    c, (v, vh, its) = _gpu_run("wave", p, N, steps=1)
    v1, vh1, oits = global_solve.dirk33_step(p, c["mesh"].h, c["ids"], c["nfaces"], c["v"], c["vh_g"],
                                             c["prm"], c["dt"])
    banner(f"dirk: Newton iterations GPU {its[0]}, oracle {oits}")
    assert rel_err(v.reshape(1, -1), v1.reshape(1, -1)) < 1e-9
    assert rel_err(vh.reshape(1, -1), vh1.reshape(1, -1)) < 1e-9


def _table(kind):
    rows = {}
    for ln in open(os.path.join(GOLDEN, f"convergence_{kind}.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        k, p, N, h, e, rate, it = ln.split()
        rows[(int(p), int(N))] = (float(h), float(e))
    return rows


def test_gpu_convergence_matches_stored_table():
    table = _table("wave")
    for p in (1, 2):
        Ns = sorted(N for (pp, N) in table if pp == p)
        errs = []
        for N in Ns:
            c, (v, vh, its) = _gpu_run("wave", p, N)
            e = mc.l2_error("wave", p, c["mesh"], v)
            h, ref = table[(p, N)]
            banner(f"dirk: wave p={p} N={N} GPU error {e:.9e}, oracle {ref:.9e}")
            assert abs(e - ref) <= 1e-6 * ref
            errs.append((h, e))
        (h0, e0), (h1, e1) = errs[-2], errs[-1]
        assert np.log(e0 / e1) / np.log(h0 / h1) > p + 1 - 0.3


def test_stage_source_ignores_stale_memory():
    """The stage source and the work vectors may start from reused allocator
    memory holding NaN: a step from NaN-filled buffers equals a step from a
    fresh stepper bit for bit (mehdg_axpby drops a zero-coefficient term
    without reading its vector)."""
    import torch
    from paper_2507_22195_amd import mehdg
    from paper_2507_22195_amd.dirk import DirkStepper
    banner("dirk: step from NaN-filled work buffers")
    c = mc.setup("wave", 1, 2)
    outs = []
    for poison in (False, True):
        st = DirkStepper(1, c["mesh"].h, c["prm"], c["dt"], c["ids"], c["nfaces"])
        if poison:
            for t in (st.src, st.dV, *st.Rsp):
                t.fill_(float("nan"))
        v, vh = dev(c["v"]), dev(c["vh_g"])
        st.step(v, vh)
        outs.append((host(v), host(vh)))
        st.close()
    assert np.all(np.isfinite(outs[1][0])) and np.all(np.isfinite(outs[1][1]))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    # the kernel itself: a = 0 must not read x, b = 0 must not read y
    x = torch.full((1000,), float("nan"), dtype=torch.float64, device="cuda")
    y = torch.ones(1000, dtype=torch.float64, device="cuda")
    mehdg.axpby(0.0, x, 2.0, y)
    assert torch.equal(y, torch.full_like(y, 2.0))
    y.fill_(float("inf"))
    z = torch.ones(1000, dtype=torch.float64, device="cuda")
    mehdg.axpby(3.0, z, 0.0, y)
    assert torch.equal(y, torch.full_like(y, 3.0))


@pytest.mark.parametrize("ptc", [True, False])
def test_nonlinear_solvers_reach_the_oracles_step(ptc):
    """Inexact Newton with pseudo-transient continuation (Sec. 6.1: tau_init =
    1, tau_max = 1e8, residual-based tau) and exact Newton both converge to the
    oracle's DIRK(3,3) step (a root does not depend on the path); with
    continuation tau grows with the residual's decrease."""
    from paper_2507_22195_amd.dirk import DirkStepper
    c = mc.setup("wave", 1, 2)
    st = DirkStepper(1, c["mesh"].h, c["prm"], c["dt"], c["ids"], c["nfaces"], ptc=ptc)
    v, vh = dev(c["v"]), dev(c["vh_g"])
    st.step(v, vh)
    its, taus = st.iterations[0], st.tau_history
    st.close()
    v1, vh1, oits = global_solve.dirk33_step(1, c["mesh"].h, c["ids"], c["nfaces"], c["v"], c["vh_g"],
                                             c["prm"], c["dt"])
    banner(f"dirk: ptc={ptc} Newton iterations per stage {its} (oracle {oits}); tau {taus}")
    assert rel_err(host(v).reshape(1, -1), v1.reshape(1, -1)) < 1e-9
    assert rel_err(host(vh).reshape(1, -1), vh1.reshape(1, -1)) < 1e-9
    if ptc:
        assert all(t[0] == 1.0 for t in taus)
        assert any(len(t) > 1 and t[-1] > t[0] for t in taus)


def test_gpu_vortex_convergence_matches_stored_table():
    """The advected isentropic vortex (Sec. 7.1.1: strength 2.5, Mach 0.5, 10 %
    of a period) on the GPU reproduces the oracle's stored L2 errors
    (tests/golden/convergence_vortex.txt) and the finest pair converges at
    order p+1 (within 0.3)."""
    table = _table("vortex")
    for p in (1, 2):
        Ns = sorted(N for (pp, N) in table if pp == p)
        errs = []
        for N in Ns:
            c, (v, vh, its) = _gpu_run("vortex", p, N)
            e = mc.l2_error("vortex", p, c["mesh"], v)
            h, ref = table[(p, N)]
            banner(f"dirk: vortex p={p} N={N} GPU error {e:.9e}, oracle {ref:.9e}")
            assert abs(e - ref) <= 1e-6 * ref
            errs.append((h, e))
        (h0, e0), (h1, e1) = errs[-2], errs[-1]
        assert np.log(e0 / e1) / np.log(h0 / h1) > p + 1 - 0.3
