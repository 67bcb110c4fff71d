"""Pins of the oracle's global trace solve and time stepping, and the p+1
convergence of its discrete solution (Sec. 7.1: optimal order p+1).

* DIRK(3,3) coefficients: the order-3 conditions and L-stability (stiffly
  accurate, R(inf) = 0) -- what makes the stage form of the time term right.
* Free stream: a uniform state stays uniform to round-off through a full
  DIRK step with Newton and the global trace solve.
* Convergence: the stored tables (tests/golden/convergence_*.txt, written
  by tests/golden/make_convergence.py, which calls only the oracle and the
  closed-form fields) show L2 rates of p+1 within 0.3 on the finest pair
  of meshes, for a smooth advected density wave and for the advected
  isentropic vortex of Sec. 7.1 (on the coarsest vortex meshes, 2 and 4
  sub-elements across the core, the rate is not yet asymptotic); the
  coarsest stored wave case is recomputed here and must agree, so the
  tables belong to the current oracle.
"""
import os

import numpy as np
import pytest

from oracle import global_solve, local
from paper_2507_22195_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_dirk33_order_conditions_and_l_stability():
    A = global_solve.dirk33_tableau()
    b = A[2]
    c = A.sum(axis=1)
    assert np.allclose(np.triu(A, 1), 0.0)
    assert abs(b.sum() - 1.0) < 1e-14
    assert abs(b @ c - 0.5) < 1e-14
    assert abs(b @ c ** 2 - 1.0 / 3.0) < 1e-14
    assert abs(b @ A @ c - 1.0 / 6.0) < 1e-14
    # stiffly accurate, so R(inf) = 1 - b^T A^-1 1 = 0 (L-stable)
    assert abs(1.0 - b @ np.linalg.solve(A, np.ones(3))) < 1e-13
    assert abs(c[2] - 1.0) < 1e-14


def test_free_stream_is_preserved_by_a_global_step():
    mesh = W.box_mesh((2, 1, 1), (0.0, 0.0, 0.0), (2.0, 1.0, 1.0))
    p, gamma = 1, 1.4
    prm = W.make_params(gamma=gamma, flux="ES", dt=1.0, alpha_ps=0.0)
    rho, V, P = 1.2, np.array([0.3, -0.2, 0.1]), 0.9
    xn = W.node_coords(mesh, p)
    shape = xn[:, 0, :].shape
    v = W.entropy_variables(np.full(shape, rho), np.broadcast_to(V[None, :, None], (shape[0], 3, shape[1])),
                            np.full(shape, P), gamma)
    ids, nfaces = global_solve.periodic_face_ids(mesh.shape, mesh.ijk)
    nf = (2 * p + 1) ** 2
    vh_g = np.broadcast_to(v[0, :, :1], (nfaces, 5, nf)).copy()
    v1, vh1, its = global_solve.dirk33_step(p, mesh.h, ids, nfaces, v, vh_g, prm, 0.1)
    assert np.abs(v1 - v).max() < 1e-12
    assert np.abs(vh1 - vh_g).max() < 1e-12
    assert max(its) <= 1


def _table(kind):
    path = os.path.join(GOLDEN, f"convergence_{kind}.txt")
    rows = []
    for ln in open(path):
        if ln.startswith("#") or not ln.strip():
            continue
        k, p, N, h, e, rate, it = ln.split()
        rows.append((int(p), int(N), float(h), float(e), float(rate), int(it)))
    return rows


@pytest.mark.parametrize("kind", ["wave", "vortex"])
def test_stored_rates_are_p_plus_one(kind):
    rows = _table(kind)
    for p in sorted({r[0] for r in rows}):
        rp = sorted([r for r in rows if r[0] == p], key=lambda r: r[1])
        assert len(rp) >= 2
        h0, e0, h1, e1 = rp[-2][2], rp[-2][3], rp[-1][2], rp[-1][3]
        rate = np.log(e0 / e1) / np.log(h0 / h1)
        assert rate > p + 1 - 0.3, (kind, p, rate)


def test_coarsest_stored_case_reproduces():
    from tests.golden import make_convergence as mc
    row = [r for r in _table("wave") if r[0] == 1][0]
    h, err, its = mc.run("wave", 1, row[1])
    assert abs(h - row[2]) < 1e-15
    assert abs(err - row[3]) <= 1e-9 * row[3], (err, row[3])
