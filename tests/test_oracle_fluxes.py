"""Pins of the oracle's two-point trace fluxes (Sec. 5.1-5.2).

Checked against: the entropy-conservation identity (Thm. 5.1), the
entropy-stability identity (Thm. 5.2), Barth's scaling A0 = R T R^T
(eq. KEPES4) at coincident states, the paper's printed R-bar for n = e_x,
consistency F(v, v) = F(v).n, symmetry, and the plain log-mean formula.
"""
import numpy as np
import pytest

from oracle import ad
from oracle import physics as ph

GAMMA = 1.4
EPS = 1e-4


def states(rng, n, Mmax=1.2):
    rho = rng.uniform(0.4, 2.5, n)
    P = rng.uniform(0.3, 2.5, n)
    c = np.sqrt(GAMMA * P / rho)
    V = rng.uniform(-1, 1, (3, n)) * c * Mmax / np.sqrt(3)
    beta = rho / P
    s = np.log(P / rho ** GAMMA)
    V2 = (V ** 2).sum(0)
    return [(GAMMA - s) / (GAMMA - 1) - beta * V2 / 2, beta * V[0], beta * V[1], beta * V[2], -beta]


def perturb(rng, v, rel):
    """A second state whose primitive variables differ by up to ``rel``."""
    rho, V, P, _ = ph.primitive_from_entropy(v, GAMMA)
    n = rho.size
    rho2 = rho * (1 + rel * rng.uniform(-1, 1, n))
    P2 = P * (1 + rel * rng.uniform(-1, 1, n))
    V2 = [V[i] + rel * rng.uniform(-1, 1, n) for i in range(3)]
    beta = rho2 / P2
    s = np.log(P2 / rho2 ** GAMMA)
    W2 = sum(x * x for x in V2)
    return [(GAMMA - s) / (GAMMA - 1) - beta * W2 / 2, beta * V2[0], beta * V2[1], beta * V2[2], -beta]


NORMALS = [np.array([1.0, 0, 0]), np.array([0, -1.0, 0]), np.array([0, 0, 1.0]),
           np.array([0.48, -0.6, 0.64])]


def entropy_residual(vh, v, F, n):
    return ph.entropy_production_integrand(vh, v, F, n, GAMMA)


def scale(vh, v, F):
    """Magnitude of the terms whose difference forms the entropy production:
    sum |[[v]]_k F_k| plus the round-off floor of [[Psi_n]] (|Psi_n| of both)."""
    Ps = ph.entropy_potential(v, GAMMA)
    Psh = ph.entropy_potential(vh, GAMMA)
    floor = sum(np.abs(Ps[j]) + np.abs(Psh[j]) for j in range(3))
    return sum(np.abs(vh[k] - v[k]) * np.abs(F[k]) for k in range(5)) + floor


@pytest.mark.parametrize("rel", [1e-7, 1e-3, 0.05, 0.3])
def test_ec_flux_conserves_entropy(rel):
    """Thm. 5.1: [[v]]^T Fbar - [[Psi_n]] = 0 for every pair of states,
    including tiny jumps handled by the log-mean series branch."""
    rng = np.random.default_rng(10)
    v = states(rng, 400)
    vh = perturb(rng, v, rel)
    for n in NORMALS:
        F, _ = ph.ec_flux(vh, v, n, GAMMA, EPS)
        r = entropy_residual(vh, v, F, n)
        assert np.max(np.abs(r) / scale(vh, v, F)) < 5e-14


def test_ec_flux_consistent_and_symmetric():
    rng = np.random.default_rng(11)
    v = states(rng, 200)
    vh = perturb(rng, v, 0.2)
    for n in NORMALS:
        F, _ = ph.ec_flux(v, v, n, GAMMA, EPS)
        Fn = ph.normal_flux(ph.inviscid_flux(v, GAMMA), n)
        for k in range(5):
            assert np.allclose(F[k], Fn[k], rtol=1e-13, atol=1e-14)
        A, _ = ph.ec_flux(vh, v, n, GAMMA, EPS)
        B, _ = ph.ec_flux(v, vh, n, GAMMA, EPS)
        for k in range(5):
            assert np.allclose(A[k], B[k], rtol=1e-13, atol=1e-14)


def test_logmean_plain_formula_and_limit():
    rng = np.random.default_rng(12)
    a = rng.uniform(0.5, 2.0, 1000)
    b = a * (1 + rng.uniform(-0.5, 0.5, 1000))
    lm = ph.logmean(a, b, EPS)
    direct = (b - a) / np.log(b / a)
    assert np.allclose(lm, direct, rtol=1e-12)
    # near equality the series branch must agree with an extended-precision
    # evaluation of the plain formula
    b2 = a * (1 + 1e-5 * rng.uniform(-1, 1, 1000))
    lm2 = ph.logmean(a, b2, EPS)
    ref = np.array([float((np.longdouble(y) - np.longdouble(x)) / np.log(np.longdouble(y) / np.longdouble(x)))
                    if x != y else x for x, y in zip(a, b2)])
    assert np.allclose(lm2, ref, rtol=1e-11)
    assert np.allclose(ph.logmean(a, a, EPS), a, rtol=1e-15)


def test_barth_scaling_at_coincident_states():
    """eq. (KEPES4): Rbar Tbar Rbar^T = A0 when vh = v, for any normal."""
    rng = np.random.default_rng(13)
    v = states(rng, 100)
    A0 = ph.entropy_jacobian(v, GAMMA)
    for n in NORMALS:
        _, R, T, _, _ = ph.kepes_parts(v, v, n, GAMMA, EPS)
        Rm = np.stack([np.stack([np.broadcast_to(R[c][k], v[0].shape) for k in range(5)], -1)
                       for c in range(5)], -1)          # [...,k(row),col]
        Tm = np.stack([np.broadcast_to(T[c], v[0].shape) for c in range(5)], -1)
        RTR = np.einsum("...ic,...c,...jc->...ij", Rm, Tm, Rm)
        assert np.max(np.abs(RTR - A0) / np.max(np.abs(A0), axis=(-1, -2), keepdims=True)) < 1e-13


def test_kepes_matches_printed_x_direction_eigenvectors():
    """For n = e_x the general-normal construction must give the same flux as
    the R-bar printed in Sec. 5.1.3 (columns 3, 4 = [0, e_y, v2], [0, e_z, v3])."""
    rng = np.random.default_rng(14)
    v = states(rng, 200)
    vh = perturb(rng, v, 0.2)
    n = np.array([1.0, 0.0, 0.0])
    F, R, T, L, m = ph.kepes_parts(vh, v, n, GAMMA, EPS)
    Vb = m["Vbar"]
    c = np.sqrt(GAMMA * m["P_bar"] / m["rho_ln"])
    hb = GAMMA / (m["beta_ln"] * (GAMMA - 1)) + m["V2_bar"] / 2
    one, zero = np.ones_like(c), np.zeros_like(c)
    printed = [
        [one, Vb[0] - c, Vb[1], Vb[2], hb - Vb[0] * c],
        [one, Vb[0], Vb[1], Vb[2], m["V2_bar"] / 2],
        [zero, zero, one, zero, Vb[1]],
        [zero, zero, zero, one, Vb[2]],
        [one, Vb[0] + c, Vb[1], Vb[2], hb + Vb[0] * c],
    ]
    jump = [vh[k] - v[k] for k in range(5)]
    ref = list(F)
    for col in range(5):
        proj = sum(printed[col][k] * jump[k] for k in range(5))
        for k in range(5):
            ref[k] = ref[k] - 0.5 * printed[col][k] * L[col] * T[col] * proj
    got = ph.kepes_flux(vh, v, n, GAMMA, EPS)
    for k in range(5):
        assert np.allclose(got[k], ref[k], rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("rel", [1e-3, 0.1, 0.4])
def test_kepes_entropy_production_is_quadratic_form(rel):
    """Thm. 5.2: [[v]]^T F - [[Psi_n]] = -1/2 sum_k |Lambda|_k T_k (r_k.[[v]])^2 <= 0."""
    rng = np.random.default_rng(15)
    v = states(rng, 400)
    vh = perturb(rng, v, rel)
    for n in NORMALS:
        F = ph.kepes_flux(vh, v, n, GAMMA, EPS)
        _, R, T, L, _ = ph.kepes_parts(vh, v, n, GAMMA, EPS)
        jump = [vh[k] - v[k] for k in range(5)]
        quad = 0.0
        for col in range(5):
            proj = sum(R[col][k] * jump[k] for k in range(5))
            quad = quad - 0.5 * L[col] * T[col] * proj * proj
        r = entropy_residual(vh, v, F, n)
        assert np.max(np.abs(r - quad) / scale(vh, v, F)) < 5e-14
        assert np.all(quad <= 0)
        for col in range(5):
            assert np.all(np.asarray(L[col]) >= 0) and np.all(np.asarray(T[col]) > 0)


def test_kepes_and_es_consistent():
    rng = np.random.default_rng(16)
    v = states(rng, 200)
    for n in NORMALS:
        Fn = ph.normal_flux(ph.inviscid_flux(v, GAMMA), n)
        K = ph.kepes_flux(v, v, n, GAMMA, EPS)
        E = ph.es_flux(v, v, n, GAMMA)
        for k in range(5):
            assert np.allclose(K[k], Fn[k], rtol=1e-13, atol=1e-14)
            assert np.allclose(E[k], Fn[k], rtol=1e-13, atol=1e-14)


def test_es_flux_dissipation_sign_small_jumps():
    """Eq. (Flux_En_Inv): the central average is entropy-conservative only up
    to O(|[[v]]|^3); the -1/2 sigma A0 [[v]] term is O(|[[v]]|^2) and
    dissipative, so small jumps produce entropy <= 0."""
    rng = np.random.default_rng(17)
    v = states(rng, 400)
    vh = perturb(rng, v, 1e-3)
    for n in NORMALS:
        F = ph.es_flux(vh, v, n, GAMMA)
        r = entropy_residual(vh, v, F, n)
        assert np.all(r <= 1e-16)


def test_trace_flux_jacobians_match_fd():
    """Dual-number Jacobians of the three trace fluxes vs fourth-order central
    FD.  Points within 1e-2 of the sqrt|x| kink of theta (P = P_hat) are
    skipped; their number is asserted small."""
    rng = np.random.default_rng(18)
    v = states(rng, 60)
    vh = perturb(rng, v, 0.05)
    rho, _, P, _ = ph.primitive_from_entropy(v, GAMMA)
    rhoh, _, Ph, _ = ph.primitive_from_entropy(vh, GAMMA)
    keep = np.abs(P - Ph) / (P + Ph) > 1e-2
    assert keep.sum() > 30
    prm = dict(gamma=GAMMA, logmean_eps=EPS)

    def flux(a, b, n):
        return np.stack(ph.inviscid_trace_flux(a, b, n, prm), -1)

    for fl in (0, 1, 2):
        prm["flux"] = fl
        for n in NORMALS[:2] + NORMALS[3:]:
            vhd = ad.seed(vh, 10, 0)
            vd = ad.seed(v, 10, 5)
            J = ad.jac(ph.inviscid_trace_flux(vhd, vd, n, prm))
            h = 1e-5
            for l in range(10):
                cols = []
                for step in (2 * h, h, -h, -2 * h):
                    a = [x.copy() for x in vh]
                    b = [x.copy() for x in v]
                    if l < 5:
                        a[l] = a[l] + step
                    else:
                        b[l - 5] = b[l - 5] + step
                    cols.append(flux(a, b, n))
                col = (-cols[0] + 8 * cols[1] - 8 * cols[2] + cols[3]) / (12 * h)
                err = np.abs(col - J[..., :, l]) / (np.abs(J[..., :, l]) + 1e-3)
                assert np.max(err[keep]) < 1e-6, (fl, l, np.max(err[keep]))


def _kepes_by_hand_x(rhoL, VL, PL, rhoR, VR, PR):
    """KEPES flux for n = e_x written out from Sec. 5.1.3 on primitive states:
    the EC flux (eq. EC), R-bar as printed, T-bar (eq. KEPES4), lambda^KEPES,
    theta and lambda_max, assembled as Fbar - 1/2 R |Lambda| T R^T [[v]]
    (eq. ES).  L is the element side (v), R the trace side (v-hat); the jump
    is trace minus element.  Returns the flux and its pieces so that the
    caller can plant a misreading into one of them."""
    g = GAMMA

    def entropy_vars(rho, V, P):
        beta = rho / P
        s = np.log(P / rho ** g)
        return np.array([(g - s) / (g - 1) - beta * (V @ V) / 2, *(beta * V), -beta])

    def lnmean(a, b):
        return (b - a) / np.log1p((b - a) / a)

    betaL, betaR = rhoL / PL, rhoR / PR
    rho_ln, beta_ln = lnmean(rhoL, rhoR), lnmean(betaL, betaR)
    Vb = (VL + VR) / 2
    V2b = (VL @ VL + VR @ VR) / 2
    Pb = ((rhoL + rhoR) / 2) / ((betaL + betaR) / 2)
    f1 = rho_ln * Vb[0]
    f2 = Vb * f1 + Pb * np.array([1.0, 0.0, 0.0])
    f3 = (1 / (beta_ln * (g - 1)) - V2b / 2) * f1 + Vb @ f2
    Fec = np.array([f1, *f2, f3])
    c = np.sqrt(g * Pb / rho_ln)
    h = g / (beta_ln * (g - 1)) + V2b / 2
    Rm = np.array([[1, 1, 0, 0, 1],
                   [Vb[0] - c, Vb[0], 0, 0, Vb[0] + c],
                   [Vb[1], Vb[1], 1, 0, Vb[1]],
                   [Vb[2], Vb[2], 0, 1, Vb[2]],
                   [h - Vb[0] * c, V2b / 2, Vb[1], Vb[2], h + Vb[0] * c]])
    parts = dict(Fec=Fec, R=Rm, rho_ln=rho_ln, rho_bar=(rhoL + rhoR) / 2, Pb=Pb, vn=Vb[0], c=c,
                 ratio=abs((PL - PR) / (PL + PR)),
                 jump=entropy_vars(rhoR, VR, PR) - entropy_vars(rhoL, VL, PL))
    return parts


def _kepes_assemble(parts, lam1_sign=1.0, theta_sqrt=True, T_rho="ln"):
    g = GAMMA
    r = parts["rho_ln"] if T_rho == "ln" else parts["rho_bar"]
    T = np.array([r / (2 * g), r * (g - 1) / g, parts["Pb"], parts["Pb"], r / (2 * g)])
    vn, c = parts["vn"], parts["c"]
    lam = np.array([vn + lam1_sign * c, vn, vn, vn, vn + c])
    lmax = abs(vn) + c
    theta = np.sqrt(parts["ratio"]) if theta_sqrt else parts["ratio"]
    L = (1 - theta) * np.abs(lam) + theta * lmax
    R = parts["R"]
    return parts["Fec"] - 0.5 * R @ (L * T * (R.T @ parts["jump"]))


@pytest.mark.parametrize("rel", [1e-3, 0.05, 0.2, 0.4])
def test_kepes_flux_against_hand_evaluation_at_distinct_states(rel):
    """Sec. 5.1.3, eq. (KEPES3)-(KEPES5), (ES), n = e_x: the oracle's KEPES flux
    equals a by-hand evaluation of the printed T-bar, lambda^KEPES (mass and
    energy waves both v_n + c), lambda_max = |v_n| + c and
    theta = sqrt|(P - P_hat)/(P + P_hat)| at distinct states.  The same
    evaluation with lambda_1 = v_n - c, with theta lacking its square root, or
    with the arithmetic mean of rho in T-bar must differ from the oracle by far
    more than the tolerance, so that each of those misreadings fails here."""
    rng = np.random.default_rng(101)
    n = np.array([1.0, 0.0, 0.0])
    worst = 0.0
    gaps = dict(lam1=np.inf, theta=np.inf, Trho=np.inf)
    for _ in range(60):
        rhoL, PL = rng.uniform(0.5, 2.0), rng.uniform(0.4, 2.0)
        cL = np.sqrt(GAMMA * PL / rhoL)
        VL = rng.uniform(-0.6, 0.6, 3) * cL
        VL[0] = np.sign(VL[0]) * max(abs(VL[0]), 0.2 * cL)   # keep v_n away from 0
        rhoR = rhoL * (1 + rel * rng.choice([-1, 1]) * rng.uniform(0.5, 1))
        PR = PL * (1 + rel * rng.choice([-1, 1]) * rng.uniform(0.5, 1))
        VR = VL + rel * rng.uniform(-1, 1, 3) * cL
        parts = _kepes_by_hand_x(rhoL, VL, PL, rhoR, VR, PR)
        ref = _kepes_assemble(parts)
        v = states_from_primitive(rhoL, VL, PL)
        vh = states_from_primitive(rhoR, VR, PR)
        got = np.array([float(x) for x in ph.kepes_flux(vh, v, n, GAMMA, EPS)])
        scale_f = np.abs(ref).max()
        worst = max(worst, np.abs(got - ref).max() / scale_f)
        for key, alt in (("lam1", _kepes_assemble(parts, lam1_sign=-1.0)),
                         ("theta", _kepes_assemble(parts, theta_sqrt=False)),
                         ("Trho", _kepes_assemble(parts, T_rho="bar"))):
            gaps[key] = min(gaps[key], np.abs(alt - got).max() / scale_f)
    assert worst < 1e-12, worst
    # Every misreading moves the flux of every sample by many times the
    # tolerance: the dissipation is O(jump^2) (O(jump^1.5) through theta), and
    # rho-bar differs from rho^ln at second order in the jump, so that
    # misreading shows only at the larger jumps.
    assert gaps["lam1"] > 1e3 * 1e-12 and gaps["theta"] > 1e3 * 1e-12, gaps
    if rel >= 0.05:
        assert gaps["Trho"] > 1e3 * 1e-12, gaps


def states_from_primitive(rho, V, P):
    beta = rho / P
    s = np.log(P / rho ** GAMMA)
    return [np.array((GAMMA - s) / (GAMMA - 1) - beta * (V @ V) / 2), np.array(beta * V[0]),
            np.array(beta * V[1]), np.array(beta * V[2]), np.array(-beta)]
