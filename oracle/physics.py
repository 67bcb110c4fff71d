"""Pointwise physics of the entropy-variable formulation (oracle, FP64).

Oracle test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import this package.

Every function takes states as lists of component arrays (float arrays or
``ad.Dual``), so the same code gives values and exact pointwise Jacobians.
Acoustic scaling throughout: rho0 = 1, c0 = 1, P0 = 1/gamma, gamma P = rho T.
"""
from __future__ import annotations

import numpy as np

from . import ad
from .ad import exp, log, sqrt, absval, sqrt_abs, where


# --------------------------------------------------------------------------
# thermodynamics (Sec. 2.1 closure, Sec. 2.2 eq. s222)
# --------------------------------------------------------------------------
def primitive_from_entropy(v, gamma):
    """(rho, [V1,V2,V3], P, beta) from entropy variables.

    Inverts eq. (s222): beta = -v5, V = (v2,v3,v4)/beta,
    s = gamma - (gamma-1)(v1 + beta|V|^2/2), and P/rho^gamma = e^s with
    P = rho/beta gives rho = exp(-(s + ln beta)/(gamma-1)).
    """
    beta = -v[4]
    V = [v[1] / beta, v[2] / beta, v[3] / beta]
    V2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2]
    s = gamma - (gamma - 1.0) * (v[0] + beta * V2 / 2.0)
    rho = exp(-(s + log(beta)) / (gamma - 1.0))
    P = rho / beta
    return rho, V, P, beta


def conservative_from_entropy(v, gamma):
    """u(v) = (rho, rho V, rho E), E = P/((gamma-1) rho) + |V|^2/2 (Sec. 2.1)."""
    rho, V, P, _ = primitive_from_entropy(v, gamma)
    V2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2]
    return [rho, rho * V[0], rho * V[1], rho * V[2], P / (gamma - 1.0) + rho * V2 / 2.0]


def entropy_from_conservative(u, gamma):
    """v(u) of eq. (s222) written from conservative variables."""
    rho = u[0]
    V = [u[1] / rho, u[2] / rho, u[3] / rho]
    V2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2]
    P = (gamma - 1.0) * (u[4] - rho * V2 / 2.0)
    beta = rho / P
    s = log(P) - gamma * log(rho)
    return [(gamma - s) / (gamma - 1.0) - beta * V2 / 2.0,
            beta * V[0], beta * V[1], beta * V[2], -beta]


def entropy_density(u, gamma):
    """H = -rho s/(gamma-1), s = log(P/rho^gamma) (eq. en)."""
    rho = u[0]
    V2 = (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / (rho * rho)
    P = (gamma - 1.0) * (u[4] - rho * V2 / 2.0)
    s = log(P) - gamma * log(rho)
    return -rho * s / (gamma - 1.0)


def entropy_flux(v, gamma):
    """Entropy flux H V (components j = 1..3).

    The paper prints -rho s V; with H = -rho s/(gamma-1) only H V satisfies the
    potential relation Psi_j = F_j^T v - (entropy flux)_j = rho V_j of
    eq. (poen), so that is the reading taken here.
    """
    u = conservative_from_entropy(v, gamma)
    H = entropy_density(u, gamma)
    rho = u[0]
    return [H * u[1] / rho, H * u[2] / rho, H * u[3] / rho]


def entropy_potential(v, gamma):
    """Psi_j = rho V_j, eq. (poen)."""
    rho, V, _, _ = primitive_from_entropy(v, gamma)
    return [rho * V[0], rho * V[1], rho * V[2]]


# --------------------------------------------------------------------------
# fluxes (Sec. 2.1 eq. C5, C6)
# --------------------------------------------------------------------------
def inviscid_flux(v, gamma):
    """F_j(u(v)) = [rho V_j, rho V_j V + P e_j, V_j (rho E + P)], j = 0..2.

    Returns F[j][k] (direction j, component k).
    """
    rho, V, P, _ = primitive_from_entropy(v, gamma)
    V2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2]
    rhoE = P / (gamma - 1.0) + rho * V2 / 2.0
    F = []
    for j in range(3):
        m = rho * V[j]
        F.append([m,
                  m * V[0] + (P if j == 0 else 0.0),
                  m * V[1] + (P if j == 1 else 0.0),
                  m * V[2] + (P if j == 2 else 0.0),
                  V[j] * (rhoE + P)])
    return F


def viscous_flux(v, q, prm):
    """G_j(v, q) of eq. (C5)-(C6) with q the gradient of the entropy variables.

    q[l][j] = d v_l / d x_j.  The velocity and temperature gradients follow
    by the chain rule from V_i = -v_{i+1}/v_5 and T = -gamma/v_5:
        d_j V_i = -(q_{i+1,j} + V_i q_{5,j}) / v_5,  d_j T = gamma q_{5,j} / v_5^2.
    tau = mu (grad V + grad V^T + lam (div V) I), phi = -kappa grad T,
    G_j = -[0, tau_{.j}, (tau V)_j - phi_j].  Returns G[j][k].
    """
    gamma, mu, kappa, lam = prm["gamma"], prm["mu"], prm["kappa"], prm["lam"]
    v5 = v[4]
    V = [-v[1] / v5, -v[2] / v5, -v[3] / v5]
    dV = [[-(q[i + 1][j] + V[i] * q[4][j]) / v5 for j in range(3)] for i in range(3)]
    dT = [gamma * q[4][j] / (v5 * v5) for j in range(3)]
    div = dV[0][0] + dV[1][1] + dV[2][2]
    tau = [[mu * (dV[i][j] + dV[j][i] + (lam * div if i == j else 0.0)) for j in range(3)]
           for i in range(3)]
    G = []
    for j in range(3):
        tV = tau[j][0] * V[0] + tau[j][1] * V[1] + tau[j][2] * V[2]
        phi = -kappa * dT[j]
        G.append([0.0 * v5, -tau[0][j], -tau[1][j], -tau[2][j], -(tV - phi)])
    return G


def normal_flux(Fj, n):
    """sum_j F_j n_j for constant normal n = (n0, n1, n2)."""
    out = []
    for k in range(5):
        acc = None
        for j in range(3):
            if n[j] == 0.0:
                continue
            t = Fj[j][k] * n[j]
            acc = t if acc is None else acc + t
        out.append(acc if acc is not None else 0.0 * Fj[0][k])
    return out


def entropy_jacobian(v, gamma):
    """A0 = du/dv in closed form (used only as an independent pin)."""
    rho, V, P, _ = primitive_from_entropy(v, gamma)
    V2 = V[0] ** 2 + V[1] ** 2 + V[2] ** 2
    E = P / ((gamma - 1.0) * rho) + V2 / 2.0
    H = E + P / rho
    c2 = gamma * P / rho
    A = np.empty(np.shape(rho) + (5, 5))
    A[..., 0, 0] = rho
    for i in range(3):
        A[..., 0, 1 + i] = A[..., 1 + i, 0] = rho * V[i]
        A[..., 4, 1 + i] = A[..., 1 + i, 4] = rho * H * V[i]
        for j in range(3):
            A[..., 1 + i, 1 + j] = rho * V[i] * V[j] + (P if i == j else 0.0)
    A[..., 0, 4] = A[..., 4, 0] = rho * E
    A[..., 4, 4] = rho * H * H - c2 * P / (gamma - 1.0)
    return A


# --------------------------------------------------------------------------
# two-point fluxes against the trace (Sec. 5.1)
# --------------------------------------------------------------------------
def logmean(a, ah, eps):
    """Logarithmic mean (a_hat - a)/ln(a_hat/a), eq. (avg).

    Near a = a_hat it uses the Ismail-Roe series: with f = (a-a_hat)/(a+a_hat)
    and w = f^2, ln(a/a_hat)/(2f) = 1 + w/3 + w^2/5 + w^3/7 + ..., and the mean
    is (a + a_hat) / (2 * that).  The series is used for w < eps.
    """
    f = (a - ah) / (a + ah)
    w = f * f
    series = 1.0 + w / 3.0 + w * w / 5.0 + w * w * w / 7.0
    wv = ad.value(w)
    small = wv < eps
    fv = ad.value(f)
    # keep the unused branch finite
    safe_f = where(small, 0.0 * f + 1.0, f)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = where(small, 0.0 * a + 1.0, a / ah)
        logbr = log(ratio) / (2.0 * safe_f)
    del fv
    F = where(small, series, logbr)
    return (a + ah) / (2.0 * F)


def _means(vh, v, gamma, eps):
    rho, V, P, beta = primitive_from_entropy(v, gamma)
    rhoh, Vh, Ph, betah = primitive_from_entropy(vh, gamma)
    m = dict(rho=rho, V=V, P=P, beta=beta, rhoh=rhoh, Vh=Vh, Ph=Ph, betah=betah)
    m["rho_ln"] = logmean(rho, rhoh, eps)
    m["beta_ln"] = logmean(beta, betah, eps)
    m["Vbar"] = [(V[i] + Vh[i]) / 2.0 for i in range(3)]
    m["rho_bar"] = (rho + rhoh) / 2.0
    m["beta_bar"] = (beta + betah) / 2.0
    m["P_bar"] = m["rho_bar"] / m["beta_bar"]
    m["V2_bar"] = ((V[0] ** 2 + V[1] ** 2 + V[2] ** 2) + (Vh[0] ** 2 + Vh[1] ** 2 + Vh[2] ** 2)) / 2.0
    return m


def ec_flux(vh, v, n, gamma, eps):
    """Entropy-conservative, kinetic-energy-preserving flux, eq. (EC):
    f1 = rho_ln Vbar.n, f2 = Vbar f1 + Pbar n, f3 = (1/(beta_ln(gamma-1)) - avg(|V|^2)/2) f1 + Vbar.f2,
    with Pbar = avg(rho)/avg(beta)."""
    m = _means(vh, v, gamma, eps)
    Vb = m["Vbar"]
    Vn = Vb[0] * n[0] + Vb[1] * n[1] + Vb[2] * n[2]
    f1 = m["rho_ln"] * Vn
    f2 = [Vb[i] * f1 + m["P_bar"] * n[i] for i in range(3)]
    f3 = (1.0 / (m["beta_ln"] * (gamma - 1.0)) - m["V2_bar"] / 2.0) * f1 \
        + Vb[0] * f2[0] + Vb[1] * f2[1] + Vb[2] * f2[2]
    return [f1, f2[0], f2[1], f2[2], f3], m


def es_flux(vh, v, n, gamma):
    """Entropy-stable flux, eq. (Flux_En_Inv):
    1/2 (F(vh) + F(v)).n - 1/2 sigma(vh) A0(vh) [[v]], [[v]] = vh - v,
    sigma = |Vh.n| + c_hat (largest characteristic speed at the trace)."""
    Fn = normal_flux(inviscid_flux(v, gamma), n)
    Fnh = normal_flux(inviscid_flux(vh, gamma), n)
    rhoh, Vh, Ph, _ = primitive_from_entropy(vh, gamma)
    sigma = absval(Vh[0] * n[0] + Vh[1] * n[1] + Vh[2] * n[2]) + sqrt(gamma * Ph / rhoh)
    # A0(vh) [[v]] as the directional derivative of u at vh along [[v]]
    jump = [vh[k] - v[k] for k in range(5)]
    A0j = _a0_times(vh, jump, gamma)
    return [0.5 * (Fnh[k] + Fn[k]) - 0.5 * sigma * A0j[k] for k in range(5)]


def _a0_times(vh, w, gamma):
    """A0(vh) w with A0 written out from its closed form."""
    rho, V, P, _ = primitive_from_entropy(vh, gamma)
    V2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2]
    E = P / ((gamma - 1.0) * rho) + V2 / 2.0
    H = E + P / rho
    c2 = gamma * P / rho
    Vw = V[0] * w[1] + V[1] * w[2] + V[2] * w[3]
    out0 = rho * w[0] + rho * Vw + rho * E * w[4]
    mom = [rho * V[i] * w[0] + rho * V[i] * Vw + P * w[1 + i] + rho * H * V[i] * w[4]
           for i in range(3)]
    out4 = rho * E * w[0] + rho * H * Vw + (rho * H * H - c2 * P / (gamma - 1.0)) * w[4]
    return [out0, mom[0], mom[1], mom[2], out4]


def tangents(n):
    """Two unit vectors completing n to an orthonormal frame."""
    n = np.asarray(n, dtype=np.float64)
    e = np.zeros(3)
    e[int(np.argmin(np.abs(n)))] = 1.0
    t1 = np.cross(n, e)
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    return t1, t2


def kepes_parts(vh, v, n, gamma, eps):
    """Pieces of the KEPES dissipation, eq. (KEPES1)-(KEPES5), (ES).

    Columns of R-bar for a general normal (the paper prints n = e_x):
      r1 = [1, Vb - c n, h - vn c], r2 = [1, Vb, avg(|V|^2)/2],
      r3,4 = [0, t, Vb.t], r5 = [1, Vb + c n, h + vn c];
    T-bar = diag(rho_ln/(2 gamma), rho_ln (gamma-1)/gamma, Pbar, Pbar, rho_ln/(2 gamma));
    |Lambda| = (1-theta)|lambda_KEPES| + theta |lambda_max| I with
    lambda_KEPES = (vn + c, vn, vn, vn, vn + c), lambda_max = |vn| + c,
    theta = sqrt(|(P - Ph)/(P + Ph)|); c = sqrt(gamma Pbar / rho_ln),
    h = gamma/(beta_ln (gamma-1)) + avg(|V|^2)/2.
    """
    F, m = ec_flux(vh, v, n, gamma, eps)
    Vb = m["Vbar"]
    vn = Vb[0] * n[0] + Vb[1] * n[1] + Vb[2] * n[2]
    c = sqrt(gamma * m["P_bar"] / m["rho_ln"])
    hb = gamma / (m["beta_ln"] * (gamma - 1.0)) + m["V2_bar"] / 2.0
    t1, t2 = tangents(n)
    R = [
        [1.0 + 0.0 * c, Vb[0] - c * n[0], Vb[1] - c * n[1], Vb[2] - c * n[2], hb - vn * c],
        [1.0 + 0.0 * c, Vb[0], Vb[1], Vb[2], m["V2_bar"] / 2.0],
        [0.0 * c, 0.0 * c + t1[0], 0.0 * c + t1[1], 0.0 * c + t1[2],
         Vb[0] * t1[0] + Vb[1] * t1[1] + Vb[2] * t1[2]],
        [0.0 * c, 0.0 * c + t2[0], 0.0 * c + t2[1], 0.0 * c + t2[2],
         Vb[0] * t2[0] + Vb[1] * t2[1] + Vb[2] * t2[2]],
        [1.0 + 0.0 * c, Vb[0] + c * n[0], Vb[1] + c * n[1], Vb[2] + c * n[2], hb + vn * c],
    ]
    T = [m["rho_ln"] / (2.0 * gamma), m["rho_ln"] * (gamma - 1.0) / gamma,
         m["P_bar"], m["P_bar"], m["rho_ln"] / (2.0 * gamma)]
    theta = sqrt_abs((m["P"] - m["Ph"]) / (m["P"] + m["Ph"]))
    lam = [vn + c, vn, vn, vn, vn + c]
    lmax = absval(vn) + c
    L = [(1.0 - theta) * absval(lam[k]) + theta * lmax for k in range(5)]
    return F, R, T, L, m


def kepes_flux(vh, v, n, gamma, eps):
    """KEPES flux, eq. (ES): Fbar - 1/2 Rbar |Lambda| Tbar Rbar^T [[v]]."""
    F, R, T, L, _ = kepes_parts(vh, v, n, gamma, eps)
    jump = [vh[k] - v[k] for k in range(5)]
    out = list(F)
    for col in range(5):
        proj = R[col][0] * jump[0]
        for k in range(1, 5):
            proj = proj + R[col][k] * jump[k]
        coef = 0.5 * L[col] * T[col] * proj
        for k in range(5):
            out[k] = out[k] - R[col][k] * coef
    return out


def inviscid_trace_flux(vh, v, n, prm):
    gamma, eps = prm["gamma"], prm["logmean_eps"]
    fl = prm["flux"]
    if fl == 0:
        return ec_flux(vh, v, n, gamma, eps)[0]
    if fl == 1:
        return es_flux(vh, v, n, gamma)
    if fl == 2:
        return kepes_flux(vh, v, n, gamma, eps)
    raise ValueError(fl)


def viscous_trace_flux(vh, v, q, n, prm):
    """Entropy viscous trace flux, eq. (Flux_En_Vis):
    G(vh, q).n - 1/2 sigma_vis [[v]] with sigma_vis diagonal."""
    Gn = normal_flux(viscous_flux(vh, q, prm), n)
    sv = prm["sigma_vis"]
    return [Gn[k] - 0.5 * sv[k] * (vh[k] - v[k]) for k in range(5)]


def entropy_production_integrand(vh, v, Fhat, n, gamma):
    """[[v]]^T Fhat - [[Psi_n]] (Thm. EC_ES), Psi_n = rho V.n."""
    Ps = entropy_potential(v, gamma)
    Psh = entropy_potential(vh, gamma)
    out = 0.0
    for k in range(5):
        out = out + (vh[k] - v[k]) * Fhat[k]
    for j in range(3):
        if n[j] != 0.0:
            out = out - (Psh[j] - Ps[j]) * n[j]
    return out
