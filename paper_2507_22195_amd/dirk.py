"""Newton + DIRK(3,3) time stepping on the GPU (Sec. 5.3, 6.1, 6.2, Algorithm 1).

A host loop over stages and Newton iterations; every arithmetic step runs
in the library: residual and condensed local systems (mehdg_assemble,
mehdg_condense), the global trace system and its GMRES solve
(mehdg_trace_*), the local recovery (mehdg_recover), the updates and norms
(mehdg_axpby, mehdg_dot).

Time integration: Alexander's L-stable three-stage DIRK(3,3) (all a_ii = g,
g the root in (1/6, 1/2) of g^3 - 3 g^2 + 3g/2 - 1/6).  Stage i solves
    alpha ((u(V_i), phi) - (u(v^n), phi)) + R_sp(V_i) + alpha dt sum_{j<i} a_ij R_sp(V_j) = 0,
alpha = 1/(g dt): the library's residual with v_old = v^n plus the constant
source s_i = alpha dt sum_{j<i} a_ij R_sp(V_j) (mehdg_add_source); R_sp(V_j)
is the residual without time term, from a second context with alpha_t = 0.
The method is stiffly accurate: v^{n+1} = V_3.  Newton stops when the
Euclidean norm of the interior residual and of the assembled trace residual
falls below tol.

Nonlinear solver (Sec. 6.1): with ``ptc`` (the default) an inexact Newton
method with pseudo-transient continuation.  The Jacobian carries the
pseudo-time term (A0 dV, w) / tau; tau starts at tau_init = 1 and follows the
residual (switched evolution-relaxation: tau <- min(tau_max, tau |R_prev| /
|R|), tau_max = 1e8; the Jacobian of iterate m uses the tau from iterates m-2
and m-1, because an iterate's residual comes from the same assembly as its
Jacobian), so early iterations are damped and late ones are Newton steps.  The trace system is solved to the relative tolerance
eta = min(eta_max, gamma (|R| / |R_prev|)^2) (Eisenstat and Walker's second
choice, eta_max = 0.1, gamma = 0.9), kept above the level where the next
residual could not tell (tol / (2 |R|)) and below the fixed gmres_rtol bound
from above only through eta_max.  With ptc = False: exact Newton (no
pseudo-time term) with every trace solve to gmres_rtol.
"""
from __future__ import annotations

import numpy as np

from . import mehdg


def dirk33_tableau():
    """Butcher matrix of Alexander's DIRK(3,3) (stiffly accurate, L-stable)."""
    roots = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
    g = float([r.real for r in roots if abs(r.imag) < 1e-12 and 1.0 / 6.0 < r.real < 0.5][0])
    return np.array([[g, 0.0, 0.0],
                     [(1.0 - g) / 2.0, g, 0.0],
                     [-(6.0 * g * g - 16.0 * g + 1.0) / 4.0, (6.0 * g * g - 20.0 * g + 5.0) / 4.0, g]])


class PseudoTime:
    """Residual-based control of the pseudo-time step (switched
    evolution-relaxation): tau_{m+1} = min(tau_max, tau_m |R_{m-1}| / |R_m|)."""

    def __init__(self, tau_init=1.0, tau_max=1e8):
        if not (tau_init > 0.0 and tau_max >= tau_init):
            raise ValueError("need 0 < tau_init <= tau_max")
        self.tau_init, self.tau_max = float(tau_init), float(tau_max)
        self.reset()

    def reset(self):
        self.tau = self.tau_init
        self.prev = None
        self.history = [self.tau]

    def update(self, rnorm):
        """Record the residual norm of a new iterate; returns the next tau."""
        if self.prev is not None and rnorm > 0.0:
            self.tau = min(self.tau_max, self.tau * self.prev / rnorm)
            self.history.append(self.tau)
        self.prev = rnorm
        return self.tau


def forcing_term(rnorm, rprev, tol, eta_max=0.1, gamma=0.9):
    """Relative tolerance of the linear solve of one inexact Newton step:
    Eisenstat and Walker's choice 2, eta = gamma (|R| / |R_prev|)^2 (eta_max on
    the first step), capped by eta_max and kept above tol / (2 |R|)."""
    eta = eta_max if rprev is None else min(eta_max, gamma * (rnorm / rprev) ** 2)
    return max(eta, 0.5 * tol / max(rnorm, 1e-300))


class DirkStepper:
    """One context per time-step size; v [M][5][n] and the global trace
    vh [faces][5][nf] are device tensors, updated in place by step()."""

    def __init__(self, p, h, params, dt, face_ids, n_faces, tol=1e-11, max_newton=15, gmres_rtol=1e-13,
                 gmres_restart=40, gmres_maxit=1000, ptc=True, tau_init=1.0, tau_max=1e8):
        import torch
        self.A = dirk33_tableau()
        self.dt = float(dt)
        g = self.A[0, 0]
        self.alpha = 1.0 / (g * self.dt)
        prm = dict(params, alpha_t=self.alpha, alpha_ps=0.0)
        self.ctx = mehdg.Context(p, h, prm)
        self.ctx_sp = mehdg.Context(p, h, dict(params, alpha_t=0.0, alpha_ps=0.0))
        self.ctx.trace_setup(face_ids, n_faces)
        self.tol, self.max_newton = tol, max_newton
        self.gmres = dict(rtol=gmres_rtol, restart=gmres_restart, maxit=gmres_maxit)
        self.ptc = PseudoTime(tau_init, tau_max) if ptc else None
        self.tau_history = []
        S = self.ctx.shapes()
        e = lambda k: torch.empty(S[k], dtype=torch.float64, device="cuda")
        self.R_q, self.R_v, self.R_vh, self.ent = e("R_q"), e("R_v"), e("R_vhat"), e("entropy")
        self.Ahat, self.bhat, self.dv, self.dq = e("Ahat"), e("bhat"), e("dv"), e("dq")
        self.vhat = e("vhat")
        self.v_old = e("v")
        T = self.ctx.trace_shape()
        self.F = torch.empty(T, dtype=torch.float64, device="cuda")
        self.Rg = torch.empty_like(self.F)
        self.dV = torch.empty_like(self.F)
        self.src = e("R_v")
        self.Rsp = [e("R_v") for _ in range(3)]
        self.iterations = []

    def _residual_norm(self):
        self.ctx.trace_rhs(self.R_vh.reshape(self.bhat.shape), self.Rg)
        return np.sqrt(self.ctx.dot(self.R_v, self.R_v) + self.ctx.dot(self.Rg, self.Rg))

    def _newton(self, v, vh, v_old, src):
        c = self.ctx
        its = 0
        rprev = None
        if self.ptc is not None:
            self.ptc.reset()
        for its in range(self.max_newton + 1):
            if self.ptc is not None:
                c.set_pseudo_time(1.0 / self.ptc.tau)
            c.trace_gather(vh, self.vhat)
            c.assemble(v, self.vhat, None, v_old, self.R_q, self.R_v, self.R_vh, self.ent, want_blocks=True)
            if src is not None:
                c.add_source(src, self.R_v)
            rnorm = self._residual_norm()
            if rnorm < self.tol or its == self.max_newton:
                break
            gm = dict(self.gmres)
            if self.ptc is not None:
                # tau of the next iterate's Jacobian (the residual of an iterate comes
                # from the same assembly as its Jacobian: one iteration of lag)
                self.ptc.update(rnorm)
                gm["rtol"] = max(self.gmres["rtol"], forcing_term(rnorm, rprev, self.tol))
            rprev = rnorm
            c.condense(self.Ahat, self.bhat)
            c.trace_rhs(self.bhat, self.F)
            mehdg.axpby(0.0, self.F, 0.0, self.dV)
            c.trace_solve(self.Ahat, self.F, self.dV, **gm)
            c.trace_gather(self.dV, self.vhat)
            c.recover(self.R_q, self.vhat, self.dv, self.dq)
            mehdg.axpby(1.0, self.dv, 1.0, v)
            mehdg.axpby(1.0, self.dV, 1.0, vh)
        rc, st = c.status()
        if rc:
            raise mehdg.MehdgError(rc, "Newton iteration")
        if self.ptc is not None:
            self.tau_history.append(list(self.ptc.history))
        return its

    def step(self, v, vh):
        """One DIRK(3,3) step: v, vh (device) are replaced by the new state."""
        import torch
        v_old = self.v_old
        mehdg.axpby(1.0, v, 0.0, v_old)
        its = []
        for i in range(3):
            src = None
            if i > 0:
                self.src.zero_()
                for j in range(i):
                    mehdg.axpby(self.alpha * self.dt * self.A[i, j], self.Rsp[j], 1.0, self.src)
                src = self.src
            its.append(self._newton(v, vh, v_old, src))
            if i < 2:
                # R_sp(V_i): residual without time term
                self.ctx.trace_gather(vh, self.vhat)
                self.ctx_sp.assemble(v, self.vhat, None, v, self.R_q, self.Rsp[i], self.R_vh, self.ent,
                                     want_blocks=False)
        self.iterations.append(its)
        torch.cuda.synchronize()
        return its

    def close(self):
        self.ctx.close()
        self.ctx_sp.close()
