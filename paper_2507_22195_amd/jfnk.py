"""Jacobian-free Newton-Krylov for the DIRK(3,3) stages, beside the assembled
Newton of dirk.DirkStepper (Sec. 6.1-6.2, Algorithm 1).

A host loop; every arithmetic step runs in the library.  The unknowns are
the interior v [M][5][n] and the global trace V [faces][5][nf] (q is the
weak gradient of (v, vhat)); the stage residual is

    G(v, V) = ( R_V(v, P V) + s,  sum_m P_m^T R_Vhat,m(v, P V) ),

P the gather of a macro's six faces.  Newton solves J_G d = -G without an
assembled Jacobian: the Krylov operator is

    J_G (x_v, x_V) = ( JR_V,  sum_m P_m^T JR_Vhat,m ),   JR = mehdg_jvp(x_v, P x_V),

the residual's JVP at the current iterate (coefficients stored by
mehdg_assemble with want_blocks = 2).  The Krylov method is flexible GMRES,
right-preconditioned by the assembled Newton solve of the stage's first
iterate, kept (lagged) for the later iterations: for a vector (a, c),

    bhat = -X S^-1 a                  (mehdg_condense_rhs, stored factors)
    K dV = c + sum_m P_m^T bhat       (mehdg_trace_solve with the lagged Ahat)
    dv   = S^-1 (a + Y P dV)          (mehdg_recover),

which is J_G^-1 exactly at that first iterate, so the first Newton step
takes one Krylov iteration and the later ones a few.
"""
from __future__ import annotations

import numpy as np

from . import mehdg
from .dirk import DirkStepper


class _Pair:
    """A vector of the global (v, V) space: two device tensors."""

    __slots__ = ("v", "V")

    def __init__(self, v, V):
        self.v, self.V = v, V

    @staticmethod
    def like(o):
        import torch
        return _Pair(torch.empty_like(o.v), torch.empty_like(o.V))


class JfnkStepper(DirkStepper):
    """DirkStepper whose Newton iterations use the residual JVP (see module
    docstring); krylov_rtol is the relative tolerance of each linear solve."""

    def __init__(self, *args, krylov_rtol=1e-9, krylov_restart=30, krylov_maxit=300, **kw):
        super().__init__(*args, **kw)
        import torch
        S = self.ctx.shapes()
        e = lambda k: torch.empty(S[k], dtype=torch.float64, device="cuda")
        self.k_rtol, self.k_restart, self.k_maxit = krylov_rtol, krylov_restart, krylov_maxit
        self.JRq, self.JRv, self.JRvh = e("R_q"), e("R_v"), e("R_vhat")
        self.xl = e("vhat")
        self.bt = e("bhat")
        self.zero_q = torch.zeros(S["R_q"], dtype=torch.float64, device="cuda")
        self.dq_tmp = e("dq")
        self.krylov = []
        self._basis = None            # Krylov vectors, allocated on the first solve

    # vector algebra through the library ------------------------------------
    def _dot(self, a, b):
        return self.ctx.dot(a.v, b.v) + self.ctx.dot(a.V, b.V)

    @staticmethod
    def _axpby(alpha, x, beta, y):
        mehdg.axpby(alpha, x.v, beta, y.v)
        mehdg.axpby(alpha, x.V, beta, y.V)

    # operators -------------------------------------------------------------
    def _apply_J(self, x, out):
        c = self.ctx
        c.trace_gather(x.V, self.xl)
        c.jvp(x.v, self.xl, None, self.JRq, self.JRv, self.JRvh)
        mehdg.axpby(1.0, self.JRv, 0.0, out.v)
        c.trace_rhs(self.JRvh.reshape(self.bt.shape), out.V)

    def _apply_M(self, r, out):
        c = self.ctx
        c.condense_rhs(r.v, None, self.bt)            # bt = -X S^-1 a
        c.trace_rhs(self.bt, self.F)                   # F = sum P^T bt
        mehdg.axpby(1.0, r.V, 1.0, self.F)             # F += c
        mehdg.axpby(0.0, self.F, 0.0, out.V)           # initial guess 0
        c.trace_solve(self.Ahat, self.F, out.V, **self.gmres)
        c.trace_gather(out.V, self.xl)
        c.recover(self.zero_q, self.xl, out.v, self.dq_tmp)

    def _fgmres(self, b, x):
        """Right-preconditioned flexible GMRES(restart) on J_G x = b from x = 0;
        returns the number of iterations."""
        bnorm = np.sqrt(self._dot(b, b))
        self._axpby(0.0, b, 0.0, x)
        if bnorm == 0.0:
            return 0
        its = 0
        if self._basis is None:
            m = self.k_restart
            self._basis = dict(r=_Pair.like(b), w=_Pair.like(b), V=[_Pair.like(b) for _ in range(m + 1)],
                               Z=[_Pair.like(b) for _ in range(m)])
        r, w = self._basis["r"], self._basis["w"]
        Vb, Zb = self._basis["V"], self._basis["Z"]
        while its < self.k_maxit:
            # r = b - J x
            self._apply_J(x, r)
            self._axpby(1.0, b, -1.0, r)
            beta = np.sqrt(self._dot(r, r))
            if beta <= self.k_rtol * bnorm:
                break
            m = self.k_restart
            V, Z = Vb, Zb
            self._axpby(1.0 / beta, r, 0.0, V[0])
            H = np.zeros((m + 1, m))
            g = np.zeros(m + 1)
            g[0] = beta
            k = 0
            for k in range(m):
                z = Z[k]
                self._apply_M(V[k], z)
                self._apply_J(z, w)
                for _ in range(2):                       # classical Gram-Schmidt, twice
                    hs = [self._dot(w, V[i]) for i in range(k + 1)]
                    for i in range(k + 1):
                        self._axpby(-hs[i], V[i], 1.0, w)
                        H[i, k] += hs[i]
                H[k + 1, k] = np.sqrt(self._dot(w, w))
                its += 1
                y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], g[:k + 2], rcond=None)
                res = np.linalg.norm(g[:k + 2] - H[:k + 2, :k + 1] @ y)
                if res <= self.k_rtol * bnorm or H[k + 1, k] == 0.0 or its >= self.k_maxit:
                    break
                self._axpby(1.0 / H[k + 1, k], w, 0.0, V[k + 1])
            for i in range(len(y)):
                self._axpby(float(y[i]), Z[i], 1.0, x)
            if res <= self.k_rtol * bnorm:
                break
        return its

    def _newton(self, v, vh, v_old, src):
        c = self.ctx
        b = _Pair(self.R_v, self.Rg)
        d = _Pair(self.dv, self.dV)
        its = 0
        kry = []
        for its in range(self.max_newton + 1):
            c.trace_gather(vh, self.vhat)
            # blocks (for the preconditioner) at the first iterate, JVP coefficients always
            c.assemble(v, self.vhat, None, v_old, self.R_q, self.R_v, self.R_vh, self.ent,
                       want_blocks=1 if its == 0 else 2)
            if src is not None:
                # R_v += s (the lagged factors take their right-hand sides from condense_rhs)
                mehdg.axpby(1.0, src, 1.0, self.R_v)
            if self._residual_norm() < self.tol or its == self.max_newton:
                break
            if its == 0:
                c.condense(self.Ahat, self.bhat)
            # b = -G
            mehdg.axpby(0.0, self.R_v, -1.0, self.R_v)
            mehdg.axpby(0.0, self.Rg, -1.0, self.Rg)
            kry.append(self._fgmres(b, d))
            mehdg.axpby(1.0, self.dv, 1.0, v)
            mehdg.axpby(1.0, self.dV, 1.0, vh)
        self.krylov.append(kry)
        rc, st = c.status()
        if rc:
            raise mehdg.MehdgError(rc, "Jacobian-free Newton iteration")
        return its
