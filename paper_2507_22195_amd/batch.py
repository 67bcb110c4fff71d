"""Macro-elements of mixed polynomial degree in one Newton step (argument
marshalling only).

The library's kernels are compiled per degree and a context holds one
degree.  A MixedBatch orders the macro-elements by degree (stable), keeps
one context per degree present, and lays every per-macro array out flat in
that order, so the macros of one degree are one contiguous slice: the
per-degree calls take views of the flat arrays, nothing is copied.  Each
degree runs on its own stream (default priority), forked from and joined
back to the caller's stream, so the small groups overlap the large ones; the
whole step can be captured in one HIP graph (torch.cuda.graph), as its calls
allocate nothing once the contexts' workspaces exist (the first step).
"""
from __future__ import annotations

import numpy as np

from . import mehdg

# per-macro sizes of the flat arrays, from mehdg.sizes(p)
_PER = {
    "v": lambda s: 5 * s["n"], "q": lambda s: 15 * s["n"], "vhat": lambda s: 30 * s["nf"],
    "R_q": lambda s: 15 * s["n"], "R_v": lambda s: 5 * s["n"], "R_vhat": lambda s: 30 * s["nf"],
    "entropy": lambda s: 1, "Ahat": lambda s: s["N_VH"] ** 2, "bhat": lambda s: s["N_VH"],
    "dv": lambda s: 5 * s["n"], "dq": lambda s: 15 * s["n"],
}


class MixedBatch:
    """p [n_macro] degrees, h [n_macro][3], one parameter set, face_bc
    [n_macro][6] wall flags or None."""

    def __init__(self, p, h, params, face_bc=None):
        p = np.asarray(p, dtype=np.int64)
        h = np.asarray(h, dtype=np.float64)
        if p.ndim != 1 or h.shape != (p.size, 3):
            raise ValueError("p must be [n_macro] and h [n_macro][3]")
        self.n_macro = int(p.size)
        self.order = np.argsort(p, kind="stable")       # batch position -> macro
        self.p_sorted = p[self.order]
        self.groups = []                                 # (degree, first, count, context)
        first = 0
        for d in sorted(set(p.tolist())):
            cnt = int((p == d).sum())
            idx = self.order[first:first + cnt]
            bc = None if face_bc is None else np.asarray(face_bc, dtype=np.uint8)[idx]
            self.groups.append((int(d), first, cnt, mehdg.Context(int(d), h[idx], params, face_bc=bc)))
            first += cnt
        self._streams = None

    def close(self):
        for g in self.groups:
            g[3].close()

    # flat layout -------------------------------------------------------------
    def count(self, key):
        """Doubles of the flat array ``key`` over the whole batch."""
        return sum(c * _PER[key](ctx.sz) for (_, _, c, ctx) in self.groups)

    def offsets(self, key):
        out, off = [], 0
        for (_, _, c, ctx) in self.groups:
            out.append(off)
            off += c * _PER[key](ctx.sz)
        return out

    def alloc(self, key):
        import torch
        return torch.empty(self.count(key), dtype=torch.float64, device="cuda")

    def view(self, flat, key, gi):
        """Group gi's slice of a flat array, shaped as its context expects."""
        d, first, c, ctx = self.groups[gi]
        off = self.offsets(key)[gi]
        return flat[off:off + c * _PER[key](ctx.sz)].view(ctx.shapes()[key])

    def pack(self, key, parts):
        """Flat host array from per-degree arrays parts[d] ([count_d][...], macro order)."""
        return np.concatenate([np.ascontiguousarray(parts[d]).reshape(-1) for (d, _, _, _) in self.groups])

    # the step ------------------------------------------------------------------
    def step(self, v, vhat, v_old, R_q, R_v, R_vhat, entropy, Ahat, bhat, dvhat, dv, dq):
        """assemble + condense + recover of every degree group (flat arrays)."""
        import torch
        if self._streams is None:
            self._streams = [torch.cuda.Stream() for _ in self.groups]
        cur = torch.cuda.current_stream()
        for gi, (d, first, c, ctx) in enumerate(self.groups):
            s = self._streams[gi]
            s.wait_stream(cur)
            with torch.cuda.stream(s):
                V = lambda t, k: self.view(t, k, gi)
                ctx.assemble(V(v, "v"), V(vhat, "vhat"), None, V(v_old, "v"), V(R_q, "R_q"), V(R_v, "R_v"),
                             V(R_vhat, "R_vhat"), V(entropy, "entropy"), want_blocks=True)
                ctx.condense(V(Ahat, "Ahat"), V(bhat, "bhat"))
                ctx.recover(V(R_q, "R_q"), V(dvhat, "vhat"), V(dv, "dv"), V(dq, "dq"))
        for s in self._streams:
            cur.wait_stream(s)

    def status(self):
        """(first non-zero code or 0, status per macro in macro order)."""
        st = np.zeros(self.n_macro, dtype=np.int32)
        first_rc = 0
        for (d, first, c, ctx) in self.groups:
            rc, s = ctx.status()
            st[self.order[first:first + c]] = s
            if rc and not first_rc:
                first_rc = rc
        return first_rc, st
