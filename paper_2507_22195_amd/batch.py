"""Macro-elements of mixed polynomial degree in one Newton step (argument
marshalling over the library's ``mehdg_batch_*`` calls).

The library's kernels are compiled per degree.  A batch orders the
macro-elements by degree (stable), keeps one context per degree present,
and lays every per-macro array out flat in that order, so the macros of one
degree are one contiguous slice that its context reads and writes in place.
One library call per phase runs every degree group, each on a stream of the
batch (default priority) forked from and joined back to the caller's stream,
so the small groups overlap the large ones; the whole FP64 step can be
captured in one HIP graph (torch.cuda.graph), as its calls allocate nothing
once the contexts' workspaces exist (the first step).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import mehdg

_KEY = {"v": "v", "q": "q", "vhat": "vhat", "R_q": "q", "R_v": "v", "R_vhat": "vhat", "entropy": "entropy",
        "Ahat": "Ahat", "bhat": "bhat", "dv": "v", "dq": "q"}


def _shape(key, cnt, s):
    n, nf, NH = s["n"], s["nf"], s["N_VH"]
    return {"v": (cnt, 5, n), "q": (cnt, 5, 3, n), "vhat": (cnt, 6, 5, nf), "entropy": (cnt,),
            "Ahat": (cnt, NH, NH), "bhat": (cnt, NH)}[_KEY[key]]


class MixedBatch:
    """p [n_macro] degrees (1..4), h [n_macro][3], one parameter set, face_bc
    [n_macro][6] wall flags or None; max_workspace_bytes bounds the contexts'
    device workspace (0: the library's default), beyond which the groups with
    the largest macros are streamed in waves (``waves``); residual_per_degree
    replaces the persistent residual launch by one launch per degree."""

    def __init__(self, p, h, params, face_bc=None, max_workspace_bytes=0, residual_per_degree=False):
        lib = mehdg.load()
        p = np.ascontiguousarray(np.asarray(p, dtype=np.int32))
        h = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
        if p.ndim != 1 or h.shape != (p.size, 3):
            raise ValueError("p must be [n_macro] and h [n_macro][3]")
        bc_ptr = None
        if face_bc is not None:
            bc = np.ascontiguousarray(np.asarray(face_bc, dtype=np.uint8))
            if bc.shape != (p.size, 6):
                raise ValueError("face_bc must be [n_macro][6]")
            bc_ptr = bc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        mesh = mehdg.BatchMesh(p.size, p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), bc_ptr, int(max_workspace_bytes),
                               int(bool(residual_per_degree)), 0)
        self._prm = mehdg.make_params(params)
        handle = ctypes.c_void_p()
        rc = lib.mehdg_batch_create(ctypes.byref(mesh), ctypes.byref(self._prm), ctypes.byref(handle))
        if rc:
            raise mehdg.MehdgError(rc, "mehdg_batch_create")
        self._handle = handle
        self.n_macro = int(p.size)
        ng = ctypes.c_int32()
        deg, first, count, wave = (ctypes.c_int32 * 4)(), (ctypes.c_int64 * 4)(), (ctypes.c_int64 * 4)(), \
            (ctypes.c_int64 * 4)()
        rc = lib.mehdg_batch_groups(handle, ctypes.byref(ng), deg, first, count, wave)
        if rc:
            raise mehdg.MehdgError(rc, "mehdg_batch_groups")
        # (degree, first batch position, count, sizes of the degree)
        self.groups = [(int(deg[i]), int(first[i]), int(count[i]), mehdg.sizes(int(deg[i])))
                       for i in range(ng.value)]
        self.waves = {int(deg[i]): int(wave[i]) for i in range(ng.value)}   # macros per wave, per degree
        order = np.empty(self.n_macro, dtype=np.int64)
        self._off = {}
        for key, code in mehdg.BATCH_KEYS.items():
            off = np.empty(self.n_macro + 1, dtype=np.int64)
            rc = lib.mehdg_batch_layout(handle, code, order.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
            if rc:
                raise mehdg.MehdgError(rc, "mehdg_batch_layout")
            self._off[key] = off
        self.order = order                                # batch position -> macro

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            mehdg.load().mehdg_batch_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # flat layout -------------------------------------------------------------
    def count(self, key):
        """Doubles of the flat array ``key`` over the whole batch."""
        return int(self._off[_KEY[key]][-1])

    def alloc(self, key):
        import torch
        return torch.empty(self.count(key), dtype=torch.float64, device="cuda")

    def view(self, flat, key, gi):
        """Group gi's slice of a flat array, shaped as a context of its degree expects."""
        d, first, c, s = self.groups[gi]
        off = self._off[_KEY[key]]
        return flat[int(off[first]):int(off[first + c])].view(_shape(key, c, s))

    def pack(self, key, parts):
        """Flat host array from per-degree arrays parts[d] ([count_d][...], macro order)."""
        return np.concatenate([np.ascontiguousarray(parts[d]).reshape(-1) for (d, _, _, _) in self.groups])

    def _flat(self, t, key, name, optional=False):
        return mehdg._ptr(t, (self.count(key),), name, optional)

    # the step ------------------------------------------------------------------
    def assemble_condense(self, v, vhat, v_old, R_q, R_v, R_vhat, entropy, Ahat, bhat, prec="fp64",
                          stream=None):
        F = self._flat
        rc = mehdg.load().mehdg_batch_assemble_condense(
            self._handle, mehdg.PRECISIONS[prec], F(v, "v", "v"), F(vhat, "vhat", "vhat"), F(v_old, "v", "v_old"),
            F(R_q, "R_q", "R_q"), F(R_v, "R_v", "R_v"), F(R_vhat, "R_vhat", "R_vhat"),
            F(entropy, "entropy", "entropy"), F(Ahat, "Ahat", "Ahat", optional=True), F(bhat, "bhat", "bhat"),
            mehdg._stream(stream))
        if rc:
            raise mehdg.MehdgError(rc, "mehdg_batch_assemble_condense")

    def recover(self, R_q, dvhat, dv, dq, v=None, vhat=None, v_old=None, stream=None):
        """Back-substitution; v, vhat, v_old (the inputs of assemble_condense) are
        needed when a group is streamed."""
        F = self._flat
        rc = mehdg.load().mehdg_batch_recover(
            self._handle, F(v, "v", "v", optional=True), F(vhat, "vhat", "vhat", optional=True),
            F(v_old, "v", "v_old", optional=True), F(R_q, "R_q", "R_q"), F(dvhat, "vhat", "dvhat"),
            F(dv, "dv", "dv"), F(dq, "dq", "dq"), mehdg._stream(stream))
        if rc:
            raise mehdg.MehdgError(rc, "mehdg_batch_recover")

    def step(self, v, vhat, v_old, R_q, R_v, R_vhat, entropy, Ahat, bhat, dvhat, dv, dq, prec="fp64"):
        """assemble + condense + recover of every degree group (flat arrays)."""
        self.assemble_condense(v, vhat, v_old, R_q, R_v, R_vhat, entropy, Ahat, bhat, prec=prec)
        self.recover(R_q, dvhat, dv, dq, v=v, vhat=vhat, v_old=v_old)

    def status(self):
        """(first non-zero code or 0, status per macro in macro order)."""
        st = np.zeros(self.n_macro, dtype=np.int32)
        rc = mehdg.load().mehdg_batch_status(self._handle, st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             mehdg._stream(None))
        if rc in (1, 3):
            raise mehdg.MehdgError(rc, "mehdg_batch_status")
        return int(rc), st
