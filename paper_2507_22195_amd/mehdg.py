"""ctypes binding of ``libmehdg.so`` (argument marshalling only).

Every step of the local work runs in the library's HIP kernels; this module
checks tensor shapes, dtypes and devices, passes raw device pointers and the
current HIP stream, and turns error codes into exceptions.  It never falls
back to anything else: if the library is missing or a call fails, it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmehdg.so")

ERRORS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ESTATE", 5: "ENONPHYSICAL",
          6: "ENONFINITE", 7: "ESINGULAR", 8: "EIRNOCONV"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
# refinement defaults of the mixed-precision condensation: the estimated relative
# forward error of S^-1 [-Y | r_V] at most 1e-10, at most 12 refinement steps
IR_TOL, IR_MAXIT = 1e-10, 12
EXPORTS = ("mehdg_sizes", "mehdg_create", "mehdg_destroy", "mehdg_assemble", "mehdg_condense",
           "mehdg_recover", "mehdg_status", "mehdg_copy_bordered", "mehdg_workspace_bytes",
           "mehdg_profile_enable", "mehdg_profile_read", "mehdg_ir_iterations", "mehdg_load_bordered")
PROF_SLOTS = ("residual", "minv_rq", "rows_v", "rows_h", "panel", "rowblock", "update", "schur",
              "recover", "trsm", "jvp", "vjp", "fsolve", "lp_panel", "lp_update", "lp_solve", "ir_resid",
              "lp_move")


class MehdgError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {ERRORS.get(code, code)}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("kappa", ctypes.c_double),
                ("lam", ctypes.c_double), ("sigma_vis", ctypes.c_double * 5),
                ("alpha_t", ctypes.c_double), ("alpha_ps", ctypes.c_double),
                ("logmean_eps", ctypes.c_double), ("T_wall", ctypes.c_double), ("flux", ctypes.c_int32),
                ("viscous", ctypes.c_int32), ("ir_tol", ctypes.c_double), ("ir_maxit", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class Mesh(ctypes.Structure):
    _fields_ = [("n_macro", ctypes.c_int64), ("p", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("h", ctypes.POINTER(ctypes.c_double)), ("face_bc", ctypes.POINTER(ctypes.c_uint8))]


class BatchMesh(ctypes.Structure):
    _fields_ = [("n_macro", ctypes.c_int64), ("p", ctypes.POINTER(ctypes.c_int32)),
                ("h", ctypes.POINTER(ctypes.c_double)), ("face_bc", ctypes.POINTER(ctypes.c_uint8)),
                ("max_workspace_bytes", ctypes.c_int64), ("residual_per_degree", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


BATCH_KEYS = {"v": 0, "q": 1, "vhat": 2, "entropy": 3, "Ahat": 4, "bhat": 5}


class TetMesh(ctypes.Structure):
    _fields_ = [("n_macro", ctypes.c_int64), ("p", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("X", ctypes.POINTER(ctypes.c_double)), ("face_bc", ctypes.POINTER(ctypes.c_uint8))]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2507_22195_amd.build")
    # torch ships its own HIP runtime; importing it first makes the library
    # bind to that same runtime (same soname), so that torch's device
    # pointers and streams are valid in the library's calls.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.mehdg_sizes.argtypes = [i32, ctypes.POINTER(ctypes.c_int64)]
    lib.mehdg_create.argtypes = [ctypes.POINTER(Mesh), ctypes.POINTER(Params), ctypes.POINTER(vp)]
    lib.mehdg_destroy.argtypes = [vp]
    lib.mehdg_assemble.argtypes = [vp] + [vp] * 8 + [i32, vp]
    lib.mehdg_condense.argtypes = [vp, i32, vp, vp, vp]
    lib.mehdg_ir_iterations.argtypes = [vp]
    lib.mehdg_ir_iterations.restype = i32
    lib.mehdg_recover.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mehdg_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.mehdg_copy_bordered.argtypes = [vp, i64, vp, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]
    lib.mehdg_load_bordered.argtypes = [vp, i64, vp]
    lib.mehdg_profile_enable.argtypes = [vp, i32]
    lib.mehdg_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32]
    lib.mehdg_workspace_bytes.argtypes = [vp]
    lib.mehdg_workspace_bytes.restype = i64
    lib.mehdg_trace_setup.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), i64]
    lib.mehdg_trace_rhs.argtypes = [vp, vp, vp, vp]
    lib.mehdg_trace_apply.argtypes = [vp, vp, vp, vp, vp]
    lib.mehdg_trace_gather.argtypes = [vp, vp, vp, vp]
    lib.mehdg_trace_precond_setup.argtypes = [vp, vp, vp]
    lib.mehdg_trace_precond_apply.argtypes = [vp, vp, vp, vp]
    lib.mehdg_trace_solve.argtypes = [vp, vp, vp, vp, ctypes.c_double, i32, i32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_double), vp]
    lib.mehdg_trace_solve_fgmres.argtypes = [vp, vp, vp, vp, ctypes.c_double, i32, i32, i32,
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_double), vp]
    lib.mehdg_add_source.argtypes = [vp, vp, vp, vp]
    lib.mehdg_jvp.argtypes = [vp] + [vp] * 6 + [vp]
    lib.mehdg_condense_rhs.argtypes = [vp, vp, vp, vp, vp]
    lib.mehdg_vjp.argtypes = [vp] + [vp] * 6 + [vp]
    lib.mehdg_axpby.argtypes = [i64, ctypes.c_double, vp, ctypes.c_double, vp, vp]
    lib.mehdg_set_pseudo_time.argtypes = [vp, ctypes.c_double]
    lib.mehdg_dot.argtypes = [vp, i64, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.mehdg_dot_noalloc.argtypes = [i64, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.mehdg_batch_create.argtypes = [ctypes.POINTER(BatchMesh), ctypes.POINTER(Params), ctypes.POINTER(vp)]
    lib.mehdg_batch_destroy.argtypes = [vp]
    lib.mehdg_batch_layout.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.mehdg_batch_groups.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64)]
    lib.mehdg_batch_assemble_condense.argtypes = [vp, i32] + [vp] * 9 + [vp]
    lib.mehdg_batch_recover.argtypes = [vp] + [vp] * 7 + [vp]
    lib.mehdg_batch_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    for name in ("mehdg_batch_create", "mehdg_batch_destroy", "mehdg_batch_layout", "mehdg_batch_groups",
                 "mehdg_batch_assemble_condense", "mehdg_batch_recover", "mehdg_batch_status"):
        getattr(lib, name).restype = ctypes.c_int
    lib.mehdg_trace_set_inner_precision.argtypes = [vp, i32]
    lib.mehdg_trace_set_inner_precision.restype = ctypes.c_int
    lib.mehdg_tile_variants.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.mehdg_set_tile.argtypes = [vp, i32, i32]
    lib.mehdg_get_tile.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32)]
    lib.mehdg_set_lu_depth.argtypes = [vp, i32]
    lib.mehdg_get_lu_depth.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    for name in ("mehdg_tile_variants", "mehdg_set_tile", "mehdg_get_tile", "mehdg_set_lu_depth",
                 "mehdg_get_lu_depth"):
        getattr(lib, name).restype = ctypes.c_int
    lib.mehdg_tet_sizes.argtypes = [i32, ctypes.POINTER(ctypes.c_int64)]
    lib.mehdg_tet_create.argtypes = [ctypes.POINTER(TetMesh), ctypes.POINTER(Params), ctypes.POINTER(vp)]
    lib.mehdg_tet_destroy.argtypes = [vp]
    lib.mehdg_tet_residual.argtypes = [vp] + [vp] * 8 + [vp]
    lib.mehdg_tet_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.mehdg_tet_jvp.argtypes = [vp] + [vp] * 9 + [vp]
    lib.mehdg_tet_assemble.argtypes = [vp] + [vp] * 7 + [vp]
    lib.mehdg_tet_condense.argtypes = [vp, vp, vp, vp]
    lib.mehdg_tet_recover.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mehdg_tet_vjp.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mehdg_tet_condense_rhs.argtypes = [vp, vp, vp, vp, vp]
    for name in ("mehdg_tet_sizes", "mehdg_tet_create", "mehdg_tet_destroy", "mehdg_tet_residual",
                 "mehdg_tet_status", "mehdg_tet_jvp", "mehdg_tet_assemble", "mehdg_tet_condense",
                 "mehdg_tet_recover", "mehdg_tet_vjp", "mehdg_tet_condense_rhs"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("mehdg_add_source", "mehdg_axpby", "mehdg_dot", "mehdg_dot_noalloc", "mehdg_jvp", "mehdg_vjp",
                 "mehdg_condense_rhs", "mehdg_set_pseudo_time"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("mehdg_sizes", "mehdg_create", "mehdg_destroy", "mehdg_assemble", "mehdg_condense",
                 "mehdg_recover", "mehdg_status", "mehdg_copy_bordered", "mehdg_load_bordered", "mehdg_profile_enable",
                 "mehdg_profile_read", "mehdg_trace_setup", "mehdg_trace_rhs", "mehdg_trace_apply",
                 "mehdg_trace_gather", "mehdg_trace_precond_setup", "mehdg_trace_precond_apply",
                 "mehdg_trace_solve", "mehdg_trace_solve_fgmres"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def axpby(a, x, b, y, stream=None):
    """y = a x + b y (device float64 tensors of one shape)."""
    if x.shape != y.shape:
        raise ValueError("x and y differ in shape")
    rc = load().mehdg_axpby(int(x.numel()), float(a), _ptr(x, tuple(x.shape), "x"), float(b),
                            _ptr(y, tuple(y.shape), "y"), _stream(stream))
    if rc:
        raise MehdgError(rc, "mehdg_axpby")


def dot_noalloc(x, y, stream=None) -> float:
    """x . y through mehdg_dot_noalloc (no context, no device allocation)."""
    if x.shape != y.shape:
        raise ValueError("x and y differ in shape")
    out = ctypes.c_double()
    rc = load().mehdg_dot_noalloc(int(x.numel()), _ptr(x, tuple(x.shape), "x"), _ptr(y, tuple(y.shape), "y"),
                                  ctypes.byref(out), _stream(stream))
    if rc:
        raise MehdgError(rc, "mehdg_dot_noalloc")
    return out.value


TILE_SITES = {"update": 0, "schur": 1}


def tile_variants() -> list:
    """The tile shapes of the batched FP64 products: per variant a dict of
    waves (WM x WN), 16 x 16 blocks per wave (BI x BJ), K chunk, waves per SIMD,
    and the workgroup tile TM x TN."""
    lib = load()
    n = ctypes.c_int32()
    rc = lib.mehdg_tile_variants(ctypes.byref(n), None)
    if rc:
        raise MehdgError(rc, "mehdg_tile_variants")
    buf = (ctypes.c_int32 * (6 * n.value))()
    lib.mehdg_tile_variants(ctypes.byref(n), buf)
    out = []
    for i in range(n.value):
        wm, wn, bi, bj, kc, occ = buf[6 * i:6 * i + 6]
        out.append(dict(WM=wm, WN=wn, BI=bi, BJ=bj, KC=kc, OCC=occ, TM=16 * wm * bi, TN=16 * wn * bj,
                        threads=64 * wm * wn))
    return out


def sizes(p: int) -> dict:
    out = (ctypes.c_int64 * 5)()
    rc = load().mehdg_sizes(p, out)
    if rc:
        raise MehdgError(rc, "mehdg_sizes")
    return dict(n=out[0], nf=out[1], N_V=out[2], N_Q=out[3], N_VH=out[4])


def make_params(prm: dict) -> Params:
    P = Params()
    P.gamma = prm["gamma"]
    P.mu = prm["mu"]
    P.kappa = prm["kappa"]
    P.lam = prm["lam"]
    for k in range(5):
        P.sigma_vis[k] = prm["sigma_vis"][k]
    P.alpha_t = prm["alpha_t"]
    P.alpha_ps = prm["alpha_ps"]
    P.logmean_eps = prm["logmean_eps"]
    P.T_wall = float(prm.get("T_wall", 1.0))
    P.flux = int(prm["flux"])
    P.viscous = int(prm["viscous"])
    P.ir_tol = float(prm.get("ir_tol", IR_TOL))
    P.ir_maxit = int(prm.get("ir_maxit", IR_MAXIT))
    return P


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t, shape, name, optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owner of one library context (tables, mesh sizes, workspaces)."""

    def __init__(self, p: int, h, params: dict, face_bc=None):
        lib = load()
        h = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
        if h.ndim != 2 or h.shape[1] != 3:
            raise ValueError("h must be [n_macro][3]")
        self.p = int(p)
        self.n_macro = int(h.shape[0])
        self._h = h
        bc_ptr = None
        if face_bc is not None:
            self._bc = np.ascontiguousarray(np.asarray(face_bc, dtype=np.uint8))
            if self._bc.shape != (self.n_macro, 6):
                raise ValueError("face_bc must be [n_macro][6]")
            bc_ptr = self._bc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        mesh = Mesh(self.n_macro, self.p, 0, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), bc_ptr)
        self._prm = make_params(params)
        self.params = dict(params)
        handle = ctypes.c_void_p()
        rc = lib.mehdg_create(ctypes.byref(mesh), ctypes.byref(self._prm), ctypes.byref(handle))
        if rc:
            raise MehdgError(rc, "mehdg_create")
        self._handle = handle
        self.sz = sizes(self.p)

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            load().mehdg_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes -------------------------------------------------------------
    def shapes(self):
        M, s = self.n_macro, self.sz
        n, nf = s["n"], s["nf"]
        return dict(v=(M, 5, n), vhat=(M, 6, 5, nf), q=(M, 5, 3, n), R_q=(M, 5, 3, n),
                    R_v=(M, 5, n), R_vhat=(M, 6, 5, nf), entropy=(M,),
                    Ahat=(M, s["N_VH"], s["N_VH"]), bhat=(M, s["N_VH"]),
                    dv=(M, 5, n), dq=(M, 5, 3, n))

    def workspace_bytes(self) -> int:
        return int(load().mehdg_workspace_bytes(self._handle))

    # global trace system ------------------------------------------------
    def trace_setup(self, face_ids, n_faces: int):
        """face_ids [n_macro][6] (int64, host): global face of every local face."""
        ids = np.ascontiguousarray(np.asarray(face_ids, dtype=np.int64))
        if ids.shape != (self.n_macro, 6):
            raise ValueError(f"face_ids has shape {ids.shape}, expected {(self.n_macro, 6)}")
        rc = load().mehdg_trace_setup(self._handle, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      int(n_faces))
        if rc:
            raise MehdgError(rc, "mehdg_trace_setup")
        self.n_faces = int(n_faces)

    def trace_shape(self):
        return (self.n_faces, 5, self.sz["nf"])

    def trace_rhs(self, bhat, F, stream=None):
        S = self.shapes()
        rc = load().mehdg_trace_rhs(self._handle, _ptr(bhat, S["bhat"], "bhat"),
                                    _ptr(F, self.trace_shape(), "F"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_trace_rhs")

    def trace_apply(self, Ahat, x, y, stream=None):
        """y = K x; Ahat None: matrix-free from the factors of the last FP64 condensation."""
        S, T = self.shapes(), self.trace_shape()
        rc = load().mehdg_trace_apply(self._handle, _ptr(Ahat, S["Ahat"], "Ahat", optional=True), _ptr(x, T, "x"),
                                      _ptr(y, T, "y"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_trace_apply")

    def trace_gather(self, xg, xl, stream=None):
        rc = load().mehdg_trace_gather(self._handle, _ptr(xg, self.trace_shape(), "xg"),
                                       _ptr(xl, self.shapes()["vhat"], "xl"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_trace_gather")

    def trace_precond_setup(self, Ahat, stream=None):
        rc = load().mehdg_trace_precond_setup(self._handle,
                                              _ptr(Ahat, self.shapes()["Ahat"], "Ahat", optional=True),
                                              _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_trace_precond_setup")

    def trace_precond_apply(self, r, z, stream=None):
        T = self.trace_shape()
        rc = load().mehdg_trace_precond_apply(self._handle, _ptr(r, T, "r"), _ptr(z, T, "z"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_trace_precond_apply")

    def set_pseudo_time(self, alpha_ps: float):
        """alpha_ps = 1/tau of the pseudo-time Jacobian term for the following assembles."""
        rc = load().mehdg_set_pseudo_time(self._handle, float(alpha_ps))
        if rc:
            raise MehdgError(rc, "mehdg_set_pseudo_time")

    def add_source(self, s, R_v, stream=None):
        S = self.shapes()
        rc = load().mehdg_add_source(self._handle, _ptr(s, S["R_v"], "s"), _ptr(R_v, S["R_v"], "R_v"),
                                     _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_add_source")

    def dot(self, x, y, stream=None):
        if x.shape != y.shape:
            raise ValueError("x and y differ in shape")
        out = ctypes.c_double()
        rc = load().mehdg_dot(self._handle, int(x.numel()), _ptr(x, tuple(x.shape), "x"),
                              _ptr(y, tuple(y.shape), "y"), ctypes.byref(out), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_dot")
        return float(out.value)

    def trace_solve(self, Ahat, F, x, rtol=1e-10, maxit=500, restart=30, stream=None):
        """GMRES on K x = F (x: initial guess in, solution out); returns (iterations, relative residual)."""
        S, T = self.shapes(), self.trace_shape()
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        rc = load().mehdg_trace_solve(self._handle, _ptr(Ahat, S["Ahat"], "Ahat", optional=True), _ptr(F, T, "F"),
                                      _ptr(x, T, "x"), float(rtol), int(maxit), int(restart),
                                      ctypes.byref(it), ctypes.byref(rr), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_trace_solve")
        return int(it.value), float(rr.value)

    def trace_solve_fgmres(self, Ahat, F, x, rtol=1e-10, maxit=200, restart=30, inner=5, stream=None):
        """FGMRES on K x = F with `inner` block-Jacobi GMRES iterations as its preconditioner
        (Ahat None: matrix-free); returns (outer iterations, inner iterations, relative residual)."""
        S, T = self.shapes(), self.trace_shape()
        it, iin = ctypes.c_int32(), ctypes.c_int32()
        rr = ctypes.c_double()
        rc = load().mehdg_trace_solve_fgmres(self._handle, _ptr(Ahat, S["Ahat"], "Ahat", optional=True),
                                             _ptr(F, T, "F"), _ptr(x, T, "x"), float(rtol), int(maxit),
                                             int(restart), int(inner), ctypes.byref(it), ctypes.byref(iin),
                                             ctypes.byref(rr), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_trace_solve_fgmres")
        return int(it.value), int(iin.value), float(rr.value)

    # calls --------------------------------------------------------------
    def assemble(self, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, want_blocks=False, stream=None):
        S = self.shapes()
        args = [_ptr(v, S["v"], "v"), _ptr(vhat, S["vhat"], "vhat"),
                _ptr(q, S["q"], "q", optional=True), _ptr(v_old, S["v"], "v_old"),
                _ptr(R_q, S["R_q"], "R_q"), _ptr(R_v, S["R_v"], "R_v"),
                _ptr(R_vhat, S["R_vhat"], "R_vhat"), _ptr(entropy, S["entropy"], "entropy")]
        mode = want_blocks if isinstance(want_blocks, int) and not isinstance(want_blocks, bool) \
            else int(bool(want_blocks))
        rc = load().mehdg_assemble(self._handle, *args, mode, _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_assemble")

    def jvp(self, dv, dvhat, dq, JR_q, JR_v, JR_vhat, stream=None):
        """J [dq; dv; dvhat] at the state of the last assemble with want_blocks 1 or 2;
        dq None: the weak gradient of (dv, dvhat)."""
        S = self.shapes()
        rc = load().mehdg_jvp(self._handle, _ptr(dv, S["v"], "dv"), _ptr(dvhat, S["vhat"], "dvhat"),
                              _ptr(dq, S["q"], "dq", optional=True), _ptr(JR_q, S["R_q"], "JR_q"),
                              _ptr(JR_v, S["R_v"], "JR_v"), _ptr(JR_vhat, S["R_vhat"], "JR_vhat"),
                              _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_jvp")

    def vjp(self, w_v, w_vhat, g_v, g_vhat, w_q=None, g_q=None, stream=None):
        """J^T w at the same state; w_q, g_q None: through the weak gradient."""
        S = self.shapes()
        rc = load().mehdg_vjp(self._handle, _ptr(w_q, S["R_q"], "w_q", optional=True),
                              _ptr(w_v, S["R_v"], "w_v"), _ptr(w_vhat, S["R_vhat"], "w_vhat"),
                              _ptr(g_q, S["q"], "g_q", optional=True), _ptr(g_v, S["v"], "g_v"),
                              _ptr(g_vhat, S["vhat"], "g_vhat"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_vjp")

    def condense(self, Ahat, bhat, stream=None, prec="fp64"):
        """Static condensation; prec "fp64", "fp32" (FP32 LU + FP64 refinement) or
        "bf16" (BF16 MFMA trailing updates + FP64 refinement)."""
        S = self.shapes()
        if prec not in PRECISIONS:
            raise ValueError(f"prec must be one of {sorted(PRECISIONS)}")
        rc = load().mehdg_condense(self._handle, PRECISIONS[prec], _ptr(Ahat, S["Ahat"], "Ahat", optional=True),
                                   _ptr(bhat, S["bhat"], "bhat"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_condense")

    def ir_iterations(self) -> int:
        """Refinement steps of the last mixed-precision condensation."""
        return int(load().mehdg_ir_iterations(self._handle))

    def condense_rhs(self, r_v, r_hat, bhat, stream=None):
        """bhat = r_hat - X S^-1 r_v with the stored factors; r_hat None means zero.
        The next recover uses r_v.  r_v shaped like v, r_hat like R_vhat or bhat."""
        S = self.shapes()
        rh = None
        if r_hat is not None:
            rh = _ptr(r_hat, S["bhat"] if r_hat.dim() == 2 else S["R_vhat"], "r_hat")
        rc = load().mehdg_condense_rhs(self._handle, _ptr(r_v, S["v"], "r_v"), rh, _ptr(bhat, S["bhat"], "bhat"),
                                       _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_condense_rhs")

    def recover(self, R_q, dvhat, dv, dq, stream=None):
        S = self.shapes()
        rc = load().mehdg_recover(self._handle, _ptr(R_q, S["R_q"], "R_q"),
                                  _ptr(dvhat, S["vhat"], "dvhat"), _ptr(dv, S["dv"], "dv"),
                                  _ptr(dq, S["dq"], "dq"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_recover")

    def bordered(self, m: int):
        """Host copy [rows][ld] of macro m's bordered matrix (diagnostics)."""
        rows, ld = ctypes.c_int64(), ctypes.c_int64()
        lib = load()
        rc = lib.mehdg_copy_bordered(self._handle, int(m), None, ctypes.byref(rows), ctypes.byref(ld))
        if rc:
            raise MehdgError(rc, "mehdg_copy_bordered")
        out = np.empty((rows.value, ld.value), dtype=np.float64)
        rc = lib.mehdg_copy_bordered(self._handle, int(m), ctypes.c_void_p(out.ctypes.data),
                                     ctypes.byref(rows), ctypes.byref(ld))
        if rc:
            raise MehdgError(rc, "mehdg_copy_bordered")
        return out

    def load_bordered(self, m: int, Bm):
        """Replaces macro m's bordered matrix with the host array Bm [rows][ld] (tests)."""
        Bm = np.ascontiguousarray(Bm, dtype=np.float64)
        rows, ld = ctypes.c_int64(), ctypes.c_int64()
        lib = load()
        rc = lib.mehdg_copy_bordered(self._handle, int(m), None, ctypes.byref(rows), ctypes.byref(ld))
        if rc:
            raise MehdgError(rc, "mehdg_copy_bordered")
        if Bm.shape != (rows.value, ld.value):
            raise ValueError(f"bordered matrix shape {Bm.shape}, expected {(rows.value, ld.value)}")
        rc = lib.mehdg_load_bordered(self._handle, int(m), ctypes.c_void_p(Bm.ctypes.data))
        if rc:
            raise MehdgError(rc, "mehdg_load_bordered")

    def trace_set_inner_precision(self, prec: str):
        """Factors read by FGMRES's inner iterations (matrix-free): "fp64" or "fp32"."""
        rc = load().mehdg_trace_set_inner_precision(self._handle, PRECISIONS[prec])
        if rc:
            raise MehdgError(rc, "mehdg_trace_set_inner_precision")

    def set_tile(self, site: str, variant: int):
        """Tile variant of a product call site ("update", "schur"); -1 = the tuned table's."""
        rc = load().mehdg_set_tile(self._handle, TILE_SITES[site], int(variant))
        if rc:
            raise MehdgError(rc, "mehdg_set_tile")

    def get_tile(self, site: str) -> int:
        out = ctypes.c_int32()
        rc = load().mehdg_get_tile(self._handle, TILE_SITES[site], ctypes.byref(out))
        if rc:
            raise MehdgError(rc, "mehdg_get_tile")
        return int(out.value)

    def set_lu_depth(self, depth: int):
        """Outer blocks per group of delayed trailing updates of the LU of S (0 = the degree's default)."""
        rc = load().mehdg_set_lu_depth(self._handle, int(depth))
        if rc:
            raise MehdgError(rc, "mehdg_set_lu_depth")

    def get_lu_depth(self) -> int:
        out = ctypes.c_int32()
        rc = load().mehdg_get_lu_depth(self._handle, ctypes.byref(out))
        if rc:
            raise MehdgError(rc, "mehdg_get_lu_depth")
        return int(out.value)

    def profile(self, enable: bool):
        rc = load().mehdg_profile_enable(self._handle, int(bool(enable)))
        if rc:
            raise MehdgError(rc, "mehdg_profile_enable")

    def profile_read(self) -> dict:
        n = len(PROF_SLOTS)
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_int64 * n)()
        rc = load().mehdg_profile_read(self._handle, ms, calls, n)
        if rc:
            raise MehdgError(rc, "mehdg_profile_read")
        return {name: (ms[i], calls[i]) for i, name in enumerate(PROF_SLOTS)}

    def status(self, stream=None):
        out = np.zeros(self.n_macro, dtype=np.int32)
        rc = load().mehdg_status(self._handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 _stream(stream))
        return rc, out


def tet_sizes(p: int) -> dict:
    out = (ctypes.c_int64 * 5)()
    rc = load().mehdg_tet_sizes(p, out)
    if rc:
        raise MehdgError(rc, "mehdg_tet_sizes")
    return dict(n=out[0], nf=out[1], N_V=out[2], N_Q=out[3], N_VH=out[4])


class TetContext:
    """Owner of one context of tetrahedral macro-elements X [n_macro][4][3]
    (vertex coordinates, host); face_bc [n_macro][4] wall flags or None."""

    def __init__(self, p: int, X, params: dict, face_bc=None):
        lib = load()
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
        if X.ndim != 3 or X.shape[1:] != (4, 3):
            raise ValueError("X must be [n_macro][4][3]")
        self.p = int(p)
        self.n_macro = int(X.shape[0])
        self._X = X
        bc_ptr = None
        if face_bc is not None:
            self._bc = np.ascontiguousarray(np.asarray(face_bc, dtype=np.uint8))
            if self._bc.shape != (self.n_macro, 4):
                raise ValueError("face_bc must be [n_macro][4]")
            bc_ptr = self._bc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        mesh = TetMesh(self.n_macro, self.p, 0, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), bc_ptr)
        self._prm = make_params(params)
        self.params = dict(params)
        handle = ctypes.c_void_p()
        rc = lib.mehdg_tet_create(ctypes.byref(mesh), ctypes.byref(self._prm), ctypes.byref(handle))
        if rc:
            raise MehdgError(rc, "mehdg_tet_create")
        self._handle = handle
        self.sz = tet_sizes(self.p)

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            load().mehdg_tet_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shapes(self):
        M, n, nf, NH = self.n_macro, self.sz["n"], self.sz["nf"], self.sz["N_VH"]
        return dict(v=(M, 5, n), vhat=(M, 4, 5, nf), q=(M, 5, 3, n), R_q=(M, 5, 3, n), R_v=(M, 5, n),
                    R_vhat=(M, 4, 5, nf), entropy=(M,), Ahat=(M, NH, NH), bhat=(M, NH), dv=(M, 5, n),
                    dq=(M, 5, 3, n))

    def assemble(self, v, vhat, v_old, R_q, R_v, R_vhat, entropy, stream=None):
        """Residual (q the weak gradient) and the bordered matrices of the condensation."""
        S = self.shapes()
        rc = load().mehdg_tet_assemble(
            self._handle, _ptr(v, S["v"], "v"), _ptr(vhat, S["vhat"], "vhat"), _ptr(v_old, S["v"], "v_old"),
            _ptr(R_q, S["R_q"], "R_q"), _ptr(R_v, S["R_v"], "R_v"), _ptr(R_vhat, S["R_vhat"], "R_vhat"),
            _ptr(entropy, S["entropy"], "entropy"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_tet_assemble")

    def vjp(self, w_v, w_vhat, g_v, g_vhat, stream=None):
        """J_r^T [w_v; w_vhat] at the state of the last assemble (before condense)."""
        S = self.shapes()
        rc = load().mehdg_tet_vjp(self._handle, _ptr(w_v, S["R_v"], "w_v"), _ptr(w_vhat, S["R_vhat"], "w_vhat"),
                                  _ptr(g_v, S["v"], "g_v"), _ptr(g_vhat, S["vhat"], "g_vhat"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_tet_vjp")

    def condense(self, Ahat, bhat, stream=None):
        S = self.shapes()
        rc = load().mehdg_tet_condense(self._handle, _ptr(Ahat, S["Ahat"], "Ahat"), _ptr(bhat, S["bhat"], "bhat"),
                                       _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_tet_condense")

    def condense_rhs(self, r_v, r_hat, bhat, stream=None):
        """bhat = r_hat - X S^-1 r_V with the stored factors (r_hat None: zero)."""
        S = self.shapes()
        rc = load().mehdg_tet_condense_rhs(self._handle, _ptr(r_v, S["R_v"], "r_v"),
                                           _ptr(r_hat, S["bhat"], "r_hat", optional=True),
                                           _ptr(bhat, S["bhat"], "bhat"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_tet_condense_rhs")

    def recover(self, R_q, dvhat, dv, dq, stream=None):
        S = self.shapes()
        rc = load().mehdg_tet_recover(self._handle, _ptr(R_q, S["R_q"], "R_q"), _ptr(dvhat, S["vhat"], "dvhat"),
                                      _ptr(dv, S["dv"], "dv"), _ptr(dq, S["dq"], "dq"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_tet_recover")

    def residual(self, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, stream=None):
        """q None: the weak gradient of (v, vhat)."""
        S = self.shapes()
        rc = load().mehdg_tet_residual(
            self._handle, _ptr(v, S["v"], "v"), _ptr(vhat, S["vhat"], "vhat"),
            _ptr(q, S["q"], "q", optional=True), _ptr(v_old, S["v"], "v_old"), _ptr(R_q, S["R_q"], "R_q"),
            _ptr(R_v, S["R_v"], "R_v"), _ptr(R_vhat, S["R_vhat"], "R_vhat"),
            _ptr(entropy, S["entropy"], "entropy"), _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_tet_residual")

    def jvp(self, v, vhat, q, dv, dvhat, dq, JR_q, JR_v, JR_vhat, stream=None):
        """J [dq; dv; dvhat] at (q, v, vhat); q / dq None: the weak gradients."""
        S = self.shapes()
        rc = load().mehdg_tet_jvp(
            self._handle, _ptr(v, S["v"], "v"), _ptr(vhat, S["vhat"], "vhat"), _ptr(q, S["q"], "q", optional=True),
            _ptr(dv, S["v"], "dv"), _ptr(dvhat, S["vhat"], "dvhat"), _ptr(dq, S["q"], "dq", optional=True),
            _ptr(JR_q, S["R_q"], "JR_q"), _ptr(JR_v, S["R_v"], "JR_v"), _ptr(JR_vhat, S["R_vhat"], "JR_vhat"),
            _stream(stream))
        if rc:
            raise MehdgError(rc, "mehdg_tet_jvp")

    def status(self, stream=None):
        out = np.zeros(self.n_macro, dtype=np.int32)
        rc = load().mehdg_tet_status(self._handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     _stream(stream))
        return rc, out
