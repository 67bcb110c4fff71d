#!/usr/bin/env python3
"""Throughput of the per-macro-element local work of one Newton step.

One step = mehdg_assemble (residual + bordered Jacobian with Q eliminated)
+ mehdg_condense (LU of S, Ahat, bhat) + mehdg_recover (dV, dQ) over every
macro-element of the workload, inputs resident in HBM.  Default workload:
viscous Taylor-Green vortex, 16^3 macro-elements of 2x2x2 p=2 hexahedra
(4096 dense 625x625 interior blocks, 750 trace dofs each), ES flux,
Re 1600, Mach 0.1, FP64.

Prints one JSON line.  The roofline object is for the kernel with the
largest share of the timed region, from HIP events recorded by the library
around every launch on the launch's own stream.  The CPU baseline runs the
FP64 oracle on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6
FP64_VALU_PEAK_TFS = 78.6


def kernel_models(p, n_macro, NV, NH, viscous, depth=1):
    """Algorithmic work per step of each kernel slot: (kind, flops or bytes).

    Follows the blocking of the condensation: outer blocks of OB = 128
    columns made of two 64-column panels, in groups of `depth` blocks whose
    trailing update is delayed to the group's last block; inside a block the
    second panel's columns are updated after the first panel (K = 64); a
    later block of a group first takes the group's pending update of its own
    columns (update slot) and of its U rows (with the triangular solve, in
    the row-block slot); after the group the S rows right of it (K = the
    group's width); the X rows are solved afterwards, panel by panel
    (L21[:, q] = (X[:, q] - L21[:, <q] U[<q, q]) U_qq^-1), and at the end
    Ahat = A' - L21 U12 with K = N_V.  Flops count useful products only (no
    padding of tiles or of the triangular inverses).
    """
    from paper_2507_22195_amd.workloads import sizes
    s = sizes(p)
    n, nf = s["n"], s["nf"]
    COLS = NV + NH + 1
    ld = (COLS + 7) // 8 * 8
    NB, OB = 64, 128
    upd = tri = panel = trsm = 0.0
    gw = max(1, depth) * OB
    for kb0 in range(0, NV, OB):
        w = min(OB, NV - kb0)
        kg = kb0 - kb0 % gw
        kpre = kb0 - kg
        group_end = kb0 + w - kg >= gw or kb0 + w >= NV
        upd += 2.0 * kpre * (NV - kb0) * w                   # the group's pending update of this block's columns
        panels = [(kb0, min(NB, w))] + ([(kb0 + NB, w - NB)] if w > NB else [])
        for kb, nb in panels:
            # panel: rank-1 updates inside the panel columns, then the two inverses
            panel += sum(2.0 * (NV - kb - j) * (nb - j) for j in range(nb)) + 2.0 * nb ** 3 / 3.0
        if w > NB:
            o = kb0 + NB
            upd += 2.0 * NB * (NV - o) * (w - NB)            # second panel's columns, S rows
            tri += NB * NB * (w - NB)                        # its U rows (unit-lower solve)
        o = kb0 + w
        tri += w * w * (COLS - o) + 2.0 * w * kpre * (COLS - o)   # U rows right of the block
        if group_end:
            upd += 2.0 * (o - kg) * (NV - o) * (COLS - o)    # S rows right of the group
    for kq in range(0, NV, NB):
        nbq = min(NB, NV - kq)
        trsm += 2.0 * NH * nbq * kq + NH * nbq * nbq          # X rows: long-K product + U_qq^-1
    schur = 2.0 * NH * (NH + 1) * NV
    M = n_macro
    return {
        "update": ("mfma", upd * M),
        "schur": ("mfma", schur * M),
        "panel": ("alu", panel * M),
        "rowblock": ("mfma", tri * M),
        "trsm": ("mfma", trsm * M),
        # bordered rows: every entry written once
        "rows_v": ("hbm", 8.0 * NV * ld * M),
        "rows_h": ("hbm", 8.0 * NH * ld * M),
        # recovery reads U (upper half) and U12, y
        "recover": ("hbm", 8.0 * (NV * (NV + 1) / 2 + NV * (NH + 1)) * M),
        "residual": ("hbm", 8.0 * (5 * n * 2 + 30 * nf + 15 * n + 5 * n + 30 * nf) * M),
        "minv_rq": ("hbm", 8.0 * 30 * n * M),
    }


# Library slot -> kernel symbol prefix in rocprofv3 output
SLOT_KERNELS = {
    "residual": "k_residual", "minv_rq": "k_minv_rq", "rows_v": "k_rows_v", "rows_h": "k_rows_h",
    "panel": "k_panel", "rowblock": "k_tri", "update": "k_gemm<0>", "schur": "k_gemm<1>", "recover": "k_recover",
    "trsm": "k_trsm_x",
}
# source file of each slot's kernel (the HBM traffic on record is void once it changes)
SLOT_SOURCES = {
    "residual": "k_residual.hpp", "minv_rq": "k_assemble.hpp", "rows_v": "k_assemble.hpp", "rows_h": "k_assemble.hpp",
    "panel": "k_condense.hpp", "rowblock": "k_condense.hpp", "update": "k_condense.hpp", "schur": "k_condense.hpp",
    "recover": "k_recover.hpp", "trsm": "k_condense.hpp",
}
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "tgv16_p2_hbm_traffic.txt")


def source_digest(slot):
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2507_22195_amd", "csrc", SLOT_SOURCES[slot])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recorded_traffic(slot, workload):
    """HBM bytes per launch of a slot's kernel from the rocprofv3 counter summary,
    or None when there is none for this workload or the kernel source changed since."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        if not ln.startswith("traffic "):
            continue
        kv = dict(tok.split("=", 1) for tok in ln.split()[1:])
        if kv.get("slot") == slot and kv.get("workload") == workload and kv.get("source") == source_digest(slot):
            return float(kv["bytes_per_launch"])
    return None


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_s=12.0, one_core_s=6.0):
    """Oracle (FP64, numpy) assemble + condense + recover on a seeded sample of
    macros, with its BLAS on every thread it starts by default, and again on a
    smaller sample with the BLAS held to one thread."""
    from oracle import local
    from paper_2507_22195_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    rng = np.random.default_rng(99)

    def run(idx):
        ws = W.subset(w, idx)
        dvh = 1e-2 * rng.standard_normal(ws.vhat.shape)
        t0 = time.perf_counter()
        c = local.condense(ws.p, ws.mesh.h, ws.v, ws.vhat, ws.v_old, ws.params)
        local.recover(c, dvh)
        return time.perf_counter() - t0

    def measure(target):
        run(np.arange(1))                              # warm caches / BLAS threads
        per = run(np.arange(2)) / 2.0
        count = int(max(2, min(256, target / max(per, 1e-3))))
        idx = rng.choice(w.n_macro, size=count, replace=False)
        return count, run(np.sort(idx))

    count, t = measure(target_s)
    out = dict(value=count / t, unit="macro-elements/s", cores=int(threads), kind="oracle",
               cpu=cpu_model(), logical_cpus=os.cpu_count(),
               sample=f"{count} of {w.n_macro} macro-elements (seeded random), assemble+condense+recover, "
                      f"{t:.1f} s, BLAS on {threads} threads")
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            c1, t1 = measure(one_core_s)
        out["one_core"] = dict(value=c1 / t1, sample=f"{c1} macro-elements, {t1:.1f} s, BLAS on 1 thread")
    return out


def trace_solve(ctx, w, Ahat, bhat, rtol=1e-8, restart=30, maxit=300):
    """Global trace system of the step's last condensation (not part of the
    metric): F = sum P^T bhat, then GMRES(restart) with block Jacobi to rtol;
    also the bandwidth of the matrix-free K x (reads every Ahat once)."""
    import torch
    from paper_2507_22195_amd import workloads as W
    gid = W.global_face_ids(w.mesh)
    nfaces = int(gid.max()) + 1
    ctx.trace_setup(gid, nfaces)
    T = ctx.trace_shape()
    F = torch.empty(T, dtype=torch.float64, device="cuda")
    x = torch.zeros(T, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    ctx.trace_rhs(bhat, F)
    ctx.trace_apply(Ahat, F, y)                       # warm
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.trace_apply(Ahat, F, y)
    torch.cuda.synchronize()
    apply_s = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    its, rr = ctx.trace_solve(Ahat, F, x, rtol=rtol, maxit=maxit, restart=restart)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    NH, NV = ctx.sz["N_VH"], ctx.sz["N_V"]
    out = {"unknowns": int(np.prod(T)), "rtol": rtol, "restart": restart, "iterations": its,
           "relres": rr, "solve_ms": round(solve_s * 1e3, 2),
           "apply_ms": round(apply_s * 1e3, 3),
           "apply_GBps": round(8.0 * NH * NH * w.n_macro / apply_s / 1e9, 1)}
    # Algorithm 1 without Ahat: K x from the stored factors (A' x - L21 (U12 x)),
    # with GMRES and with Sec. 6.4's FGMRES + inner block-Jacobi GMRES
    ctx.trace_apply(None, F, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.trace_apply(None, F, y)
    torch.cuda.synchronize()
    mf_apply_s = (time.perf_counter() - t0) / reps
    mf = {"apply_ms": round(mf_apply_s * 1e3, 3),
          "apply_GBps": round(8.0 * (NH * NH + 2 * NV * NH) * w.n_macro / mf_apply_s / 1e9, 1)}
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_m, rr_m = ctx.trace_solve(None, F, x, rtol=rtol, maxit=maxit, restart=restart)
    torch.cuda.synchronize()
    mf["gmres"] = {"iterations": its_m, "relres": rr_m, "solve_ms": round((time.perf_counter() - t0) * 1e3, 2)}
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_f, inner_f, rr_f = ctx.trace_solve_fgmres(None, F, x, rtol=rtol, maxit=maxit, restart=restart, inner=5)
    torch.cuda.synchronize()
    mf["fgmres_inner5"] = {"outer_iterations": its_f, "inner_iterations": inner_f, "relres": rr_f,
                           "solve_ms": round((time.perf_counter() - t0) * 1e3, 2)}
    # the same with the inner iterations on single-precision copies of the
    # factors (the first solve after a condensation makes the copies)
    ctx.trace_set_inner_precision("fp32")
    f32 = {}
    for key in ("first_solve", "solve"):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its_s, inner_s, rr_s = ctx.trace_solve_fgmres(None, F, x, rtol=rtol, maxit=maxit, restart=restart, inner=5)
        torch.cuda.synchronize()
        f32[key + "_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    f32.update({"outer_iterations": its_s, "inner_iterations": inner_s, "relres": rr_s})
    mf["fgmres_inner5_fp32_factors"] = f32
    ctx.trace_set_inner_precision("fp64")
    out["matrix_free"] = mf
    return out


def differentiation(reps=5):
    """Residual JVP / VJP on the differentiation workload (8^3 macros, p = 2,
    inviscid ES, Mach 0.4; not part of the metric).  Both kernels are bound by
    reading the pointwise coefficients: algorithmic bytes per macro = the
    coefficient blocks a product reads (inviscid: the v-blocks only) + its
    inputs + its outputs, each once."""
    import torch
    from paper_2507_22195_amd import mehdg
    from paper_2507_22195_amd import workloads as W
    w = W.workload(3)
    ctx = mehdg.Context(w.p, w.mesh.h, w.params)
    S = ctx.shapes()
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    e = lambda k: torch.empty(S[k], dtype=torch.float64, device="cuda")
    v, vh, vo = dev(w.v), dev(w.vhat), dev(w.v_old)
    R_q, R_v, R_vh, ent = e("R_q"), e("R_v"), e("R_vhat"), e("entropy")
    g = torch.Generator(device="cuda").manual_seed(2)
    rnd = lambda k: torch.randn(S[k], dtype=torch.float64, device="cuda", generator=g)
    dv, dh, wv, wh = rnd("v"), rnd("vhat"), rnd("R_v"), rnd("R_vhat")
    Jq, Jv, Jh, gv, gh = e("R_q"), e("R_v"), e("R_vhat"), e("v"), e("vhat")

    def run():
        ctx.assemble(v, vh, None, vo, R_q, R_v, R_vh, ent, want_blocks=2)
        ctx.jvp(dv, dh, None, Jq, Jv, Jh)
        ctx.vjp(wv, wh, gv, gh)

    run()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    for _ in range(reps):
        run()
    prof = ctx.profile_read()
    ctx.profile(False)
    rc, _ = ctx.status()
    sz = ctx.sz
    n, nf, M = sz["n"], sz["nf"], w.n_macro
    G = (2 * (w.p + 1)) ** 3
    Sf = 6 * (2 * (w.p + 1)) ** 2
    visc = bool(w.params["viscous"])
    coef = 8 * (G * (325 if visc else 100) + Sf * (125 if visc else 50))
    io_jvp = 8 * (5 * n + 30 * nf + 15 * n + 5 * n + 30 * nf)
    io_vjp = 8 * (5 * n + 30 * nf + 5 * n + 30 * nf)
    out = {"workload": f"inviscid TGV 8x8x8 macro-elements of 2x2x2 p=2 hexahedra, ES flux, Mach 0.4",
           "n_macro": M, "status_ok": bool(rc == 0),
           "bytes_per_macro": {"jvp": coef + io_jvp, "vjp": coef + io_vjp}}
    for name, kb in (("residual", None), ("jvp", coef + io_jvp), ("vjp", coef + io_vjp)):
        ms, calls = prof[name]
        avg = ms / max(calls, 1)
        out[f"{name}_ms"] = round(avg, 4)
        if kb is not None:
            out[f"{name}_GBps"] = round(kb * M / (avg / 1e3) / 1e9, 1)
            out[f"{name}_frac_hbm"] = round(kb * M / (avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    ctx.close()
    return out


def _batch_run(degrees, steps, compare_per_degree=False):
    """A mixed-degree batch of 16^3 viscous Taylor-Green macro-elements, degrees
    drawn uniformly (seed 41) from ``degrees``, 20% with an isothermal wall on
    the -z face (seed 42): assemble + condense and recover timed apart (eager),
    and the whole step replayed from one graph."""
    import torch
    from paper_2507_22195_amd import workloads as W
    from paper_2507_22195_amd.batch import MixedBatch
    torch.cuda.empty_cache()
    p, bc, parts = W.mixed_degree_tgv(shape=(16, 16, 16), degrees=degrees, seed_p=41, wall_frac=0.2,
                                      seed_wall=42)
    h = np.empty((p.size, 3))
    for d, w in parts.items():
        h[np.nonzero(p == d)[0]] = w.mesh.h
    b = MixedBatch(p, h, parts[1].params, face_bc=bc)
    prm = parts[1].params
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    rng = np.random.default_rng(1)
    v = dev(b.pack("v", {d: w.v for d, w in parts.items()}))
    vh = dev(b.pack("vhat", {d: w.vhat for d, w in parts.items()}))
    vo = dev(b.pack("v", {d: w.v_old for d, w in parts.items()}))
    dvh = dev(b.pack("vhat", {d: 1e-2 * rng.standard_normal(w.vhat.shape) for d, w in parts.items()}))
    del parts
    out = {k: b.alloc(k) for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
    args = (v, vh, vo, out["R_q"], out["R_v"], out["R_vhat"], out["entropy"], out["Ahat"], out["bhat"], dvh,
            out["dv"], out["dq"])
    b.step(*args)                                  # workspaces
    torch.cuda.synchronize()
    ac = rec = 0.0
    for _ in range(steps):
        t0 = time.perf_counter()
        b.assemble_condense(*args[:9])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        b.recover(out["R_q"], dvh, out["dv"], out["dq"], v=v, vhat=vh, v_old=vo)
        torch.cuda.synchronize()
        ac += t1 - t0
        rec += time.perf_counter() - t1
    ac, rec = ac / steps, rec / steps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.step(*args)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    replay = (time.perf_counter() - t0) / steps
    rc, st = b.status()
    flops = 0.0
    for (d, _, c, sz) in b.groups:
        NV, NH = sz["N_V"], sz["N_VH"]
        flops += c * (2.0 / 3.0 * NV ** 3 + 2.0 * NV ** 2 * NH + 2.0 * NH ** 2 * NV)
    res = {"n_macro": b.n_macro, "macros_per_degree": {str(d): c for (d, _, c, _) in b.groups},
           "macros_per_wave": {str(d): b.waves[d] for (d, _, _, _) in b.groups},
           "wall_faces": int(bc.sum()), "status_ok": bool(rc == 0),
           "assemble_condense_ms": round(ac * 1e3, 2), "recover_ms": round(rec * 1e3, 2),
           "ms_per_step": round((ac + rec) * 1e3, 2), "graph_ms_per_step": round(replay * 1e3, 2),
           "assemble_condense_macro_per_s": round(b.n_macro / ac, 1),
           "step_macro_per_s": round(b.n_macro / min(ac + rec, replay), 1),
           "dense_condense_TFLOP/s": round(flops / ac / 1e12, 2)}
    del g
    b.close()
    if compare_per_degree:
        # the same step with one residual launch per degree instead of the persistent one
        b = MixedBatch(p, h, prm, face_bc=bc, residual_per_degree=True)
        b.step(*args)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.assemble_condense(*args[:9])
        torch.cuda.synchronize()
        res["assemble_condense_ms_residual_per_degree"] = round((time.perf_counter() - t0) / steps * 1e3, 2)
        b.close()
    del out, args, v, vh, vo, dvh
    torch.cuda.empty_cache()
    return res


def mixed_degree(steps=1):
    """The batching workload: 4096 macro-elements (16^3 viscous Taylor-Green
    box, Re 1600, Mach 0.1, ES flux) of degree drawn uniformly from {1, 2, 3, 4},
    20% with an isothermal wall, one library call per phase (not part of the
    metric).  Beside it the same box with degrees {1, 2, 3} only."""
    res = {"workload": "viscous TGV 16x16x16 macro-elements of 2x2x2 hexahedra, degree drawn uniformly from "
                       "{1, 2, 3, 4} (seed 41), isothermal wall on the -z face of 20% of them (seed 42), ES flux, "
                       "Re 1600, Mach 0.1, one Newton step (assemble + condense + recover): one batch call per "
                       "phase, each degree on a stream of its own, groups beyond the workspace budget streamed "
                       "in waves (their recovery re-forms each wave's factors)"}
    res.update(_batch_run((1, 2, 3, 4), steps))
    res["degrees_1_to_3"] = _batch_run((1, 2, 3), steps, compare_per_degree=True)
    return res


def tet_residual(reps=5):
    """Residual of tetrahedral macro-elements (mehdg_tet_residual) on the
    paper's viscous Taylor-Green mesh at p = 3: 12^3 cubes of six macro-
    tetrahedra, eight P_3 sub-tetrahedra each (84 nodes, 28 per face), KEPES
    flux, Re 1600, Mach 0.1 (not part of the metric).  Timed with HIP events
    on the launch stream; bytes per macro = inputs (v, v_old, vhat) + outputs
    (R_Q, R_V, R_Vhat, entropy), each once.  Then the reduced JVP
    (mehdg_tet_jvp, dq the weak gradient) in a seeded random direction."""
    import torch
    from paper_2507_22195_amd import mehdg
    from paper_2507_22195_amd import workloads as W
    w = W.tet_tgv_workload(shape=(12, 12, 12), p=3, M0=0.1, Re=1600.0, flux="KEPES", seed_v=61, seed_vh=62)
    ctx = mehdg.TetContext(w.p, w.mesh.X, w.params)
    S = ctx.shapes()
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    e = lambda k: torch.empty(S[k], dtype=torch.float64, device="cuda")
    v, vh, vo = dev(w.v), dev(w.vhat), dev(w.v_old)
    R_q, R_v, R_vh, ent = e("R_q"), e("R_v"), e("R_vhat"), e("entropy")
    g = torch.Generator(device="cuda").manual_seed(3)
    dv = torch.randn(S["v"], dtype=torch.float64, device="cuda", generator=g)
    dvh = torch.randn(S["vhat"], dtype=torch.float64, device="cuda", generator=g)
    Jq, Jv, Jh = e("R_q"), e("R_v"), e("R_vhat")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms = timed(lambda: ctx.residual(v, vh, None, vo, R_q, R_v, R_vh, ent))
    ms_jvp = timed(lambda: ctx.jvp(v, vh, None, dv, dvh, None, Jq, Jv, Jh))
    rc, _ = ctx.status()
    n, nf, M = ctx.sz["n"], ctx.sz["nf"], w.n_macro
    bytes_per = 8 * (2 * 5 * n + 20 * nf + 15 * n + 5 * n + 20 * nf + 1)
    ctx.close()
    return {"workload": "viscous TGV, 12x12x12 cubes of 6 tetrahedral macro-elements of 8 P_3 sub-tetrahedra, "
                        "KEPES flux, Re 1600, Mach 0.1, residual with the weak gradient",
            "n_macro": M, "status_ok": bool(rc == 0), "ms": round(ms, 4),
            "macro_per_s": round(M / (ms / 1e3), 1), "bytes_per_macro": bytes_per,
            "GBps": round(bytes_per * M / (ms / 1e3) / 1e9, 1),
            "jvp_ms": round(ms_jvp, 4), "jvp_macro_per_s": round(M / (ms_jvp / 1e3), 1)}


def tet_step(reps=2, shape=(6, 6, 6)):
    """Local work of one Newton step on tetrahedral macro-elements (not part of
    the metric): viscous Taylor-Green, cubes of six macro-tetrahedra of eight
    P_3 sub-tetrahedra, KEPES flux, Re 1600, Mach 0.1; assemble (residual and
    bordered matrices from reduced-Jacobian columns), condense, recover, each
    timed with HIP events on the launch stream.  Dense work of the
    condensation per macro: 2/3 N_V^3 + 2 N_V^2 N_VH + 2 N_VH^2 N_V."""
    import torch
    from paper_2507_22195_amd import mehdg
    from paper_2507_22195_amd import workloads as W
    w = W.tet_tgv_workload(shape=shape, p=3, M0=0.1, Re=1600.0, flux="KEPES", seed_v=61, seed_vh=62)
    ctx = mehdg.TetContext(w.p, w.mesh.X, w.params)
    S = ctx.shapes()
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    e = {k: torch.empty(S[k], dtype=torch.float64, device="cuda")
         for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat", "dv", "dq")}
    v, vh, vo = dev(w.v), dev(w.vhat), dev(w.v_old)
    dvh = dev(1e-2 * np.random.default_rng(1).standard_normal(w.vhat.shape))
    calls = {"assemble": lambda: ctx.assemble(v, vh, vo, e["R_q"], e["R_v"], e["R_vhat"], e["entropy"]),
             "condense": lambda: ctx.condense(e["Ahat"], e["bhat"]),
             "recover": lambda: ctx.recover(e["R_q"], dvh, e["dv"], e["dq"])}
    for f in calls.values():
        f()
    torch.cuda.synchronize()
    ms = {k: 0.0 for k in calls}
    for _ in range(reps):
        for k, f in calls.items():
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            f()
            b.record()
            torch.cuda.synchronize()
            ms[k] += a.elapsed_time(b) / reps
    rc, _ = ctx.status()
    M, NV, NH = w.n_macro, ctx.sz["N_V"], ctx.sz["N_VH"]
    total = sum(ms.values())
    flops = M * (2.0 / 3.0 * NV ** 3 + 2.0 * NV ** 2 * NH + 2.0 * NH ** 2 * NV)
    ctx.close()
    return {"workload": f"viscous TGV, {shape[0]}x{shape[1]}x{shape[2]} cubes of 6 tetrahedral macro-elements of 8 "
                        "P_3 sub-tetrahedra (84 nodes, N_V 420, N_VH 560), KEPES flux, Re 1600, Mach 0.1, one "
                        "Newton step (assemble + condense + recover)",
            "n_macro": M, "status_ok": bool(rc == 0), "ms_per_step": round(total, 2),
            "ms": {k: round(x, 2) for k, x in ms.items()},
            "macro_per_s": round(M / (total / 1e3), 1),
            "condense_TFLOP/s": round(flops / (ms["condense"] / 1e3) / 1e12, 2)}


def precision(steps=2, shape=None, sample=64):
    """Mixed precision against FP64 on the precision workload (16x16x8 macros of
    2x2x2 p = 3 hexahedra, KEPES, viscous, Re 5000, Mach 0.3): the metric's
    assemble + condense time per precision mode and the mixed-vs-FP64 speedup;
    the recovery beside it; refinement steps; the largest per-macro normwise
    relative difference to the FP64 result of bhat and dV (every macro) and of
    Ahat (a seeded sample of macros; its FP64 copy for all would not fit)."""
    import torch
    from paper_2507_22195_amd import mehdg
    from paper_2507_22195_amd import workloads as W
    torch.cuda.empty_cache()
    w = W.workload(5, shape=shape)
    ctx = mehdg.Context(w.p, w.mesh.h, w.params)
    S = ctx.shapes()
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    e = lambda k: torch.empty(S[k], dtype=torch.float64, device="cuda")
    v, vh, vo = dev(w.v), dev(w.vhat), dev(w.v_old)
    dvh = dev(1e-2 * np.random.default_rng(1).standard_normal(w.vhat.shape))
    R_q, R_v, R_vh, ent = e("R_q"), e("R_v"), e("R_vhat"), e("entropy")
    Ahat, bhat, dv, dq = e("Ahat"), e("bhat"), e("dv"), e("dq")
    M = w.n_macro
    idx = torch.tensor(np.sort(np.random.default_rng(77).choice(M, min(sample, M), replace=False)), device="cuda")
    NV, NH = ctx.sz["N_V"], ctx.sz["N_VH"]
    out = {"workload": f"viscous TGV, {w.mesh.shape[0]}x{w.mesh.shape[1]}x{w.mesh.shape[2]} macro-elements of "
                       f"2x2x2 p={w.p} hexahedra (N_V {NV}, N_VH {NH}), KEPES flux, Re 5000, Mach 0.3",
           "n_macro": M, "ir_tol": mehdg.IR_TOL, "ir_maxit": mehdg.IR_MAXIT}
    ref = None

    def relmax(a, b):
        a, b = a.reshape(a.shape[0], -1), b.reshape(b.shape[0], -1)
        return float(((a - b).norm(dim=1) / b.norm(dim=1)).max())

    for prec in ("fp64", "fp32", "bf16"):
        ctx.assemble(v, vh, None, vo, R_q, R_v, R_vh, ent, want_blocks=True)
        ctx.condense(Ahat, bhat, prec=prec)
        ctx.recover(R_q, dvh, dv, dq)
        torch.cuda.synchronize()
        ctx.status()
        ctx.profile(True)
        ctx.profile_read()
        t_ac = t_rec = 0.0
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.assemble(v, vh, None, vo, R_q, R_v, R_vh, ent, want_blocks=True)
            ctx.condense(Ahat, bhat, prec=prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx.recover(R_q, dvh, dv, dq)
            torch.cuda.synchronize()
            t_ac += t1 - t0
            t_rec += time.perf_counter() - t1
        prof = ctx.profile_read()
        ctx.profile(False)
        rc, st = ctx.status()
        ms = t_ac * 1e3 / steps
        entry = {"assemble_condense_ms": round(ms, 2), "macro_per_s": round(M / (ms / 1e3), 1),
                 "recover_ms": round(t_rec * 1e3 / steps, 2), "status_ok": bool(rc == 0),
                 "flagged": {mehdg.ERRORS.get(int(c), int(c)): int((st == c).sum()) for c in np.unique(st) if c},
                 "kernels_ms": {k: round(m_ / steps, 2) for k, (m_, n_) in prof.items() if n_}}
        if prec == "fp64":
            ref = dict(Ahat=Ahat[idx].clone(), bhat=bhat.clone(), dv=dv.clone())
        else:
            entry["ir_steps"] = ctx.ir_iterations()
            entry["speedup_vs_fp64"] = round(out["fp64"]["assemble_condense_ms"] / ms, 3)
            ok = torch.isfinite(bhat).all(dim=1)
            entry["max_rel_diff_vs_fp64"] = {
                "Ahat": relmax(Ahat[idx], ref["Ahat"]) if bool(ok[idx].all()) else None,
                "bhat": relmax(bhat[ok], ref["bhat"][ok]) if bool(ok.any()) else None,
                "dv": relmax(dv[ok], ref["dv"][ok]) if bool(ok.any()) else None}
        out[{"fp64": "fp64", "fp32": "fp32_ir", "bf16": "bf16_ir"}[prec]] = entry
    ctx.close()
    del Ahat, bhat, dv, dq, R_q, R_v, R_vh, ent, ref
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--shape", type=int, nargs=3, default=None, help="macro grid (default 16 16 16)")
    ap.add_argument("--no-trace", action="store_true", help="skip the global trace solve measurement")
    ap.add_argument("--no-diff", action="store_true", help="skip the JVP / VJP measurement")
    ap.add_argument("--diff-only", action="store_true", help="only the JVP / VJP measurement (profiling)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-degree measurement")
    ap.add_argument("--mixed-only", action="store_true", help="only the mixed-degree measurement (profiling)")
    ap.add_argument("--no-tet", action="store_true", help="skip the tetrahedral residual measurement")
    ap.add_argument("--tet-only", action="store_true", help="only the tetrahedral residual measurement")
    ap.add_argument("--config", type=int, default=2, choices=(2, 5),
                    help="2: viscous TGV 16^3, p=2, ES (default); 5: viscous TGV 16x16x8, p=3, KEPES, Re 5000, "
                         "Mach 0.3 (the FP64 path of the precision workload)")
    ap.add_argument("--no-precision", action="store_true", help="skip the mixed-precision measurement")
    ap.add_argument("--precision-only", action="store_true", help="only the mixed-precision measurement")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="before warm-up, copy a MIB-sized buffer three times (untimed) so that a counter "
                         "run sees a plain copy kernel of known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the per-macro local work would shard by macro-element, "
                                   "one contiguous range of macros per GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2507_22195_amd import mehdg
    from paper_2507_22195_amd import workloads as W

    if args.mixed_only:
        print(json.dumps({"mixed_degree": mixed_degree()}), flush=True)
        return
    if args.diff_only:
        print(json.dumps({"differentiation": differentiation(reps=args.steps)}), flush=True)
        return
    if args.precision_only:
        print(json.dumps({"mixed": precision(steps=args.steps)}), flush=True)
        return
    if args.tet_only:
        print(json.dumps({"tet_residual": tet_residual(reps=args.steps), "tet_step": tet_step()}), flush=True)
        return
    w = W.workload(args.config, shape=tuple(args.shape) if args.shape else None)
    ctx = mehdg.Context(w.p, w.mesh.h, w.params)
    S = ctx.shapes()
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    v, vh, vo = dev(w.v), dev(w.vhat), dev(w.v_old)
    rng = np.random.default_rng(1)
    dvh = dev(1e-2 * rng.standard_normal(w.vhat.shape))
    e = lambda k: torch.empty(S[k], dtype=torch.float64, device="cuda")
    R_q, R_v, R_vh, ent = e("R_q"), e("R_v"), e("R_vhat"), e("entropy")
    Ahat, bhat, dv, dq = e("Ahat"), e("bhat"), e("dv"), e("dq")

    if args.copy_calib > 0:
        src = torch.ones(args.copy_calib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        ctx.assemble(v, vh, None, vo, R_q, R_v, R_vh, ent, want_blocks=True)
        ctx.condense(Ahat, bhat)
        ctx.recover(R_q, dvh, dv, dq)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rc, st = ctx.status()
    if rc != 0:
        print(json.dumps({"error": f"device status {rc} on {int((st != 0).sum())} macro-elements"}))
        sys.exit(1)
    ctx.profile(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    rc, st = ctx.status()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # the same step captured once in a HIP graph and replayed
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        step()
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    del graph
    M = w.n_macro
    value = M / (ms_per_step / 1e3)
    sz = ctx.sz
    NV, NH = sz["N_V"], sz["N_VH"]

    models = kernel_models(w.p, M, NV, NH, w.params["viscous"], depth=ctx.get_lu_depth())
    kernels = {}
    for name, (ms, calls) in prof.items():
        if calls == 0:
            continue
        kind, work = models[name]
        per_step_ms = ms / args.steps
        entry = {"ms_per_step": round(per_step_ms, 4), "launches_per_step": calls // args.steps,
                 "avg_launch_ms": round(ms / calls, 5)}
        if kind == "hbm":
            entry["GB/s"] = round(work / (per_step_ms / 1e3) / 1e9, 1)
        else:
            entry["TFLOP/s"] = round(work / (per_step_ms / 1e3) / 1e12, 2)
        kernels[name] = entry
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kind, work = models[dom]
    dom_ms = kernels[dom]["ms_per_step"]
    calls = max(1, kernels[dom]["launches_per_step"])
    if kind == "hbm":
        achieved = work / (dom_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    else:
        achieved = work / (dom_ms / 1e3) / 1e12
        peak = FP64_MFMA_PEAK_TFS if kind == "mfma" else FP64_VALU_PEAK_TFS
        roof = {"bound": "mfma" if kind == "mfma" else "alu", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None}
    wl = f"tgv{w.mesh.shape[0]}x{w.mesh.shape[1]}x{w.mesh.shape[2]}_p{w.p}"
    flux_name = ("EC", "ES", "KEPES")[int(w.params["flux"])]
    re_, m0 = (1600.0, 0.1) if args.config == 2 else (5000.0, 0.3)
    tb = recorded_traffic(dom, wl)
    # HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated), and the rate it implies
    roof["traffic"] = None if tb is None else round(tb)
    if tb is not None:
        roof["traffic_GBps"] = round(tb / (dom_ms / calls / 1e3) / 1e9, 1)
    roof["kernel"] = SLOT_KERNELS[dom]
    roof["work_per_launch"] = work / calls
    # whole condensation against the dense algorithmic count (2/3 N^3 + 2 N^2 M + 2 M^2 N per macro)
    cond_ms = sum(kernels[k]["ms_per_step"] for k in ("panel", "rowblock", "update", "schur", "trsm")
                  if k in kernels)
    cond_flops = M * (2.0 / 3.0 * NV ** 3 + 2.0 * NV ** 2 * NH + 2.0 * NH ** 2 * NV)
    out = {
        "metric": "macro-elements/s for assemble+condense; mixed vs FP64 at 1e-10 rel err",
        "value": round(value, 1),
        "unit": "macro-elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"viscous TGV, {w.mesh.shape[0]}x{w.mesh.shape[1]}x{w.mesh.shape[2]} macro-elements "
                               f"of 2x2x2 p={w.p} hexahedra, {flux_name} flux, Re {re_:g}, Mach {m0:g}, one Newton "
                               f"step (assemble + condense + recover)",
                   "n_macro": M, "p": w.p, "N_V": NV, "N_VH": NH, "flux": flux_name, "viscous": True},
        "dof_per_s": round(value * (NV + sz["N_Q"]), 1),
        "graph_ms_per_step": round(graph_ms, 3),
        "status_ok": bool(rc == 0),
        "roofline": roof,
        "condense": {"ms_per_step": round(cond_ms, 3),
                     "TFLOP/s": round(cond_flops / (cond_ms / 1e3) / 1e12, 2),
                     "frac_fp64_peak": round(cond_flops / (cond_ms / 1e3) / 1e12 / FP64_MFMA_PEAK_TFS, 4)},
        "kernels": kernels,
    }
    if not args.no_trace:
        out["trace_solve"] = trace_solve(ctx, w, Ahat, bhat)
    ctx.close()
    del Ahat, bhat, dv, dq, R_q, R_v, R_vh, ent
    torch.cuda.empty_cache()
    if not args.no_precision:
        out["mixed"] = precision()
    if not args.no_diff:
        out["differentiation"] = differentiation()
    if not args.no_mixed:
        out["mixed_degree"] = mixed_degree()
    if not args.no_tet:
        out["tet_residual"] = tet_residual()
        out["tet_step"] = tet_step()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
