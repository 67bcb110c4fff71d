"""Autotuner of the FP64 condensation: tile shapes and LU update depth.

The library carries a fixed list of tile shapes for its batched products
(``mehdg.tile_variants()``) and two call sites that take one: the trailing
updates of the LU of S and the Schur product [Ahat | bhat] = [A' | r_hat] -
L21 [U12 | y] (Sec. 6.2).  It also groups the outer blocks of the LU for
delayed trailing updates (``Context.set_lu_depth``).  The choices per degree
are compiled into the library from ``csrc/tile_table.hpp``; this module makes
that table:

* ``sweep`` times every variant at every site on the device, on the viscous
  Taylor-Green batch of each degree (16^3 macro-elements at p = 1 and 2,
  16 x 16 x 8 at p = 3, 4^3 at p = 4, whose 295 MB bordered matrices allow
  no more in one context beside the others), with the library's own per-site event timers
  (``mehdg_profile_read``), best of ``reps`` condensations each after a fresh
  assembly.  Every variant must give the same bits as variant 0 (the
  shapes add the products of one output element in the same order): the
  sweep checks a 64-bit wrap-around sum of Ahat's bit patterns against
  variant 0's and refuses a variant that differs.  Then, with the fastest
  variants, it times the whole condensation (the sum of its kernels' event
  times) at each depth of ``DEPTHS`` up to the degree's block count; a depth
  changes the rounding, so its Ahat must agree with depth 1's to 1e-12
  (relative, Frobenius) or the depth is refused.
* ``render`` turns a sweep's result into the header: the fastest variant per
  degree and site and the fastest depth per degree, with every measured time
  in its comments.

    python -m paper_2507_22195_amd.autotune --sweep --out sweep.json     (device)
    python -m paper_2507_22195_amd.autotune --render sweep.json          (writes the header)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import mehdg
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "tile_table.hpp")
SHAPES = {1: (16, 16, 16), 2: (16, 16, 16), 3: (16, 16, 8), 4: (4, 4, 4)}
DEPTHS = (1, 2, 3, 4, 7, 1024)
OB = 128          # columns per outer block of the LU of S


def _bits_sum(t) -> int:
    """Sum of the 64-bit patterns of a float64 device tensor, mod 2^64."""
    import torch
    return int(t.view(torch.int64).sum().item())


def sweep_degree(p: int, shape=None, reps: int = 2, log=print) -> dict:
    import torch
    shape = shape or SHAPES[p]
    w = W.tgv_workload(shape=shape, p=p, M0=0.1, Re=1600.0, flux="ES", seed_v=21, seed_vh=22)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    ctx = mehdg.Context(p, w.mesh.h, w.params)
    S = ctx.shapes()
    v, vh, vo = dev(w.v), dev(w.vhat), dev(w.v_old)
    del w
    out = {k: torch.empty(S[k], dtype=torch.float64, device="cuda")
           for k in ("R_q", "R_v", "R_vhat", "entropy", "Ahat", "bhat")}
    variants = mehdg.tile_variants()
    res = {"p": p, "shape": list(shape), "n_macro": ctx.n_macro, "reps": reps, "sites": {}}

    def run():
        ctx.assemble(v, vh, None, vo, out["R_q"], out["R_v"], out["R_vhat"], out["entropy"], want_blocks=True)
        torch.cuda.synchronize()
        ctx.profile_read()                 # drop the assembly's times
        ctx.condense(out["Ahat"], out["bhat"])
        torch.cuda.synchronize()
        return ctx.profile_read()

    ctx.profile(True)
    run()                                  # workspaces, first-launch costs
    ref = None
    for site in mehdg.TILE_SITES:
        times = {}
        for i in range(len(variants)):
            ctx.set_tile(site, i)
            best = float("inf")
            for _ in range(reps):
                best = min(best, run()[site][0])
            rc, st = ctx.status()
            if rc:
                raise RuntimeError(f"p={p} site {site} variant {i}: status {mehdg.ERRORS.get(rc, rc)}")
            chk = _bits_sum(out["Ahat"]) ^ _bits_sum(out["bhat"])
            if ref is None:
                ref = chk
            same = chk == ref
            times[i] = {"ms": round(best, 4), "same_bits": bool(same)}
            log(f"  p={p} {site:6s} variant {i} {variants[i]['TM']}x{variants[i]['TN']}/{variants[i]['KC']}: "
                f"{best:9.3f} ms  {'ok' if same else 'DIFFERENT BITS'}")
        ctx.set_tile(site, 0)
        res["sites"][site] = times
    # LU update depth, with the fastest bit-identical variants
    for site, times in res["sites"].items():
        ok = {int(i): t["ms"] for i, t in times.items() if t["same_bits"]}
        ctx.set_tile(site, min(ok, key=ok.get) if ok else 0)
    nblk = (ctx.sz["N_V"] + OB - 1) // OB
    depths = sorted({min(d, nblk) for d in DEPTHS})
    res["nblk"] = nblk
    res["depths"] = {}
    a1 = None
    for d in depths:
        ctx.set_lu_depth(d)
        best = float("inf")
        for _ in range(reps):
            best = min(best, sum(ms for ms, calls in run().values() if calls))
        rc, st = ctx.status()
        if rc:
            raise RuntimeError(f"p={p} depth {d}: status {mehdg.ERRORS.get(rc, rc)}")
        if a1 is None:
            a1 = out["Ahat"].clone()
        dev_rel = float(((out["Ahat"] - a1).norm() / a1.norm()).item())
        ok = dev_rel < 1e-12
        res["depths"][str(d)] = {"ms": round(best, 3), "rel_to_depth1": dev_rel, "ok": ok}
        log(f"  p={p} depth {d:2d}: {best:9.2f} ms per condensation  (Ahat vs depth 1: {dev_rel:.1e})"
            + ("" if ok else "  REFUSED"))
    ctx.set_lu_depth(0)
    ctx.close()
    return res


def sweep(degrees=(1, 2, 3, 4), reps: int = 2, log=print) -> dict:
    import torch
    out = {"device": torch.cuda.get_device_name(0), "variants": mehdg.tile_variants(), "degrees": {}}
    for p in degrees:
        t0 = time.perf_counter()
        out["degrees"][str(p)] = sweep_degree(p, reps=reps, log=log)
        log(f"p={p} swept in {time.perf_counter() - t0:.1f} s")
        torch.cuda.empty_cache()
    return out


def pick(res: dict) -> dict:
    """Fastest bit-identical variant per degree and site, and fastest accepted depth."""
    table = {}
    for p, r in res["degrees"].items():
        table[int(p)] = {}
        for site, times in r["sites"].items():
            ok = {int(i): t["ms"] for i, t in times.items() if t["same_bits"]}
            table[int(p)][site] = min(ok, key=ok.get) if ok else 0
        dep = {int(d): t["ms"] for d, t in r.get("depths", {}).items() if t["ok"]}
        table[int(p)]["depth"] = min(dep, key=dep.get) if dep else 1
    return table


def render(res: dict) -> str:
    table = pick(res)
    var = res["variants"]
    lines = [
        "// Tile variant of the batched FP64 MFMA products per degree p (row) and call",
        "// site (column: trailing update, Schur product), indices into the variant",
        "// list of k_condense.hpp, and outer blocks per group of delayed trailing",
        "// updates of the LU of S per degree.  Written by `python -m",
        "// paper_2507_22195_amd.autotune --render`; edit by rerunning the sweep, not",
        "// by hand.",
        "//",
        f"// sweep on {res['device']}: milliseconds per condensation spent at the site,",
        "// best of the repetitions, viscous Taylor-Green batch of each degree; then,",
        "// with the fastest variants, milliseconds per condensation (all its kernels)",
        "// at each depth",
    ]
    for p, r in sorted(res["degrees"].items()):
        lines.append(f"//   p = {p}, {r['n_macro']} macro-elements ({'x'.join(map(str, r['shape']))}):")
        for site, times in r["sites"].items():
            cells = []
            for i, t in sorted(times.items(), key=lambda kv: int(kv[0])):
                v = var[int(i)]
                cells.append(f"{i}:{v['TM']}x{v['TN']}/{v['KC']} {t['ms']:.2f}" + ("" if t["same_bits"] else "!"))
            lines.append(f"//     {site:6s} " + ", ".join(cells))
        if r.get("depths"):
            cells = [f"{d}:{t['ms']:.1f}" + ("" if t["ok"] else "!")
                     for d, t in sorted(r["depths"].items(), key=lambda kv: int(kv[0]))]
            lines.append(f"//     depth  ({r['nblk']} blocks) " + ", ".join(cells))
    lines += ["#pragma once", "", "namespace mehdg {", "constexpr int kTileTable[5][2] = {",
              "    {0, 0},   // (unused)"]
    for p in (1, 2, 3, 4):
        row = table.get(p)
        if row is None:
            lines.append(f"    {{0, 0}},   // p = {p} (not swept)")
        else:
            lines.append(f"    {{{row['update']}, {row['schur']}}},   // p = {p}")
    lines += ["};", "constexpr int kLuDepth[5] = {1"]
    for p in (1, 2, 3, 4):
        row = table.get(p)
        lines[-1] += f", {row['depth'] if row else 1}"
    lines[-1] += "};   // (unused), p = 1, 2, 3, 4"
    lines += ["}  // namespace mehdg", ""]
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sweep", action="store_true", help="time every variant on the device")
    ap.add_argument("--degrees", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default=None, help="sweep result (JSON)")
    ap.add_argument("--render", default=None, metavar="JSON", help="write the table header from a sweep")
    a = ap.parse_args(argv)
    if a.sweep:
        res = sweep(tuple(a.degrees), a.reps, log=lambda s: print(s, flush=True))
        txt = json.dumps(res, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(txt)
        else:
            print(txt)
    if a.render:
        with open(a.render) as f:
            res = json.load(f)
        with open(TABLE, "w") as f:
            f.write(render(res))
        print(f"wrote {TABLE}: {pick(res)}")
    if not a.sweep and not a.render:
        ap.print_help()
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main())
