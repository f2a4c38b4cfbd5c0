"""Autotuner of the projector pair's launch shapes.

For each level of a geometry it times, with the library's own kernel timer
(imask_time_kernel: HIP events around the exact launches a step makes), every
candidate transpose tile (rows per wavefront x wavefronts) and workgroup
target, with the ordered sum of the partial images it writes (more angle
groups make the transpose faster and the sum slower), then every forward
band budget, and keeps the fastest.  The table
is saved as JSON keyed by "N_l x angles x bins" and applied with
imask_set_tiles.  Shapes change only the order of floating-point sums, never
the matrices, so any table gives a correct projector.

Usage (on the GPU):
  python -m paper_2412_10249_amd.autotune            # the default geometries below
  python -m paper_2412_10249_amd.autotune --geometry 512x720x768
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

from . import _abi
from ._abi import check, lib

PKG = os.path.dirname(os.path.abspath(__file__))
TILES_JSON = os.path.join(PKG, "tiles.json")

BP_SHAPES = [(2, 8), (4, 4), (2, 4), (1, 4)]
BP_TARGETS = [512, 1024, 2048, 4096]
FWD_BUDGETS_KB = [64, 78, 96, 128, 156]


def key(nl: int, na: int, nd: int) -> str:
    return f"{nl}x{na}x{nd}"


def set_tiles(nl: int, na: int, nd: int, bp=(0, 0), bp_wg: int = 0, fwd_lds_kb: int = 0) -> None:
    t = _abi.Tiles(bp[0], bp[1], bp_wg, fwd_lds_kb)
    check(lib().imask_set_tiles(nl, na, nd, ctypes.byref(t)), "imask_set_tiles")


def reset_tiles(nl: int, na: int, nd: int) -> None:
    check(lib().imask_set_tiles(nl, na, nd, None), "imask_set_tiles")


def get_tiles(nl: int, na: int, nd: int) -> dict:
    t = _abi.Tiles()
    check(lib().imask_get_tiles(nl, na, nd, ctypes.byref(t)), "imask_get_tiles")
    return {"bp": [t.bp_rows, t.bp_waves], "bp_wg": t.bp_wg, "fwd_lds_kb": t.fwd_lds_kb}


def default_fwd_kb(nl: int) -> int:
    """The forward's default band budget (a tuned one may only be larger)."""
    return 156 if nl >= 512 else 78 if nl >= 256 else 64


def tune_geometry(n: int, na: int, nd: int, levels=(0, 1, 2, 3), reps: int = 10, log=print) -> dict:
    """Fastest shapes of each level of the n x n, na x nd parallel geometry."""
    import torch

    from ._abi import KERNEL_FORWARD, KERNEL_TRANSPOSE_SUM
    from .imask import Geometry, time_kernel, workspace

    geom = Geometry(n, na, nd)
    work = workspace(geom)
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.rand((n, n), device="cuda", generator=gen)
    y = torch.rand((na, nd), device="cuda", generator=gen)
    out = {}
    for lvl in levels:
        nl = n >> lvl
        if nl < 2:
            continue
        reset_tiles(nl, na, nd)
        base_bp = time_kernel(geom, KERNEL_TRANSPOSE_SUM, lvl, y, work, reps)
        base_fwd = time_kernel(geom, KERNEL_FORWARD, lvl, x, work, reps)
        best_bp = (base_bp, (0, 0), 0)
        for shape in BP_SHAPES:
            for wg in BP_TARGETS:
                set_tiles(nl, na, nd, shape, wg)
                t = time_kernel(geom, KERNEL_TRANSPOSE_SUM, lvl, y, work, reps)
                if t < best_bp[0]:
                    best_bp = (t, shape, wg)
        best_fwd = (base_fwd, 0)
        if nl <= 1024:  # larger levels use the direct forward (no bands)
            for kb in FWD_BUDGETS_KB:
                if kb < default_fwd_kb(nl):
                    continue
                set_tiles(nl, na, nd, best_bp[1], best_bp[2], kb)
                t = time_kernel(geom, KERNEL_FORWARD, lvl, x, work, reps)
                if t < best_fwd[0]:
                    best_fwd = (t, kb)
        set_tiles(nl, na, nd, best_bp[1], best_bp[2], best_fwd[1])
        ent = {"bp": list(best_bp[1]), "bp_wg": best_bp[2], "fwd_lds_kb": best_fwd[1],
               "transpose_sum_us": {"default": round(base_bp * 1e6, 2), "tuned": round(best_bp[0] * 1e6, 2)},
               "forward_us": {"default": round(base_fwd * 1e6, 2), "tuned": round(best_fwd[0] * 1e6, 2)}}
        out[key(nl, na, nd)] = ent
        log(f"N_l {nl} ({na} x {nd}): transpose + sum {ent['transpose_sum_us']} with {ent['bp']} wg {ent['bp_wg']}; "
            f"forward {ent['forward_us']} with {ent['fwd_lds_kb']} KB")
    del work
    return out


def apply(table: dict) -> int:
    """Set every entry of a tuned table; returns how many were applied."""
    for k, ent in table.items():
        nl, na, nd = (int(v) for v in k.split("x"))
        set_tiles(nl, na, nd, tuple(ent.get("bp", (0, 0))), int(ent.get("bp_wg", 0)), int(ent.get("fwd_lds_kb", 0)))
    return len(table)


def reset(table: dict) -> None:
    for k in table:
        nl, na, nd = (int(v) for v in k.split("x"))
        reset_tiles(nl, na, nd)


def load(path: str = TILES_JSON) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f).get("tiles", {})


def apply_saved(path: str = TILES_JSON) -> int:
    return apply(load(path))


# The geometries tuned by default: the 512^2 / 720 x 768 workload and the
# batched workload's grids (angles = bins = 1.5 N).
DEFAULT_GEOMETRIES = ["512x720x768"] + [f"{n}x{3 * n // 2}x{3 * n // 2}" for n in (256, 384, 512, 768, 1024)]


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--geometry", nargs="+", default=DEFAULT_GEOMETRIES, help="N x angles x bins, e.g. 512x720x768")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=TILES_JSON)
    args = ap.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    table = {}
    for geo in args.geometry:
        n, na, nd = (int(v) for v in geo.split("x"))
        print(f"tuning {n}^2, {na} x {nd}", flush=True)
        table.update(tune_geometry(n, na, nd, reps=args.reps, log=lambda m: print(m, flush=True)))
    doc = {"device": torch.cuda.get_device_name(0), "arch": torch.cuda.get_device_properties(0).gcnArchName,
           "command": "python -m paper_2412_10249_amd.autotune " + " ".join(argv if argv is not None else sys.argv[1:]),
           "tiles": table}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {len(table)} entries to {args.out}", flush=True)


if __name__ == "__main__":
    main()
