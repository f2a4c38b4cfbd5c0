"""ImaSk throughput on one MI355X (epochs/s) for the 512x512 smoothed-TV workload.

One step = one iteration of Alg. 1 (draw, restriction, forward projection,
dual update, backprojection, prolongation, primal update, smoothed-TV prox)
on a 512 x 512 random-ellipse phantom with 720 angles x 768 bins, Poisson
I0 = 1e5, smoothed TV (eps = 1e-3) + lambda = 1e-3, levels 512/256/128/64
with p = 1/4 (the paper's literal construction, PAPER mode).  Epochs count
equivalent full-resolution operator applications (cost 2^{-l} per step).

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, NA, ND = 512, 720, 768
I0 = 1e5
LEVELS = (0, 1, 2, 3)
LAM, TV_W, TV_EPS, TV_J = 1e-3, 2e-4, 1e-3, 10
SIGMA = 1e-3
SEED, STREAM = 42, 0
# Joseph sample arithmetic counted per (ray, step) sample: the right-tap
# weight (1 - w) and two fused multiply-adds into the accumulator.
FLOP_PER_SAMPLE = 5
PEAK_FP32_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def sample_counts(n, na, nd, lvl):
    """Samples (ray, step) with a tap inside the level-l image (geometry only)."""
    nl = n >> lvl
    h = 2.0 / nl
    th = np.arange(na) * np.pi / na
    s = (np.arange(nd) - (nd - 1) / 2.0) * (2.0 / n)
    rows = (4 * np.arange(na) <= na) | (4 * np.arange(na) >= 3 * na)
    c0 = -1.0 + 0.5 * h
    total = 0
    k = -1.0 + (np.arange(nl) + 0.5) * h
    for a in range(na):
        ct, st = np.cos(th[a]), np.sin(th[a])
        if rows[a]:
            u = ((s[:, None] - k[None, :] * st) / ct - c0) / h
        else:
            u = ((s[:, None] - k[None, :] * ct) / st - c0) / h
        q = np.floor(u)
        total += int(np.count_nonzero((q >= -1) & (q < nl)))
    return total


def cpu_baseline(b, budget_s=12.0):
    """The FP64 oracle running the same iteration on the host cores."""
    import oracle

    g = oracle.Geometry(N, NA, ND)
    lv = oracle.Levels(list(LEVELS), [1.0 / len(LEVELS)] * len(LEVELS))
    reg = oracle.Reg(oracle.REG_SMOOTH_TV, lam=LAM, tv_weight=TV_W, tv_eps=TV_EPS, tv_inner=TV_J)
    st = None
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        st = oracle.imask_run(g, lv, reg, SIGMA, SEED, STREAM, b, 1, st)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": st.epochs / el, "unit": "epochs/s", "cores": cores, "kind": "oracle",
            "sample": f"first {st.k} ImaSk iterations ({st.epochs:.3f} epochs) of the same workload, FP64, "
                      f"{el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path does not shard "
              f"across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_10249_amd as pk
    import synth

    torch.cuda.set_device(0)
    _, b = synth.ct_problem(N, NA, ND, I0, 1000, 2000)
    b32 = torch.from_numpy(b.astype(np.float32)).cuda()
    geom = pk.Geometry(N, NA, ND)
    lv = pk.Levels.uniform(LEVELS, pk.FULL_PAPER)
    reg = pk.Regularizer(pk.REG_SMOOTH_TV, LAM, TV_W, TV_EPS, TV_J)
    prob = pk.Problem(geom, lv, reg, pk.Params(SIGMA, SEED, STREAM), b32)

    prob.step(args.warmup)
    torch.cuda.synchronize()
    k0, e0 = prob.k, prob.epochs
    t0 = time.perf_counter()
    prob.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    epochs = prob.epochs - e0
    assert torch.isfinite(prob.x_cur).all(), "non-finite iterate"
    draws = pk.draws(prob.params, lv, k0, args.steps)
    mix = np.bincount(draws, minlength=len(LEVELS)) / args.steps

    # per-kernel durations of the projector pair, HIP events on the stream
    # the kernels run on (torch's current stream, which the library uses)
    work = prob.work
    x = prob.x_cur.clone()
    y = prob.y_cur.clone()
    sino = torch.empty((NA, ND), device="cuda")
    img = torch.empty((N, N), device="cuda")
    stream = torch.cuda.current_stream()
    kern = {}
    for lvl in LEVELS:
        for name, fn in (("fwd", lambda: pk.project(geom, lvl, x, work, sino)),
                         ("bp", lambda: pk.backproject(geom, lvl, y, work, img))):
            fn()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(args.kernel_reps):
                fn()
            ev1.record(stream)
            torch.cuda.synchronize()
            kern[(name, lvl)] = ev0.elapsed_time(ev1) / 1e3 / args.kernel_reps
    samples = {lvl: sample_counts(N, NA, ND, lvl) for lvl in LEVELS}
    # dominant kernel: largest expected time share per step under p
    share = {key: t * (1.0 / len(LEVELS)) for key, t in kern.items()}
    dom = max(share, key=share.get)
    dom_t = kern[dom]
    achieved = samples[dom[1]] * FLOP_PER_SAMPLE / dom_t / 1e12
    proj_pair_sps = {f"l{lvl}": samples[lvl] * 2 / (kern[("fwd", lvl)] + kern[("bp", lvl)]) for lvl in LEVELS}

    out = {
        "metric": "ImaSk epochs/s (512x512 smoothed-TV race workload)",
        "value": epochs / el,
        "unit": "epochs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded random-ellipse phantom, analytic line integrals, Poisson I0=1e5",
        "config": {"workload": "2D parallel-beam CT 512x512, 720 angles x 768 bins, smoothed TV eps=1e-3 + "
                               "lambda=1e-3, levels 512/256/128/64 uniform p, ImaSk (PAPER sketches)",
                   "steps_level_mix": [round(float(v), 4) for v in mix], "epochs_timed": epochs},
        "roofline": {"bound": "alu", "kernel": f"k_{dom[0]} level {dom[1]}", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": None, "samples_per_launch": samples[dom[1]],
                     "avg_launch_us": dom_t * 1e6,
                     "effective_gather_frac_hbm": samples[dom[1]] * 8 / dom_t / 1e9 / HBM_PEAK_GBS},
        "kernels_us": {f"{k[0]}_l{k[1]}": round(v * 1e6, 2) for k, v in kern.items()},
        "projector_pair_samples_per_s": proj_pair_sps,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(b)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
