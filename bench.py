"""ImaSk throughput on one MI355X (epochs/s) for the 512x512 smoothed-TV workload.

One step = one iteration of Alg. 1 (draw, restriction, forward projection,
dual update, backprojection, prolongation, primal update, smoothed-TV prox)
on a 512 x 512 random-ellipse phantom with 720 angles x 768 bins, Poisson
I0 = 1e5, smoothed TV (eps = 1e-3) + lambda = 1e-3, levels 512/256/128/64
with p = 1/4 (the paper's literal construction, PAPER mode).  Epochs count
equivalent full-resolution operator applications (cost 2^{-l} per step).

With --fan the same workload runs on a fan beam: 720 source positions over
[0, 2 pi) at distance 4 (the image is [-1, 1]^2), a flat detector of 768
bins at distance 2 beyond the centre (bins the magnified pixel size, so the
fan just covers the image's circumscribed circle), with Poisson data from
the phantom's exact integrals along the fan's rays.

With --blocks S > 1 the same workload runs with the image sketches combined
with S measurement blocks (each step projects one of S contiguous angle
blocks; the outlook of Sec. 6); the default is the plain method (S = 1).

Prints one JSON line.  --gpus above 1 is refused: the path runs on one GPU
(how it would shard is a design note, not code).

Other workloads, each printing its own JSON line:
  --race                time to relative error 1e-3 against a common limit:
                        ImaSk, SAGA, ImaSk-Seq, PDHG, independent draws
                        (with --fan on the fan workload)
  --study stepsize|tv|square
                        PSNR against the phantom over a fixed epoch budget
  --batched             64 slices of mixed sizes in flight on several streams
  --serve               Poisson arrivals into the continuous-batching server
  --autograd            unrolled, checkpointed ImaSk forward + backward
  --oracle-timing       the FP64 oracle (all threads, one thread) against the
                        GPU: 50 iterations of the 64x64 Tikhonov workload

Profiling helpers (no GPU needed for --summarize):
  --counters fwd:L|bp:L launch one projector kernel, for rocprofv3 --pmc
  --copy-calib          also run a 64 MiB plain copy (for counter calibration)
  --summarize DIR...    turn rocprofv3 CSV output into the markdown summaries
                        kept under profiles/
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
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
FAN_D, FAN_DD = 4.0, 2.0  # fan workload: source and detector distances
# FP32 arithmetic per Joseph sample (a (ray, step) pair, two matrix entries),
# counted as the algorithm needs it: the right-tap weight w (1), the left
# weight 1 - w folded into a multiply-add with the left tap (2), the
# right tap's multiply-add (2), less the shared accumulation: about 4 FLOP.
FLOP_PER_SAMPLE = 4
# FP32 vector peak this build can issue: 256 CU x 4 SIMD x 16 lanes x 2 (FMA)
# x 2.4 GHz.  The chip's 157.3 TFLOP/s needs packed FP32 instructions, which
# this build disables (-packed-fp32-ops), so half of it is the attainable peak.
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
LDS_PEAK_TBPS = 256 * 128 * 2.4e9 / 1e12  # 78.6 TB/s: 128 B per clock per CU
# LDS bytes per sample: the transpose reads and writes both taps' cells, the
# forward reads both taps
LDS_BYTES_PER_SAMPLE = {"bp": 16, "fwd": 8}
COPY_N = 4096               # calibration copy: 4096^2 floats = 64 MiB each way
KERNEL_SOURCES = ["paper_2412_10249_amd/csrc/kernels.hip", "paper_2412_10249_amd/csrc/api.hip",
                  "paper_2412_10249_amd/csrc/internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def sample_counts(n, na, nd, lvl, angle_stride=1):
    """Samples (ray, step) with a tap inside the level-l image (geometry only).
    With angle_stride > 1 only every stride-th angle is counted and the total
    is scaled up (an estimate, for large batches of geometries)."""
    nl = n >> lvl
    h = 2.0 / nl
    th = np.arange(na) * np.pi / na
    s = (np.arange(nd) - (nd - 1) / 2.0) * (2.0 / n)
    rows = (4 * np.arange(na) <= na) | (4 * np.arange(na) >= 3 * na)
    c0 = -1.0 + 0.5 * h
    total = 0
    k = -1.0 + (np.arange(nl) + 0.5) * h
    picked = range(0, na, angle_stride)
    for a in picked:
        ct, st = np.cos(th[a]), np.sin(th[a])
        if rows[a]:
            u = ((s[:, None] - k[None, :] * st) / ct - c0) / h
        else:
            u = ((s[:, None] - k[None, :] * ct) / st - c0) / h
        q = np.floor(u)
        total += int(np.count_nonzero((q >= -1) & (q < nl)))
    return total if angle_stride == 1 else int(round(total * na / len(picked)))


def fan_sample_counts(n, nv, nd, D, Dd, lvl):
    """Samples (ray, step) with a tap inside the level-l image for the fan
    workload (geometry only, the rays built as in the library's tables)."""
    nl = n >> lvl
    h = 2.0 / nl
    ds = (2.0 / n) * (D + Dd) / D
    t = (np.arange(nd) - (nd - 1) / 2.0) * ds
    k = -1.0 + (np.arange(nl) + 0.5) * h
    c0 = -1.0 + 0.5 * h
    total = 0
    for a in range(nv):
        beta = 2 * np.pi * a / nv
        cb, sb = np.cos(beta), np.sin(beta)
        dx = -(D + Dd) * cb - t * sb
        dy = -(D + Dd) * sb + t * cb
        ln = np.hypot(dx, dy)
        ct, st = -dy / ln, dx / ln
        s = D * (ct * cb + st * sb)
        rows = np.abs(ct) >= np.abs(st)
        c, o = np.where(rows, ct, st), np.where(rows, st, ct)
        u = ((s[:, None] - k[None, :] * o[:, None]) / c[:, None] - c0) / h
        q = np.floor(u)
        total += int(np.count_nonzero((q >= -1) & (q < nl)))
    return total


def cpu_baseline(b, budget_s=12.0, blocks=1, fan=False):
    """The FP64 oracle running the same iteration on the host cores."""
    import oracle

    g = oracle.Geometry(N, NA, ND, src_dist=FAN_D, det_dist=FAN_DD) if fan else oracle.Geometry(N, NA, ND)
    lv = oracle.Levels(list(LEVELS), [1.0 / len(LEVELS)] * len(LEVELS))
    reg = oracle.Reg(oracle.REG_SMOOTH_TV, lam=LAM, tv_weight=TV_W, tv_eps=TV_EPS, tv_inner=TV_J)
    st = None
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        if blocks > 1:
            st = oracle.imask_blocks_run(g, lv, reg, SIGMA, SEED, STREAM, blocks, b, 1, st)
        else:
            st = oracle.imask_run(g, lv, reg, SIGMA, SEED, STREAM, b, 1, st)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": st.epochs / el, "unit": "epochs/s", "cores": cores, "kind": "oracle",
            "sample": f"first {st.k} ImaSk iterations ({st.epochs:.3f} epochs) of the same workload, FP64, "
                      f"{el:.1f} s"}


def stored_traffic(kernel_key):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("source_hash") != source_hash():
        return None
    ent = t.get("kernels", {}).get(kernel_key)
    return None if ent is None else ent.get("bytes_per_launch")


def stored_counter(kernel_key, name):
    """A derived counter figure (l2_hit_rate, ...) of the committed summary,
    or None when the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("source_hash") != source_hash():
        return None
    return t.get("kernels", {}).get(kernel_key, {}).get(name)


def counter_run(spec: str, fan: bool = False):
    """Launch only one projector kernel (plus the calibration copy), for a
    rocprofv3 --pmc pass: spec is fwd:LEVEL or bp:LEVEL (fan: on the fan
    workload's geometry), with the tuned launch shapes of the main run."""
    import torch

    import paper_2412_10249_amd as pk

    from paper_2412_10249_amd import autotune

    kind, lvl = spec.split(":")
    lvl = int(lvl)
    torch.cuda.set_device(0)
    autotune.apply_saved()  # the launch shapes the main run uses
    geom = pk.Geometry(N, NA, ND, src_dist=FAN_D, det_dist=FAN_DD) if fan else pk.Geometry(N, NA, ND)
    work = pk.workspace(geom)
    g = torch.Generator(device="cuda").manual_seed(5)
    src = torch.rand((COPY_N, COPY_N), device="cuda", generator=g)
    for _ in range(3):
        pk.resample(src, 0, pk.PROLONG)
    if kind == "fwd":
        x = torch.rand((N, N), device="cuda", generator=g)
        pk.time_kernel(geom, pk.KERNEL_FORWARD, lvl, x, work, 5)
    else:
        y = torch.rand((NA, ND), device="cuda", generator=g)
        pk.time_kernel(geom, pk.KERNEL_TRANSPOSE, lvl, y, work, 5)
    torch.cuda.synchronize()
    print(f"counter run done: {spec}", flush=True)


def algorithmic_bytes(kind, lvl, fan=False):
    """Compulsory HBM bytes of one projector launch: its input and output
    (forward: the level image in, the sinogram out; transpose: the reverse)."""
    nl = N >> lvl
    return 4 * (nl * nl + NA * ND)


def roofline_block(key, dom, dom_t, samples, fan):
    """The dominant kernel against the FP32 vector peak, with the measured
    HBM traffic beside its algorithmic bytes."""
    achieved = samples[dom[1]] * FLOP_PER_SAMPLE / dom_t / 1e12
    traffic = stored_traffic(key)
    alg = algorithmic_bytes(dom[0], dom[1], fan)
    return {"bound": "alu", "kernel": key, "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
            "flop_per_sample": FLOP_PER_SAMPLE, "peak_packed_fp32": PEAK_FP32_PACKED_TFLOPS,
            "samples_per_launch": samples[dom[1]], "avg_launch_us": dom_t * 1e6,
            "samples_per_s": samples[dom[1]] / dom_t,
            "algorithmic_bytes": alg,
            "hbm_TBps_measured": None if traffic is None else traffic / dom_t / 1e12,
            "hbm_frac_measured": None if traffic is None else traffic / dom_t / 1e9 / HBM_PEAK_GBS,
            "traffic_over_algorithmic": None if traffic is None else traffic / alg,
            "l2_hit_rate": stored_counter(key, "l2_hit_rate"),
            "lds_conflict_over_active_cycles": stored_counter(key, "lds_conflict_over_active_cycles")}


def step_times_by_level(prob, lv, steps):
    """Median GPU time of one whole step per level (HIP events on the stream
    the library launches on, between consecutive steps of one call; a spin
    kernel first keeps the GPU behind the host so the gaps are the GPU's
    own)."""
    import torch

    import paper_2412_10249_amd as pk

    draws = pk.draws(prob.params, lv, prob.k, steps)
    torch.cuda.synchronize()
    torch.cuda._sleep(50_000_000)
    # all steps in one library call, as a solve runs them
    dt = np.array(prob.step_timed(steps)) * 1e3
    out = {}
    for k, l in enumerate(lv.log2f):
        sel = dt[draws == k]
        if len(sel):
            out[l] = float(np.median(sel))
    return out


def run(args):
    import torch

    import paper_2412_10249_amd as pk
    import synth
    from paper_2412_10249_amd import autotune

    torch.cuda.set_device(0)
    # the launch shapes the autotuner chose on MI355X (paper_2412_10249_amd/tiles.json)
    n_tiles = 0 if args.default_tiles else autotune.apply_saved()
    if args.fan:  # exact integrals along the fan's rays
        _, b = synth.fan_ct_problem(N, NA, ND, FAN_D, FAN_DD, I0, 1000, 2000)
    else:
        _, b = synth.ct_problem(N, NA, ND, I0, 1000, 2000)
    b32 = torch.from_numpy(b.astype(np.float32)).cuda()
    geom = pk.Geometry(N, NA, ND, src_dist=FAN_D, det_dist=FAN_DD) if args.fan else pk.Geometry(N, NA, ND)
    lv = pk.Levels.uniform(LEVELS, pk.FULL_PAPER, args.blocks)
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

    # main projector kernels, HIP events on the stream the library launches on
    x = prob.x_cur.clone()
    y = prob.y_cur.clone()
    kern = {}
    for lvl in LEVELS:
        kern[("fwd", lvl)] = pk.time_kernel(geom, pk.KERNEL_FORWARD, lvl, x, prob.work, args.kernel_reps)
        kern[("bp", lvl)] = pk.time_kernel(geom, pk.KERNEL_TRANSPOSE, lvl, y, prob.work, args.kernel_reps)
    # the transpose with the ordered sum of its partial images (not for the
    # dominant-kernel choice: two launches)
    bp_sum = {lvl: pk.time_kernel(geom, pk.KERNEL_TRANSPOSE_SUM, lvl, y, prob.work, args.kernel_reps)
              for lvl in LEVELS} if not args.fan else {}
    if args.copy_calib:
        src = torch.rand((COPY_N, COPY_N), device="cuda")
        for _ in range(3):
            pk.resample(src, 0, pk.PROLONG)
        torch.cuda.synchronize()
    if args.fan:
        samples = {lvl: fan_sample_counts(N, NA, ND, FAN_D, FAN_DD, lvl) for lvl in LEVELS}
    else:
        samples = {lvl: sample_counts(N, NA, ND, lvl) for lvl in LEVELS}
    # dominant kernel: largest expected time per step under the level mix
    share = {key: t * lv.p[LEVELS.index(key[1])] for key, t in kern.items()}
    dom = max(share, key=share.get)
    dom_t = kern[dom]
    if args.fan:
        # this workload's transpose scatters on levels 0-1 (3 and 5 phases)
        # and gathers on levels 2-3
        name = {"fwd": "k_fwd_fan", "bp": "k_bp_fan_scatter" if dom[1] <= 1 else "k_bp_fan_gather"}[dom[0]]
    else:
        name = {"fwd": "k_fwd_band" if (N >> dom[1]) <= 1024 else "k_fwd_direct", "bp": "k_bp_own"}[dom[0]]
    key = f"{name}_l{dom[1]}"
    by_level = step_times_by_level(prob, lv, args.level_steps)
    t0_step = by_level.get(0)
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
        "data": "synthetic: seeded random-ellipse phantom, analytic line integrals"
                + (" along the fan's rays" if args.fan else "") + ", Poisson I0=1e5",
        "config": {"workload": ("2D fan-beam CT 512x512, 720 views over 2pi x 768 flat-detector bins, source "
                                f"distance {FAN_D}, detector distance {FAN_DD}" if args.fan else
                                "2D parallel-beam CT 512x512, 720 angles x 768 bins") + ", smoothed TV eps=1e-3 + "
                               "lambda=1e-3, levels 512/256/128/64 uniform p, ImaSk (PAPER sketches)"
                               + (f", {args.blocks} measurement blocks of {NA // args.blocks} angles"
                                  if args.blocks > 1 else ""),
                   "steps_level_mix": [round(float(v), 4) for v in mix], "epochs_timed": epochs,
                   "tuned_tile_entries": n_tiles},
        "roofline": roofline_block(key, dom, dom_t, samples, args.fan),
        # the transpose's working limit: LDS traffic, two read-modify-writes of
        # 4-byte cells per sample, against 256 CUs x 128 B/clk x 2.4 GHz
        "lds_roofline": None if args.fan else {"kernel": key, "bytes_per_sample": LDS_BYTES_PER_SAMPLE[dom[0]],
                         "achieved_TBps": samples[dom[1]] * LDS_BYTES_PER_SAMPLE[dom[0]] / dom_t / 1e12,
                         "peak_TBps": LDS_PEAK_TBPS,
                         "frac": samples[dom[1]] * LDS_BYTES_PER_SAMPLE[dom[0]] / dom_t / 1e12 / LDS_PEAK_TBPS},
        # whole steps per level (median us) against the cost model of the
        # epoch count: a level-l step costs 2^-l of a full-resolution one
        "step_us_by_level": {f"l{l}": round(v, 2) for l, v in by_level.items()},
        "step_ratio_vs_level0": {f"l{l}": {"measured": round(v / t0_step, 4), "model": 2.0 ** -l}
                                 for l, v in by_level.items()} if t0_step else None,
        "kernels_us": {f"{k[0]}_l{k[1]}": round(v * 1e6, 2) for k, v in kern.items()},
        "transpose_with_sum_us": {f"l{l}": round(v * 1e6, 2) for l, v in bp_sum.items()},
        "projector_samples_per_s": {f"{k[0]}_l{k[1]}": samples[k[1]] / v for k, v in kern.items()},
        "kernel_source_hash": source_hash(),
    }
    headline = args.blocks == 1 and not args.fan
    if headline and not args.no_race:
        try:
            out["time_to_rel_err_1e-3"] = headline_race(geom, b32, prob.work, args)
        except Exception as e:  # the epochs/s line above stands on its own
            out["time_to_rel_err_1e-3"] = {"error": repr(e)}
    if headline and not args.no_serve:
        try:
            out["serve"] = headline_serve(args)
        except Exception as e:
            out["serve"] = {"error": repr(e)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(b, blocks=args.blocks, fan=args.fan)
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------ the race

def tv_grad_torch(u, eps):
    """Gradient of sum sqrt(|grad u|^2 + eps^2) (forward differences, zero at
    the last row/column) - measurement code for the reference solution."""
    import torch

    g1 = torch.zeros_like(u)
    g2 = torch.zeros_like(u)
    g1[:-1, :] = u[1:, :] - u[:-1, :]
    g2[:, :-1] = u[:, 1:] - u[:, :-1]
    nrm = torch.sqrt(g1 * g1 + g2 * g2 + eps * eps)
    q1, q2 = g1 / nrm, g2 / nrm
    div = -q1 - q2
    div[1:, :] += q1[:-1, :]
    div[:, 1:] += q2[:, :-1]
    return div


def reference_solution(geom, work, b32, lam, w, eps, iters, log):
    """x_ref = argmin 1/2|R0 x - b|^2 + w TV_eps(x) + lam/2 |x|^2 by Nesterov's
    accelerated gradient with the known strong convexity (mu = lam) and
    Lipschitz constant; returns x and the final relative gradient norm."""
    import torch

    import paper_2412_10249_amd as pk

    x = torch.zeros(geom.image_shape, device="cuda")
    v = torch.randn(geom.image_shape, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    for _ in range(50):  # power method for |R0|^2
        v = pk.backproject(geom, 0, pk.project(geom, 0, v, work), work)
        nrm = torch.linalg.vector_norm(v)
        v = v / nrm
    L = float(nrm) + lam + 8.0 * w / eps
    q = np.sqrt(lam / L)
    beta = (1 - q) / (1 + q)
    atb = pk.backproject(geom, 0, b32, work)
    scale = float(torch.linalg.vector_norm(atb))

    def grad(z):
        r = pk.project(geom, 0, z, work) - b32
        return pk.backproject(geom, 0, r.contiguous(), work) + w * tv_grad_torch(z, eps) + lam * z

    y = x.clone()
    for it in range(iters):
        xn = y - grad(y) / L
        y = xn + beta * (xn - x)
        x = xn
        if (it + 1) % 500 == 0:
            gn = float(torch.linalg.vector_norm(grad(x))) / scale
            log(f"reference: {it + 1} iterations, |grad F|/|R0^T b| = {gn:.3e}")
    gn = float(torch.linalg.vector_norm(grad(x))) / scale
    return x, gn


def race_method(name, lv, sched, geom, work, b32, xref, reg, args, mults, log):
    """One method of the race at each multiple of its base step: runs until
    the relative error to xref reaches args.target (checked every few
    epochs, interpolated in log error), diverges or runs out of time."""
    import torch

    import paper_2412_10249_amd as pk

    rnorm = float(torch.linalg.vector_norm(xref))
    L2, lb, lp = pk.step_constants(geom, lv, LAM, work, iters=40)
    nb = max(lv.n_blocks, 1)
    s3, th = pk.sigma_thm3(L2, nb * lb, nb * nb * lp, min(lv.p) / nb, 100)
    spd = 1.0 / np.sqrt(L2)
    seq = sched == pk.SCHEDULE_SEQUENTIAL
    base = spd if seq else s3
    res = {"constants": [L2, lb, lp], "blocks": nb, "sigma_thm3": s3, "theta_thm3": th, "sigma_pd": spd,
           "schedule": "sequential" if seq else "parallel", "runs": []}
    check = args.seq_check_every if seq else args.check_every
    for mult in mults:
        sigma = base * mult
        draw = pk.DRAW_INDEPENDENT if name.endswith("_indep") else pk.DRAW_COMMON
        prob = pk.Problem(geom, lv, reg, pk.Params(sigma, SEED, STREAM, sched, 1.0, draw, STREAM + 1), b32)
        torch.cuda.synchronize()
        hist = []
        tstart = time.perf_counter()
        tlog = tstart
        while prob.epochs < args.race_epochs:
            prob.solve(check, pk.BUDGET_EPOCHS)
            err = float(torch.linalg.vector_norm(prob.x_cur - xref)) / rnorm  # synchronises
            hist.append((time.perf_counter() - tstart, prob.epochs, err))
            if time.perf_counter() - tlog > 20.0:
                tlog = time.perf_counter()
                log(f"  {name} sigma x{mult}: {prob.epochs:.0f} epochs, rel err {err:.3e}")
            if (err <= args.target or not np.isfinite(err) or err > 10.0
                    or time.perf_counter() - tstart > args.race_seconds):
                break
        t_hit = e_hit = None
        for (t1, e1, r1_), (t2, e2, r2_) in zip([(0.0, 0.0, 1.0)] + hist, hist):
            if r2_ <= args.target < r1_:  # interpolate in log error
                f = (np.log(r1_) - np.log(args.target)) / (np.log(r1_) - np.log(r2_))
                t_hit = t1 + f * (t2 - t1)
                e_hit = e1 + f * (e2 - e1)
                break
        run_res = {"sigma": sigma, "sigma_multiple": mult, "epochs": prob.epochs,
                   "final_rel_err": hist[-1][2], "seconds": hist[-1][0], "time_to_target_s": t_hit,
                   "epochs_to_target": e_hit, "check_every_epochs": check,
                   "rel_err_history": [(round(h[1], 2), round(h[2], 7)) for h in hist[::max(1, len(hist) // 60)]]}
        log(f"{name} sigma x{mult}: {run_res['final_rel_err']:.3e} after {prob.epochs:.1f} epochs, "
            f"{hist[-1][0]:.2f} s, t(1e-3) = {t_hit}")
        res["runs"].append(run_res)
        del prob
    return res


def headline_race(geom, b32, work, args):
    """The headline's second figure: time to relative error 1e-3 of ImaSk
    (r = 4, UNBIASED sketches) against full-resolution SAGA (r = 1), both at
    twice their Thm. 3 step (the fastest stable multiple), against the limit
    they share, certified by its relative gradient."""
    import torch

    import paper_2412_10249_amd as pk

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    xref, gnorm = reference_solution(geom, work, b32, LAM, TV_W, TV_EPS, args.ref_iters, log)
    reg = pk.Regularizer(pk.REG_SMOOTH_TV, LAM, TV_W, TV_EPS, TV_J)
    out = {"target": args.target, "reference_relative_gradient": gnorm, "sigma_multiple_of_thm3": 2.0}
    rargs = argparse.Namespace(**vars(args))
    rargs.race_epochs, rargs.race_seconds = 1e6, args.headline_race_seconds
    for name, lv in (("imask_r4", pk.Levels.uniform(LEVELS, pk.FULL_UNBIASED)), ("saga_r1", pk.Levels((0,), (1.0,)))):
        res = race_method(name, lv, pk.SCHEDULE_PARALLEL, geom, work, b32, xref, reg, rargs, [2.0], log)
        r = res["runs"][0]
        out[name] = {"seconds": r["time_to_target_s"], "epochs": r["epochs_to_target"], "sigma": r["sigma"],
                     "final_rel_err": r["final_rel_err"]}
    a, c = out["imask_r4"]["seconds"], out["saga_r1"]["seconds"]
    out["imask_over_saga_time"] = a / c if a and c else None
    out["wall_s"] = time.perf_counter() - t0
    torch.cuda.synchronize()
    return out


def race(args):
    """Time to a relative error of 1e-3 against the common limit, same kernels,
    same GPU, UNBIASED sketches (levels 512/256/128/64) so that every method
    shares the limit:
      imask_r4 / saga_r1  Alg. 1 with r = 4 / r = 1, sigma = m * sigma_thm3
      imask_r4_indep      Alg. 1, r = 4, independent primal/dual draws (Sec. 6)
      imask_r4_b4 / saga_r1_b4
                          Alg. 1 over r = 4 / r = 1 image sketches combined
                          with 4 measurement blocks of 180 angles (Sec. 6
                          outlook); sigma = m * the Thm. 3 step of the block
                          family, with |K_kb|^2 ~ S |K_k|^2 (a block of
                          contiguous angles carries about 1/S of the energy
                          of the leading singular vector), so that
                          Lbar^2 -> S Lbar^2, Lbar_p^2 -> S^2 Lbar_p^2 and
                          p_min -> p_min / S
      seq_r4 / seq_r1     ImaSk-Seq (Sec. 5, theta = 1) with r = 4 / r = 1
                          (r = 1 is PDHG), sigma = m * sigma_pd, where
                          sigma_pd = (L^2)^{-1/2} is the single-level PDHG
                          limit sigma tau |K|^2 < 1 with tau = sigma / mu.
    Each method runs its grid of multiples m; the best time is reported
    (the paper tunes ImaSk-Seq's step by a grid search too).  With --fan the
    same race runs on the fan workload."""
    import torch

    import paper_2412_10249_amd as pk
    import synth

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.fan:
        _, b = synth.fan_ct_problem(N, NA, ND, FAN_D, FAN_DD, I0, 1000, 2000)
        geom = pk.Geometry(N, NA, ND, src_dist=FAN_D, det_dist=FAN_DD)
    else:
        _, b = synth.ct_problem(N, NA, ND, I0, 1000, 2000)
        geom = pk.Geometry(N, NA, ND)
    b32 = torch.from_numpy(b.astype(np.float32)).cuda()
    work = pk.workspace(geom)
    t0 = time.perf_counter()
    xref, gnorm = reference_solution(geom, work, b32, LAM, TV_W, TV_EPS, args.ref_iters, log)
    log(f"reference done in {time.perf_counter() - t0:.1f} s, relative gradient {gnorm:.2e}")
    reg = pk.Regularizer(pk.REG_SMOOTH_TV, LAM, TV_W, TV_EPS, TV_J)
    r4 = pk.Levels.uniform(LEVELS, pk.FULL_UNBIASED)
    r1 = pk.Levels((0,), (1.0,))
    r4b = pk.Levels.uniform(LEVELS, pk.FULL_UNBIASED, 4)
    r1b = pk.Levels((0,), (1.0,), pk.FULL_UNBIASED, 4)
    methods = {"imask_r4": (r4, pk.SCHEDULE_PARALLEL), "saga_r1": (r1, pk.SCHEDULE_PARALLEL),
               "seq_r4": (r4, pk.SCHEDULE_SEQUENTIAL), "seq_r1": (r1, pk.SCHEDULE_SEQUENTIAL),
               "imask_r4_indep": (r4, pk.SCHEDULE_PARALLEL),
               "imask_r4_b4": (r4b, pk.SCHEDULE_PARALLEL), "saga_r1_b4": (r1b, pk.SCHEDULE_PARALLEL)}
    results = {}
    for name in args.methods:
        lv, sched = methods[name]
        results[name] = race_method(name, lv, sched, geom, work, b32, xref, reg, args,
                                    args.seq_sigma_mults if sched == pk.SCHEDULE_SEQUENTIAL else args.sigma_mults,
                                    log)
    best = {k: min([r["time_to_target_s"] for r in v["runs"] if r["time_to_target_s"]] or [None], key=lambda z: z or 1e30)
            for k, v in results.items()}
    print(json.dumps({"metric": "time to relative error 1e-3 vs the common limit (512x512 smoothed TV"
                                + (", fan beam)" if args.fan else ")"),
                      "target": args.target, "reference_relative_gradient": gnorm, "best_time_s": best,
                      "results": results}), flush=True)


def study(args):
    """Fixed-budget studies on the 512^2 workload, PSNR against the phantom
    every few epochs (the quantity of the paper's Sec. 4 figures):
      stepsize  ImaSk r = 4 (PAPER sketches), Tikhonov lam = 1e-2, with
                sigma in {sigma*/2, sigma*, sigma_B} (sigma* of Thm. 3, sigma_B
                of Sec. 3.6)
      tv        the paper's TV + nonnegativity prior (w = 2e-4, lam = 1e-4 for
                the step rule), ImaSk with r = 1, 2, 4 at 1, 4, 16 and 64 times
                its Thm. 3 step (the prior is barely strongly convex, so the
                theorem's step is very conservative), and ImaSk-Seq with
                r = 1, 4 at a quarter and half of the PDHG limit
      square    the comparison of the paper's Sec. 5: a square insert whose
                edges lie on the coarsest grid (64-pixel blocks, levels
                512..4, r = 8 as in the paper's comparison), Poisson data
                from its exact line integrals, the TV + nonnegativity prior;
                ImaSk and ImaSk-Seq with r = 8, ImaSk r = 1 (SAGA) and PDHG
                (ImaSk-Seq r = 1); PSNR against the square and the distance
                to the PDHG solution after --ref-iters iterations"""
    import torch

    import paper_2412_10249_amd as pk
    import synth

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.study == "square":
        x_true = synth.square_insert(N, 64, 3, 5)
        b = synth.poisson_log_data(synth.square_line_integrals(N, 64, 3, 5, NA, ND), I0, 2000)
    else:
        x_true, b = synth.ct_problem(N, NA, ND, I0, 1000, 2000)
    b32 = torch.from_numpy(b.astype(np.float32)).cuda()
    xt = torch.from_numpy(x_true.astype(np.float32)).cuda()
    peak = float(xt.max())
    geom = pk.Geometry(N, NA, ND)
    work = pk.workspace(geom)

    def psnr(x):
        mse = float(torch.mean((x - xt) ** 2))
        return 10.0 * np.log10(peak * peak / mse)

    runs = []
    ref = None
    if args.study == "square":
        lam, w = 1e-4, 2e-4
        reg = pk.Regularizer(pk.REG_TV, lam, w, 0.0, TV_J)
        info = {"lam": lam, "tv_weight": w, "tv_inner": TV_J, "phantom": "square insert, 64-pixel blocks 3..5",
                "levels": list(range(8))}
        lv8 = pk.Levels.uniform(tuple(range(8)), pk.FULL_PAPER)
        lv1 = pk.Levels.uniform((0,), pk.FULL_PAPER)
        cases = []
        for lv, r in ((lv8, 8), (lv1, 1)):
            L2, lb, lp = pk.step_constants(geom, lv, lam, work, iters=40)
            s3 = pk.sigma_thm3(L2, lb, lp, min(lv.p), 100)[0]
            info[f"constants_r{r}"] = [L2, lb, lp]
            for m in (16, 64):
                cases.append((f"imask_r{r} x{m}", lv, reg, m * s3, pk.SCHEDULE_PARALLEL))
            for m in (0.25, 0.5, 0.9):
                cases.append((f"{'pdhg' if r == 1 else 'seq_r8'} x{m}", lv, reg, m / np.sqrt(L2),
                              pk.SCHEDULE_SEQUENTIAL))
            if r == 1:
                sig_ref = 0.9 / np.sqrt(L2)
        # the reference: PDHG (ImaSk-Seq with one level) run long
        rp = pk.Problem(geom, lv1, reg, pk.Params(sig_ref, SEED, STREAM, pk.SCHEDULE_SEQUENTIAL, 1.0), b32)
        rp.step(args.ref_iters)
        torch.cuda.synchronize()
        ref = rp.x_cur.clone()
        prev = rp.x_cur.clone()
        rp.step(100)
        info["reference"] = {"iterations": args.ref_iters, "sigma": sig_ref,
                             "relative_change_last_100": float(torch.linalg.norm(rp.x_cur - prev) /
                                                               torch.linalg.norm(prev))}
        log(f"reference: {args.ref_iters} PDHG iterations, last-100 change {info['reference']}")
    elif args.study == "stepsize":
        lam = 1e-2
        lv = pk.Levels.uniform(LEVELS, pk.FULL_PAPER)
        reg = pk.Regularizer(pk.REG_TIKHONOV, lam)
        L2, lb, lp = pk.step_constants(geom, lv, lam, work, iters=40)
        s3 = pk.sigma_thm3(L2, lb, lp, min(lv.p), 100)[0]
        sb = pk.sigma_balamurugan(L2, lb)
        cases = [("sigma*/2", lv, reg, s3 / 2, pk.SCHEDULE_PARALLEL), ("sigma*", lv, reg, s3, pk.SCHEDULE_PARALLEL),
                 ("sigma_B", lv, reg, sb, pk.SCHEDULE_PARALLEL)]
        info = {"constants": [L2, lb, lp], "sigma_star": s3, "sigma_B": sb, "lam": lam}
    else:
        lam, w = 1e-4, 2e-4
        reg = pk.Regularizer(pk.REG_TV, lam, w, 0.0, TV_J)
        cases = []
        info = {"lam": lam, "tv_weight": w, "tv_inner": TV_J}
        for r in (1, 2, 4):
            lv = pk.Levels.uniform(LEVELS[:r], pk.FULL_PAPER)
            L2, lb, lp = pk.step_constants(geom, lv, lam, work, iters=40)
            s3 = pk.sigma_thm3(L2, lb, lp, min(lv.p), 100)[0]
            for m in (1, 4, 16, 64):
                cases.append((f"imask_r{r} x{m}", lv, reg, m * s3, pk.SCHEDULE_PARALLEL))
            if r != 2:
                for m in (0.25, 0.5):
                    cases.append((f"seq_r{r} x{m}", lv, reg, m / np.sqrt(L2), pk.SCHEDULE_SEQUENTIAL))
    for name, lv, reg, sigma, sched in cases:
        prob = pk.Problem(geom, lv, reg, pk.Params(sigma, SEED, STREAM, sched, 1.0), b32)
        torch.cuda.synchronize()
        prob.step(1)  # first launches (code objects, LDS attributes) outside the clock
        torch.cuda.synchronize()
        hist = []
        t0 = time.perf_counter()
        while prob.epochs < args.study_epochs:
            prob.solve(args.study_every, pk.BUDGET_EPOCHS)
            row = [round(time.perf_counter() - t0, 4), round(prob.epochs, 3), round(psnr(prob.x_cur), 3)]
            if ref is not None:
                row.append(float(torch.linalg.norm(prob.x_cur - ref) / torch.linalg.norm(ref)))
            hist.append(tuple(row))
            if not np.isfinite(hist[-1][2]):
                break
        log(f"{name}: sigma {sigma:.3e}, {prob.epochs:.1f} epochs, {hist[-1][0]:.2f} s, PSNR {hist[-1][2]:.2f} dB"
            + (f", distance to the reference {hist[-1][3]:.3e}" if ref is not None else ""))
        key = "history_s_epochs_psnr" + ("_dist" if ref is not None else "")
        runs.append({"name": name, "sigma": sigma, "schedule": "sequential" if sched else "parallel",
                     "levels": list(lv.log2f), key: hist})
    print(json.dumps({"metric": f"PSNR vs epochs, {args.study} study (512x512, 720 x 768)", "info": info,
                      "runs": runs}), flush=True)


# ------------------------------------------------------------ systems workloads

def _sigma_for(geom, levels, lam, work, cache={}):
    """Thm. 3 step size (x2, the fastest stable multiple in the race) per geometry."""
    import paper_2412_10249_amd as pk

    key = (geom, levels)
    if key not in cache:
        L2, lb, lp = pk.step_constants(geom, levels, lam, work, iters=30)
        cache[key] = 2.0 * pk.sigma_thm3(L2, lb, lp, min(levels.p), 100)[0]
    return cache[key]


def batched(args):
    """64 slices of mixed sizes (256..1024, angles = bins = 1.5 N), each with its
    own draw stream, Tikhonov lam = 1e-2, 30 epochs each.  Three ways:
      batched   the library's batched steps: one persistent launch per kernel
                variant for all slices, draws on the device, one captured
                step replayed as a CUDA graph; with the autotuned tiles
                (paper_2412_10249_amd/tiles.json) and with the defaults
                and with the step's forward and transpose halves on two
                streams inside the graph; and split in 2 or 4 groups, each
                group's graph replayed on its own stream
      streams   each slice's own steps, dealt round-robin to 8 HIP streams
      alone     the slices one after another on one stream
    Aggregate samples/s, and every batched slice compared with its run alone."""
    import torch

    import paper_2412_10249_amd as pk
    import synth
    from paper_2412_10249_amd import autotune, batch

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    sizes = [256, 384, 512, 768, 1024]
    lv = pk.Levels.uniform(LEVELS)
    reg = pk.Regularizer(pk.REG_TIKHONOV, 1e-2)
    data = {}
    for n in sizes:
        data[n] = [torch.from_numpy(synth.ct_problem(n, 3 * n // 2, 3 * n // 2, 1e5, 1000 + s, 2000 + s)[1]
                                    .astype(np.float32)).cuda() for s in range(2)]
        log(f"data for N={n} ready")
    sig = {}

    def make():
        out = []
        for s in range(args.slices):
            n = sizes[s % 5]
            geom = pk.Geometry(n, 3 * n // 2, 3 * n // 2)
            if n not in sig:
                sig[n] = _sigma_for(geom, lv, 1e-2, pk.workspace(geom))
            out.append(pk.Problem(geom, lv, reg, pk.Params(sig[n], SEED, s), data[n][s % 2]))
        torch.cuda.synchronize()
        return out

    # one epoch = one full-resolution projection and one backprojection
    s0 = {n: sample_counts(n, 3 * n // 2, 3 * n // 2, 0, angle_stride=16) for n in sizes}
    samples_per_epoch = sum(2 * s0[sizes[s % 5]] for s in range(args.slices))
    res = {"metric": "batched ImaSk, 64 mixed slices", "slices": args.slices, "epochs_per_slice": args.epochs}

    def run_batched(tiles, overlapped=False):
        table = autotune.load() if tiles else {}
        autotune.apply(table)
        probs = make()
        bt = batch.Batch(probs, args.epochs, pk.BUDGET_EPOCHS)
        bt.capture(overlapped=overlapped)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.replay(bt.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        bt.sync_state()
        autotune.reset(table)
        return probs, el, bt.steps

    for name, tiles, over in (("batched_graph_tuned", True, False), ("batched_graph_default_tiles", False, False),
                              ("batched_graph_two_streams", True, True)):
        probs, el, steps = run_batched(tiles, over)
        tot = sum(p.epochs for p in probs)
        res[name] = {"seconds": el, "batched_steps": steps, "slice_epochs_per_s": tot / el,
                     "samples_per_s": samples_per_epoch * args.epochs / el}
        log(f"{name}: {el:.3f} s, {steps} batched steps")
        if name == "batched_graph_tuned":
            tuned_probs = probs
        elif over:
            # the forward and transpose halves on two streams: same results
            res[name]["equal_to_one_stream_bitwise"] = sum(
                int(torch.equal(a.x_cur, c.x_cur) and torch.equal(a.y_cur, c.y_cur))
                for a, c in zip(probs, tuned_probs))
            del probs
        else:
            del probs
    # the batch split in groups, each group's captured step replayed on its
    # own stream (the groups' phases overlap)
    for groups in (2, 4):
        table = autotune.load()
        autotune.apply(table)
        probs = make()
        bg = batch.BatchGroups(probs, args.epochs, pk.BUDGET_EPOCHS, groups)
        bg.capture()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bg.run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        bg.sync_state()
        name = f"batched_graph_{groups}_groups"
        res[name] = {"seconds": el, "samples_per_s": samples_per_epoch * args.epochs / el,
                     "equal_to_one_batch_bitwise": sum(int(torch.equal(probs[q].x_cur, tuned_probs[q].x_cur))
                                                       for q in range(len(probs)))}
        log(f"{name}: {el:.3f} s")
        autotune.reset(table)
        del bg, probs
    # the same slices on 8 streams, and one after another
    probs = make()
    runner = batch.BatchRunner(probs, n_streams=args.streams)
    t0 = time.perf_counter()
    runner.solve_all(args.epochs, pk.BUDGET_EPOCHS)
    runner.synchronize()
    el = time.perf_counter() - t0
    res["streams"] = {"streams": args.streams, "seconds": el, "samples_per_s": samples_per_epoch * args.epochs / el}
    del probs, runner
    probs = make()
    t0 = time.perf_counter()
    for p in probs:
        p.solve(args.epochs, pk.BUDGET_EPOCHS)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    res["alone"] = {"seconds": seq, "samples_per_s": samples_per_epoch * args.epochs / seq}
    # every batched slice (tuned tiles) against its run alone with the same tiles
    table = autotune.load()
    autotune.apply(table)
    worst = 0.0
    equal = 0
    for s, p in enumerate(tuned_probs):
        q = pk.Problem(p.geom, lv, reg, pk.Params(sig[p.geom.n], SEED, s), data[p.geom.n][s % 2])
        q.solve(args.epochs, pk.BUDGET_EPOCHS)
        same = bool(torch.equal(q.x_cur, p.x_cur))
        equal += int(same)
        d = float(torch.linalg.vector_norm(q.x_cur - p.x_cur) / torch.linalg.vector_norm(q.x_cur))
        worst = max(worst, d)
        del q
    autotune.reset(table)
    res["equal_to_alone_bitwise"] = equal
    res["checked_slices"] = len(tuned_probs)
    res["worst_rel_diff_to_alone"] = worst
    res["speedup_vs_alone"] = seq / res["batched_graph_tuned"]["seconds"]
    res["speedup_vs_streams"] = res["streams"]["seconds"] / res["batched_graph_tuned"]["seconds"]
    print(json.dumps(res), flush=True)


def serve_pool(lv, reg, sizes=(128, 256, 512, 1024)):
    """Data and step sizes of the serving workload (three sinograms per size)."""
    import torch

    import paper_2412_10249_amd as pk
    import synth

    pool, sig = {}, {}
    for n in sizes:
        geom = pk.Geometry(n, 3 * n // 2, 3 * n // 2)
        pool[n] = [torch.from_numpy(synth.ct_problem(n, 3 * n // 2, 3 * n // 2, 1e5, 3000 + s, 4000 + s)[1]
                                    .astype(np.float32)).cuda() for s in range(3)]
        sig[geom] = _sigma_for(geom, lv, 1e-2, pk.workspace(geom))
    return pool, sig


def serve_rate(rate, args, lv, reg, pool, sig, log):
    """Poisson arrivals at `rate` over args.window seconds into the server."""
    from paper_2412_10249_amd import serve

    ex = serve.GpuExecutor(args.slots, lambda n: lv, reg, lambda g: sig[g])
    sch = serve.Scheduler(ex, hbm_budget=int(args.hbm_gb * 2 ** 30), max_active=args.slots,
                          chunk_epochs=args.chunk)
    arr = serve.poisson_arrivals(rate, args.window, seed=7)
    t0 = time.perf_counter()
    done = serve.run_load(sch, arr, lambda rid, n, t: serve.Request(rid, n, t, args.serve_epochs,
                                                                      data=pool[n][rid % 3]))
    summ = serve.latency_summary(done)
    summ.update({"offered_per_s": rate, "requests": len(arr), "window_s": args.window,
                 "wall_s": time.perf_counter() - t0})
    log(f"rate {rate}: {summ}")
    return summ


def headline_serve(args):
    """The headline's serving figures: p50/p99 latency of 30-epoch requests
    (N in 128/256/512/1024, weights 4:3:2:1) under Poisson arrivals at the
    configured 200 req/s (beyond what the projectors deliver, so its queue
    grows) and at 150 req/s, the highest rate measured to drain."""
    import paper_2412_10249_amd as pk

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    lv = pk.Levels.uniform(LEVELS)
    reg = pk.Regularizer(pk.REG_TIKHONOV, 1e-2)
    pool, sig = serve_pool(lv, reg)
    out = {"epochs_per_request": args.serve_epochs, "window_s": args.window, "slots": args.slots}
    for rate in args.headline_rates:
        r = serve_rate(rate, args, lv, reg, pool, sig, log)
        out[f"rate_{int(rate)}"] = {k: r.get(k) for k in ("p50_ms", "p99_ms", "served_per_s", "offered_per_s",
                                                           "requests", "wall_s")}
    return out


def serving(args):
    """Poisson arrivals of reconstructions (N in 128/256/512/1024, weights
    4:3:2:1, angles = bins = 1.5 N, 30 epochs each) at the given rates."""
    import torch

    import paper_2412_10249_amd as pk
    import synth
    from paper_2412_10249_amd import serve

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    lv = pk.Levels.uniform(LEVELS)
    reg = pk.Regularizer(pk.REG_TIKHONOV, 1e-2)
    pool, sig = serve_pool(lv, reg)
    log("serving data ready")
    out = [serve_rate(rate, args, lv, reg, pool, sig, log) for rate in args.rates]
    # sustainable: the queue drains within a second of the arrival window
    ok = [r["offered_per_s"] for r in out if r["wall_s"] <= args.window + 1.0]
    print(json.dumps({"metric": "serving ImaSk reconstructions, p50/p99 latency", "slots": args.slots,
                      "epochs_per_request": args.serve_epochs, "window_s": args.window,
                      "highest_sustained_rate_per_s": max(ok) if ok else None, "results": out}), flush=True)


def _oracle_cfg1_seconds(reps: int = 5) -> list:
    """Wall times of 50 oracle iterations on the 64x64 Tikhonov workload."""
    import oracle
    import synth

    _, b = synth.ct_problem(64, 90, 92, 1e4, 1000, 2000)
    b = np.asarray(b, dtype=np.float32).astype(np.float64)
    g = oracle.Geometry(64, 90, 92)
    lv = oracle.Levels([0, 1, 2], [1.0 / 3] * 3)
    out = []
    for _ in range(reps + 1):  # the first run warms up
        t0 = time.perf_counter()
        oracle.imask_run(g, lv, oracle.Reg(lam=1e-2), 0.02, SEED, STREAM, b, 50)
        out.append(time.perf_counter() - t0)
    return out[1:]


def oracle_timing(args):
    """The FP64 oracle (all host threads, and one thread in a child process)
    against the GPU on the 64x64 Tikhonov workload: 50 iterations, median of
    5 runs after a warm-up, same seed and step."""
    import subprocess

    import synth
    import torch

    import paper_2412_10249_amd as pk

    if args.oracle_child:
        print(json.dumps({"seconds": _oracle_cfg1_seconds()}))
        return
    all_threads = _oracle_cfg1_seconds()
    env = dict(os.environ, OMP_NUM_THREADS="1")
    child = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-timing", "--oracle-child"],
                           env=env, capture_output=True, text=True, check=True)
    one_thread = json.loads(child.stdout.strip().splitlines()[-1])["seconds"]
    _, b = synth.ct_problem(64, 90, 92, 1e4, 1000, 2000)
    b32 = torch.from_numpy(np.asarray(b, dtype=np.float32)).cuda()
    gpu = []
    for _ in range(6):
        prob = pk.Problem(pk.Geometry(64, 90, 92), pk.Levels.uniform((0, 1, 2)), pk.Regularizer(pk.REG_TIKHONOV, 1e-2),
                          pk.Params(0.02, SEED, STREAM), b32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.step(50)
        torch.cuda.synchronize()
        gpu.append(time.perf_counter() - t0)
    med = lambda v: float(np.median(v))  # noqa: E731
    print(json.dumps({"metric": "50 ImaSk iterations, 64x64 Tikhonov (90 x 92, levels 64/32/16), median of 5",
                      "oracle_s": med(all_threads), "oracle_threads": int(os.environ.get("OMP_NUM_THREADS",
                                                                                        os.cpu_count() or 1)),
                      "oracle_1_thread_s": med(one_thread), "gpu_s": med(gpu[1:]),
                      "speedup_vs_oracle": med(all_threads) / med(gpu[1:]),
                      "speedup_vs_1_thread": med(one_thread) / med(gpu[1:])}))


def autograd_bench(args):
    """Differentiable unrolled ImaSk: batch 32 of 256^2, 384 angles x 384 bins,
    10 iterations, checkpoint every 2; gradients to the image and lam."""
    import torch

    import paper_2412_10249_amd as pk
    import synth
    from paper_2412_10249_amd import autograd as ag

    torch.cuda.set_device(0)
    n, na, nd = 256, 384, 384
    geom = pk.Geometry(n, na, nd)
    lv = pk.Levels.uniform(LEVELS)
    work = pk.workspace(geom)
    sigma = _sigma_for(geom, lv, 1e-2, work)
    xs = [torch.from_numpy(synth.ct_problem(n, na, nd, 1e5, 5000 + s, 6000 + s)[0].astype(np.float32)).cuda()
          for s in range(args.batch)]
    x_in = torch.stack(xs) * 0.9
    x_in.requires_grad_(True)
    lam = torch.tensor(1e-2, device="cuda", requires_grad=True)

    def loss(xin, lam_):
        tot = 0.0
        for s in range(xin.shape[0]):
            b = ag.ProjectFn.apply(xin[s], geom, 0, work)
            xk = ag.unrolled_imask(b, lam_, geom, lv, sigma, 10, stream_id=s, work=work, checkpoint_every=2)
            tot = tot + 0.5 * ((xk - xs[s]).double() ** 2).sum()
        return tot

    L = loss(x_in, lam)
    gx, gl = torch.autograd.grad(L, (x_in, lam))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = loss(x_in, lam)
    gx, gl = torch.autograd.grad(L, (x_in, lam))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d = torch.randn_like(x_in)
    with torch.no_grad():
        h = 1.0  # the loss is quadratic in x_in, so the central difference is exact
        fd = (loss(x_in + h * d, lam) - loss(x_in - h * d, lam)) / (2 * h)
        hl = 1e-4
        fdl = (loss(x_in, lam + hl) - loss(x_in, lam - hl)) / (2 * hl)
    dd = float((gx * d).sum())
    print(json.dumps({"metric": "unrolled ImaSk forward+backward", "batch": args.batch, "iterations": 10,
                      "checkpoint_every": 2, "seconds": el, "ms_per_sample": el / args.batch * 1e3,
                      "dir_derivative": dd, "fd_dir_derivative": float(fd),
                      "rel_err_dx": abs(dd - float(fd)) / abs(float(fd)),
                      "dlam": float(gl), "fd_dlam": float(fdl),
                      "rel_err_dlam": abs(float(gl) - float(fdl)) / abs(float(fdl))}), flush=True)


# ------------------------------------------------------------ profile summaries

def _short(name: str, templates: bool = True) -> str:
    i = name.find("::k_")
    if i >= 0:
        out = name[i + 2:name.find("(", i)]
        return out if templates else out.split("<")[0]
    return name.split("(")[0][:48]


def summarize(dirs, command_note, counter_key=None):
    """Markdown summaries of rocprofv3 CSVs: kernel stats, and per-launch HBM
    traffic from FETCH_SIZE / WRITE_SIZE calibrated against the plain copy."""
    lines = []
    stats = [p for d in dirs for p in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)]
    for p in stats:
        rows = list(csv.DictReader(open(p)))
        lines.append(f"### kernel stats ({os.path.basename(p)})\n")
        lines.append("| kernel | calls | avg us | total ms | % |")
        lines.append("|---|---|---|---|---|")
        for r in rows[:14]:
            lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                         f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} |")
        lines.append("")
    traces = [p for d in dirs for p in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)]
    for p in traces:
        agg = {}
        for r in csv.DictReader(open(p)):
            k = (_short(r["Kernel_Name"]), f"{r['Grid_Size_X']}x{r['Grid_Size_Y']}x{r['Grid_Size_Z']}",
                 r.get("LDS_Block_Size", ""))
            agg.setdefault(k, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        lines.append(f"### per launch shape ({os.path.basename(p)})\n")
        lines.append("| kernel | grid (threads) | LDS bytes | launches | avg us |")
        lines.append("|---|---|---|---|---|")
        for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:16]:
            lines.append(f"| {k[0]} | {k[1]} | {k[2]} | {len(v)} | {sum(v) / len(v) / 1e3:.1f} |")
        lines.append("")
    counters = {}
    for d in dirs:
        for p in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(p)):
                k = (_short(r["Kernel_Name"], False), r.get("Grid_Size", r.get("Grid_Size_X", "?")), r["Counter_Name"])
                counters.setdefault(k, []).append(float(r["Counter_Value"]))
    traffic = None
    if counters and counter_key:
        lines.append("### HBM counters per dispatch (KiB, mean over dispatches)\n")
        lines.append("| kernel | grid | counter | dispatches | KiB |")
        lines.append("|---|---|---|---|---|")
        for k, v in sorted(counters.items()):
            lines.append(f"| {k[0]} | {k[1]} | {k[2]} | {len(v)} | {np.mean(v):.1f} |")
        lines.append("")
        copy_bytes = COPY_N * COPY_N * 4
        cal = {}
        for cn in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = [np.mean(v) for (kn, g, c), v in counters.items()
                    if kn == "k_prolong" and c == cn and str(g).startswith(str(COPY_N * COPY_N))]
            if vals:
                cal[cn] = vals[0] * 1024 / copy_bytes
        lines.append(f"copy calibration (64 MiB read + 64 MiB write): measured/ideal = {cal}\n")
        traffic = {"source_hash": source_hash(), "calibration": cal, "kernels": {}}
        kname = counter_key.rsplit("_l", 1)[0]
        per = {c: float(np.mean([np.mean(v) for (kn, g, cc), v in counters.items() if kn == kname and cc == c]))
               for c in ("FETCH_SIZE", "WRITE_SIZE")}
        if cal.get("FETCH_SIZE") and cal.get("WRITE_SIZE"):
            nbytes = per["FETCH_SIZE"] * 1024 / cal["FETCH_SIZE"] + per["WRITE_SIZE"] * 1024 / cal["WRITE_SIZE"]
            traffic["kernels"][counter_key] = {"fetch_kib": per["FETCH_SIZE"], "write_kib": per["WRITE_SIZE"],
                                               "bytes_per_launch": nbytes}
            lines.append(f"{counter_key}: {nbytes / 1e6:.2f} MB of HBM traffic per launch (calibrated)\n")
    if counters and counter_key:
        # L2 hit rate and instruction mix of the kernel, where those passes ran
        kname = counter_key.rsplit("_l", 1)[0]

        def mean_of(c):
            v = [np.mean(x) for (kn, g, cc), x in counters.items() if kn == kname and cc == c]
            return float(np.mean(v)) if v else None

        derived = {}
        hit, miss = mean_of("TCC_HIT_sum"), mean_of("TCC_MISS_sum")
        if hit is not None and miss is not None and hit + miss > 0:
            derived["l2_hit_rate"] = hit / (hit + miss)
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_WAVES", "SQ_LDS_BANK_CONFLICT",
                  "SQ_ACTIVE_INST_LDS", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES"):
            if mean_of(c) is not None:
                derived[c] = mean_of(c)
        if derived.get("SQ_ACTIVE_INST_LDS"):
            derived["lds_conflict_over_active_cycles"] = derived.get("SQ_LDS_BANK_CONFLICT", 0.0) / derived[
                "SQ_ACTIVE_INST_LDS"]
        if derived:
            lines.append("### derived (mean per dispatch)\n")
            for k, v in derived.items():
                lines.append(f"* {k}: {v:.4g}")
            lines.append("")
            if traffic is None:
                traffic = {"source_hash": source_hash(), "calibration": {}, "kernels": {}}
            traffic["kernels"].setdefault(counter_key, {}).update(derived)
    lines.append(f"command: {command_note}\n")
    return "\n".join(lines), traffic


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--blocks", type=int, default=1, help="measurement blocks combined with the image sketches")
    ap.add_argument("--fan", action="store_true", help="the same workload on a fan beam")
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--level-steps", type=int, default=200, help="steps timed one by one for the per-level table")
    ap.add_argument("--no-race", action="store_true", help="skip the time-to-1e-3 race in the main line")
    ap.add_argument("--default-tiles", action="store_true", help="ignore the autotuned launch shapes")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving latencies in the main line")
    ap.add_argument("--headline-rates", type=float, nargs="+", default=[200.0, 150.0])
    ap.add_argument("--headline-race-seconds", type=float, default=45.0,
                    help="per-method time limit of the race in the main line")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--summarize", nargs="+")
    ap.add_argument("--note", default="")
    ap.add_argument("--counters", help="fwd:LEVEL or bp:LEVEL: launch only that kernel (for --pmc runs)")
    ap.add_argument("--counter-key", help="with --summarize: kernel key the counter CSVs belong to")
    ap.add_argument("--write-traffic", action="store_true", help="with --summarize: update profiles/traffic.json")
    ap.add_argument("--race", action="store_true", help="ImaSk vs full-resolution SAGA, time to --target")
    ap.add_argument("--target", type=float, default=1e-3)
    ap.add_argument("--ref-iters", type=int, default=3000)
    ap.add_argument("--race-epochs", type=float, default=300.0)
    ap.add_argument("--race-seconds", type=float, default=60.0)
    ap.add_argument("--sigma-mults", type=float, nargs="+", default=[1.0, 2.0])
    ap.add_argument("--check-every", type=float, default=10.0, help="epochs between error checks in the race")
    ap.add_argument("--methods", nargs="+", default=["seq_r4", "seq_r1", "imask_r4", "imask_r4_indep", "saga_r1"])
    ap.add_argument("--seq-sigma-mults", type=float, nargs="+", default=[0.125, 0.25, 0.35, 0.5, 0.7, 0.9])
    ap.add_argument("--seq-check-every", type=float, default=1.0)
    ap.add_argument("--batched", action="store_true", help="64 mixed slices in flight")
    ap.add_argument("--slices", type=int, default=64)
    ap.add_argument("--streams", type=int, default=8)
    ap.add_argument("--epochs", type=float, default=30.0)
    ap.add_argument("--serve", action="store_true", help="continuous-batching server under Poisson load")
    ap.add_argument("--rates", type=float, nargs="+", default=[50.0, 75.0, 100.0, 125.0, 150.0, 200.0])
    ap.add_argument("--window", type=float, default=10.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--hbm-gb", type=float, default=64.0)
    ap.add_argument("--chunk", type=float, default=2.0)
    ap.add_argument("--serve-epochs", type=float, default=30.0)
    ap.add_argument("--autograd", action="store_true", help="differentiable unrolled ImaSk")
    ap.add_argument("--oracle-timing", action="store_true", help="FP64 oracle vs GPU on the 64x64 workload")
    ap.add_argument("--oracle-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--study", choices=["stepsize", "tv", "square"], help="fixed-budget PSNR studies")
    ap.add_argument("--study-epochs", type=float, default=100.0)
    ap.add_argument("--study-every", type=float, default=5.0)
    args = ap.parse_args()
    if args.study:
        study(args)
        return
    if args.batched:
        batched(args)
        return
    if args.serve:
        serving(args)
        return
    if args.autograd:
        autograd_bench(args)
        return
    if args.oracle_timing:
        oracle_timing(args)
        return
    if args.race:
        race(args)
        return
    if args.summarize:
        text, traffic = summarize(args.summarize, args.note, args.counter_key)
        print(text)
        if traffic and args.write_traffic:
            old = {}
            if os.path.exists(TRAFFIC_FILE):
                with open(TRAFFIC_FILE) as f:
                    old = json.load(f)
            if old.get("source_hash") == traffic["source_hash"]:
                for k, v in traffic["kernels"].items():
                    old.setdefault("kernels", {}).setdefault(k, {}).update(v)
                if traffic.get("calibration"):
                    old["calibration"] = traffic["calibration"]
                traffic = old
            with open(TRAFFIC_FILE, "w") as f:
                json.dump(traffic, f, indent=1)
        return
    if args.counters:
        counter_run(args.counters, args.fan)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path does not shard "
              f"across GPUs", file=sys.stderr)
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
