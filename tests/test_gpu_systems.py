"""GPU checks of the systems layers: autograd through the projector pair and
through unrolled ImaSk, many problems in flight on several streams, and the
continuous-batching server (each result identical alone and in the mix)."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, f32, host, rel, say

import paper_2412_10249_amd as pk
from paper_2412_10249_amd import autograd as ag
from paper_2412_10249_amd import batch, serve

pytestmark = pytest.mark.gpu


def test_sketch_fn_backward_is_the_transpose():
    g = pk.Geometry(32, 40, 48)
    lv = pk.Levels((0, 1, 2), (0.4, 0.3, 0.3), pk.FULL_UNBIASED)
    work = pk.workspace(g)
    x = dev(synth.random_image(32, 1)).requires_grad_(True)
    v = dev(synth.random_sinogram(40, 48, 2))
    for k in range(3):
        out = ag.SketchFn.apply(x, g, lv, k, False, work)
        (gx,) = torch.autograd.grad((out * v).sum(), x)
        expect = pk.sketch_apply(g, lv, k, v, True, work)
        torch.cuda.synchronize()
        assert torch.equal(gx, expect)
    s = dev(synth.random_sinogram(40, 48, 3)).requires_grad_(True)
    w = dev(synth.random_image(32, 4))
    out = ag.BackprojectFn.apply(s, g, 1, work)
    (gs,) = torch.autograd.grad((out * w).sum(), s)
    assert torch.equal(gs, pk.project(g, 1, w, work))


def _problem(n=32, na=48, nd=48, seed=0):
    x_true, b = synth.ct_problem(n, na, nd, 1e4, 1000 + seed, 2000 + seed)
    return f32(x_true), f32(b)


def test_unrolled_matches_library_step():
    n, na, nd = 32, 48, 48
    g = pk.Geometry(n, na, nd)
    lv = pk.Levels.uniform((0, 1, 2))
    _, b = _problem(n, na, nd)
    lam, sigma, iters = 0.5, 0.02, 9
    with torch.no_grad():
        xu = ag.unrolled_imask(dev(b), torch.tensor(lam, device="cuda"), g, lv, sigma, iters)
    prob = pk.Problem(g, lv, pk.Regularizer(pk.REG_TIKHONOV, lam), pk.Params(sigma, 42, 0), dev(b))
    prob.step(iters)
    assert rel(host(xu), host(prob.x_cur)) <= 1e-5


def test_unrolled_gradients_match_finite_differences():
    """Loss 1/2|x^K - x_true|^2 with b = K x_in: d/dx_in (along a random
    direction) and d/dlam against central differences."""
    n, na, nd = 32, 48, 48
    g = pk.Geometry(n, na, nd)
    lv = pk.Levels.uniform((0, 1, 2))
    work = pk.workspace(g)
    x_true, _ = _problem(n, na, nd, 5)
    xt = dev(x_true)
    x_in = dev(synth.random_image(n, 6) * 0.5 + 0.5)
    sigma, iters = 0.03, 8

    def loss(xin, lam):
        b = ag.ProjectFn.apply(xin, g, 0, work)
        xk = ag.unrolled_imask(b, lam, g, lv, sigma, iters, work=work, checkpoint_every=2)
        return 0.5 * ((xk - xt) ** 2).sum()

    xin = x_in.clone().requires_grad_(True)
    lam = torch.tensor(0.3, device="cuda", requires_grad=True)
    L = loss(xin, lam)
    gx, gl = torch.autograd.grad(L, (xin, lam))
    d = dev(np.random.default_rng(9).standard_normal((n, n)))
    with torch.no_grad():
        h = 1e-2
        fd = (loss(x_in + h * d, lam) - loss(x_in - h * d, lam)) / (2 * h)
        hl = 1e-3
        fdl = (loss(x_in, lam + hl) - loss(x_in, lam - hl)) / (2 * hl)
    dd = float((gx * d).sum())
    say(f"directional {dd} vs {float(fd)}; dlam {float(gl)} vs {float(fdl)}")
    assert abs(dd - float(fd)) <= 2e-3 * max(1.0, abs(float(fd)))
    assert abs(float(gl) - float(fdl)) <= 1e-2 * max(1e-3, abs(float(fdl)))


def test_batch_runner_equals_alone():
    geoms = [(64, 96, 96), (32, 48, 48), (48, 72, 72), (64, 96, 96)]
    probs, alone = [], []
    for q, (n, na, nd) in enumerate(geoms):
        _, b = synth.ct_problem(n, na, nd, 1e4, 1020 + q, 2020 + q)

        def mk():
            return pk.Problem(pk.Geometry(n, na, nd), pk.Levels.uniform((0, 1, 2)),
                              pk.Regularizer(pk.REG_TIKHONOV, 0.1), pk.Params(0.01, 42, q), dev(b))
        probs.append(mk())
        alone.append(mk())
    runner = batch.BatchRunner(probs, n_streams=3)
    runner.step_all(12)
    runner.synchronize()
    for p in alone:
        p.step(12)
    torch.cuda.synchronize()
    for a, c in zip(probs, alone):
        assert torch.equal(a.x_cur, c.x_cur) and torch.equal(a.y_cur, c.y_cur)
        assert batch.footprint_bytes(a) == batch.state_bytes(a.geom, a.levels)


def test_server_results_equal_alone():
    levels_for = lambda n: pk.Levels.uniform((0, 1, 2))  # noqa: E731
    reg = pk.Regularizer(pk.REG_TIKHONOV, 0.1)
    sigma_for = lambda geom: 0.01  # noqa: E731
    data = {n: f32(synth.ct_problem(n, 3 * n // 2, 3 * n // 2, 1e4, 1030 + n, 2030 + n)[1]) for n in (32, 64)}
    ex = serve.GpuExecutor(4, levels_for, reg, sigma_for)
    sch = serve.Scheduler(ex, hbm_budget=64 << 20, max_active=4, chunk_epochs=1.0)
    arrivals = [(0.001 * i, 32 if i % 3 else 64) for i in range(10)]
    done = serve.run_load(sch, arrivals, lambda rid, n, t: serve.Request(rid, n, t, 4.0, data=dev(data[n])))
    assert len(done) == 10 and all(r.latency is not None and r.latency > 0 for r in done)
    for r in done:
        geom = pk.Geometry(r.n, 3 * r.n // 2, 3 * r.n // 2)
        p = pk.Problem(geom, levels_for(r.n), reg, pk.Params(0.01, 42, r.rid), dev(data[r.n]))
        p.solve(4.0, pk.BUDGET_EPOCHS)
        torch.cuda.synchronize()
        assert torch.equal(p.x_cur, r.result), r.rid
