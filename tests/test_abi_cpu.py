"""Host-side checks of libimask that need no GPU: the library loads, exports
every function include/imask.h declares, validates arguments before touching
the device, and its host sketch draw equals the oracle's bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2412_10249_amd import _abi
from paper_2412_10249_amd import imask as im

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "imask.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t)\s+(imask_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    names = _header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_abi.EXPORTS)


def test_struct_sizes_match_c_layout():
    assert ctypes.sizeof(_abi.Geometry) == 4 * 3 + 4 + 8 * 3 + 8 + 8 * 2
    assert ctypes.sizeof(_abi.Levels) == 4 + 32 + 4 + 64 + 4 + 4
    assert ctypes.sizeof(_abi.Params) == 8 + 8 + 4 + 4 + 8 + 4 + 4 + 4 + 4
    assert ctypes.sizeof(_abi.State) == 8 * 7 + 8 + 8 + 8 + 8 + 16 + 8


def test_workspace_and_table_sizes():
    g = _abi.Geometry(64, 90, 92, 0.0, 0.0)
    assert _abi.lib().imask_workspace_bytes(ctypes.byref(g)) > 4 * 64 * 64 * 4
    lv = im.Levels((0, 1, 2), (1 / 3,) * 3).c()
    assert _abi.lib().imask_phi_floats(ctypes.byref(g), ctypes.byref(lv)) == 64 * 64 + 32 * 32 + 16 * 16


@pytest.mark.parametrize("geom", [(0, 90, 92), (63, 90, 92), (40, 90, 92), (64, 0, 92), (64, 90, -1)])
def test_invalid_geometry_rejected_before_any_launch(geom):
    g = _abi.Geometry(*geom, 0.0, 0.0)
    assert _abi.lib().imask_workspace_bytes(ctypes.byref(g)) == 0
    rc = _abi.lib().imask_project(ctypes.byref(g), 0, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                  ctypes.c_void_p(16), None)
    assert rc == _abi.EINVAL


def test_listed_angles_and_extent_validated():
    L = _abi.lib()
    good = im.Geometry(64, 5, 92, extent=2.0, angles=(0.1, 1.0, 2.0, 4.0, -7.5))
    g0 = _abi.Geometry(64, 5, 92, 0.0, 0.0)
    assert L.imask_workspace_bytes(ctypes.byref(good.c())) == L.imask_workspace_bytes(ctypes.byref(g0)) > 0
    for bad in [im.Geometry(64, 3, 92, angles=(0.1, float("nan"), 0.2)),
                im.Geometry(64, 3, 92, angles=(0.1, float("inf"), 0.2)),
                im.Geometry(64, 3, 92, extent=float("nan"))]:
        gc = bad.c()
        assert L.imask_workspace_bytes(ctypes.byref(gc)) == 0
        assert L.imask_prepare(ctypes.byref(gc), ctypes.c_void_p(16), 1 << 30, None) == _abi.EINVAL
    with pytest.raises(_abi.ImaskError):
        im.Geometry(64, 3, 92, angles=(0.1, 0.2))
    # spacing within [1/64, 64] pixels of 2E/N, offset within 4E
    pix = 2 * 2.0 / 64
    for sp, off, ok in [(pix / 64, 0.0, True), (pix / 65, 0.0, False), (64 * pix, 0.0, True),
                        (65 * pix, 0.0, False), (0.0, 8.0, True), (0.0, -8.01, False)]:
        gc = im.Geometry(64, 3, 92, det_spacing=sp, det_offset=off, extent=2.0).c()
        assert (L.imask_workspace_bytes(ctypes.byref(gc)) > 0) == ok, (sp, off)


@pytest.mark.parametrize("bad", [
    ((1, 2), (0.5, 0.5)),          # level 0 missing
    ((0, 0), (0.5, 0.5)),          # not increasing
    ((0, 1), (0.6, 0.6)),          # p does not sum to one
    ((0, 1), (1.0, 0.0)),          # p must be positive
    ((0, 9), (0.5, 0.5)),          # deeper than the geometry allows
])
def test_invalid_level_sets_rejected(bad):
    g = _abi.Geometry(64, 10, 10, 0.0, 0.0)
    lv = im.Levels(*bad).c()
    assert _abi.lib().imask_phi_floats(ctypes.byref(g), ctypes.byref(lv)) == 0


def test_invalid_step_arguments_rejected():
    g = _abi.Geometry(64, 10, 10, 0.0, 0.0)
    lv = im.Levels((0, 1), (0.5, 0.5)).c()
    reg = _abi.Reg(_abi.REG_TIKHONOV, 0.01, 0.0, 1e-3, 10)
    prm = _abi.Params(0.01, 1, 0)
    s = _abi.State()  # null pointers
    b = (ctypes.c_void_p * 1)(16)
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), b,
                                 ctypes.byref(s), 1, None) == _abi.EINVAL
    s.x[0], s.x[1], s.y[0], s.y[1] = 16, 32, 48, 64
    s.phi, s.psi, s.work = 80, 96, 112
    bad_reg = _abi.Reg(_abi.REG_TIKHONOV, -1.0, 0.0, 1e-3, 10)
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(bad_reg), ctypes.byref(prm),
                                 b, ctypes.byref(s), 1, None) == _abi.EINVAL
    tv = _abi.Reg(_abi.REG_SMOOTH_TV, 0.01, 1.0, 1e-3, 99)
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(tv), ctypes.byref(prm),
                                 b, ctypes.byref(s), 1, None) == _abi.EINVAL
    bad_prm = _abi.Params(-0.5, 1, 0)
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(bad_prm),
                                 b, ctypes.byref(s), 1, None) == _abi.EINVAL
    bad_prm = _abi.Params(0.01, 1, 0, _abi.SCHEDULE_PARALLEL, 1.0, _abi.DRAW_COMMON, 0, 1, 3)  # reserved != 0
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(bad_prm),
                                 b, ctypes.byref(s), 1, None) == _abi.EINVAL
    assert _abi.lib().imask_solve(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm),
                                  b, ctypes.byref(s), 5.0, 7, None) == _abi.EINVAL
    # the TV prior needs two distinct dual buffers and a positive weight
    tvr = _abi.Reg(_abi.REG_TV, 0.01, 1.0, 0.0, 10)
    s.tvd[0], s.tvd[1] = 144, 144
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(tvr), ctypes.byref(prm),
                                 b, ctypes.byref(s), 1, None) == _abi.EINVAL
    s.tvd[0], s.tvd[1] = 144, 160
    tv0 = _abi.Reg(_abi.REG_TV, 0.01, 0.0, 0.0, 10)
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(tv0), ctypes.byref(prm),
                                 b, ctypes.byref(s), 1, None) == _abi.EINVAL
    s.tvd[0], s.tvd[1] = None, None
    # schedules: unknown value; sequential without xbar, with xbar aliasing x, with theta outside [0, 1]
    for sched, theta, xbar in [(5, 1.0, 128), (_abi.SCHEDULE_SEQUENTIAL, 1.0, None),
                               (_abi.SCHEDULE_SEQUENTIAL, 1.0, 16), (_abi.SCHEDULE_SEQUENTIAL, 1.5, 128),
                               (_abi.SCHEDULE_SEQUENTIAL, -0.1, 128)]:
        s.xbar = xbar
        bad = _abi.Params(0.01, 1, 0, sched, theta)
        assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(bad),
                                     b, ctypes.byref(s), 1, None) == _abi.EINVAL, (sched, theta, xbar)


@pytest.mark.parametrize("seed,stream,p", [(42, 0, (1 / 3,) * 3), (7, 5, (0.25,) * 4),
                                           (2 ** 63 + 11, 123, (0.3, 0.3, 0.2, 0.2)), (1, 9, (1.0,))])
def test_host_draws_match_oracle_bitwise(seed, stream, p):
    lv = im.Levels(tuple(range(len(p))), p)
    got = im.draws(im.Params(0.1, seed, stream), lv, 1000, 100_000)
    exp = oracle.draws(seed, stream, 1000, 100_000, list(p))
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("consts", [(6.0, 2.0, 6.0, 1 / 3), (543.0, 181.0, 543.0, 1 / 3), (5.7, 1.9, 5.8, 0.25),
                                    (50.0, 0.5, 80.0, 0.1)])
def test_sigma_thm3_matches_oracle(consts):
    from oracle import steps

    L2, lb, lp, pmin = consts
    sig, th = im.sigma_thm3(L2, lb, lp, pmin, 60)
    osig, oth, _, _ = steps.sigma_thm3(L2, lb, lp, pmin, 60, 60)
    assert sig == pytest.approx(osig, rel=1e-12) and th == pytest.approx(oth, rel=1e-12)


def test_sigma_thm3_rejects_bad_constants():
    with pytest.raises(im.ImaskError):
        im.sigma_thm3(-1.0, 1.0, 1.0, 0.5)
    with pytest.raises(im.ImaskError):
        im.sigma_thm3(1.0, 1.0, 1.0, 0.0)


def test_sigma_balamurugan_matches_oracle():
    from oracle import steps

    for L2, lb in [(5431.3, 1357.9), (7.0, 2.5), (1.0, 1.0)]:
        assert abs(im.sigma_balamurugan(L2, lb) - steps.sigma_balamurugan(L2, lb)) <= 1e-15 * steps.sigma_balamurugan(L2, lb)
    out = ctypes.c_double()
    assert _abi.lib().imask_sigma_balamurugan(-1.0, 1.0, ctypes.byref(out)) == _abi.EINVAL



def test_compact_tables_need_parallel_schedule():
    g = _abi.Geometry(64, 10, 10, 0.0, 0.0)
    lv = im.Levels((0, 1), (0.5, 0.5)).c()
    reg = _abi.Reg(_abi.REG_TIKHONOV, 0.01, 0.0, 1e-3, 10)
    s = _abi.State()
    s.x[0], s.x[1], s.y[0], s.y[1] = 16, 32, 48, 64
    s.phi, s.psi, s.work, s.xbar, s.ztab = 80, 96, 112, 128, 144
    b = (ctypes.c_void_p * 1)(16)
    seq = _abi.Params(0.01, 1, 0, _abi.SCHEDULE_SEQUENTIAL, 1.0)
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(seq), b,
                                 ctypes.byref(s), 1, None) == _abi.ENOTSUP
    s.ztab = 80  # aliases phi
    par = _abi.Params(-1.0, 1, 0, _abi.SCHEDULE_PARALLEL, 1.0)  # and an invalid sigma: never launches
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(par), b,
                                 ctypes.byref(s), 1, None) == _abi.EINVAL


def test_independent_draws_limits():
    g = _abi.Geometry(64, 10, 10, 0.0, 0.0)
    lv = im.Levels((0, 1), (0.5, 0.5)).c()
    reg = _abi.Reg(_abi.REG_TIKHONOV, 0.01, 0.0, 1e-3, 10)
    s = _abi.State()
    s.x[0], s.x[1], s.y[0], s.y[1] = 16, 32, 48, 64
    s.phi, s.psi, s.work, s.xbar = 80, 96, 112, 128
    b = (ctypes.c_void_p * 1)(16)
    for prm, want in [(_abi.Params(0.01, 1, 0, _abi.SCHEDULE_PARALLEL, 1.0, 7, 1), _abi.EINVAL),
                      (_abi.Params(0.01, 1, 0, _abi.SCHEDULE_SEQUENTIAL, 1.0, _abi.DRAW_INDEPENDENT, 1),
                       _abi.ENOTSUP)]:
        assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), b,
                                     ctypes.byref(s), 1, None) == want
    s.ztab = 144
    prm = _abi.Params(0.01, 1, 0, _abi.SCHEDULE_PARALLEL, 1.0, _abi.DRAW_INDEPENDENT, 1)
    assert _abi.lib().imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), b,
                                 ctypes.byref(s), 1, None) == _abi.ENOTSUP



def test_remaining_entry_points_validate_before_any_launch():
    """Every entry point rejects bad arguments with IMASK_EINVAL (or ESIZE)
    before it touches the device; the pointers passed are never dereferenced."""
    L = _abi.lib()
    g = _abi.Geometry(64, 10, 12, 0.0, 0.0)
    gr = ctypes.byref(g)
    lv = im.Levels((0, 1), (0.5, 0.5)).c()
    P = ctypes.c_void_p
    a, b2, w = P(16), P(32), P(4096)
    need = L.imask_workspace_bytes(gr)
    assert L.imask_prepare(gr, None, need, None) == _abi.EINVAL
    assert L.imask_prepare(gr, w, need - 1, None) == _abi.ESIZE
    for bad in (-1, 7):
        assert L.imask_project(gr, bad, w, a, b2, None) == _abi.EINVAL
        assert L.imask_backproject(gr, bad, w, a, b2, None) == _abi.EINVAL
    assert L.imask_resample(64, 1, _abi.RESTRICT, None, a, a, None) == _abi.EINVAL     # in == out
    assert L.imask_resample(64, 7, _abi.RESTRICT, None, a, b2, None) == _abi.EINVAL    # too deep
    assert L.imask_resample(64, 1, 99, None, a, b2, None) == _abi.EINVAL               # unknown mode
    assert L.imask_resample(63, 1, _abi.RESTRICT, None, a, b2, None) == _abi.EINVAL    # bad side
    for k in (-1, 2):
        assert L.imask_sketch_apply(gr, ctypes.byref(lv), k, 0, w, a, b2, None) == _abi.EINVAL
    assert L.imask_sketch_apply(gr, ctypes.byref(lv), 0, 0, w, a, a, None) == _abi.EINVAL
    ms = ctypes.c_double()
    assert L.imask_time_kernel(gr, 0, 0, w, a, b2, 0, None, ctypes.byref(ms)) == _abi.EINVAL   # reps
    assert L.imask_time_kernel(gr, 7, 0, w, a, b2, 3, None, ctypes.byref(ms)) == _abi.EINVAL   # which
    assert L.imask_time_kernel(gr, 0, 9, w, a, b2, 3, None, ctypes.byref(ms)) == _abi.EINVAL   # level
    out = (ctypes.c_double * 3)()
    assert L.imask_step_constants(gr, ctypes.byref(lv), 0.0, 10, 1, w, a, out, None) == _abi.EINVAL
    assert L.imask_step_constants(gr, ctypes.byref(lv), 1.0, 0, 1, w, a, out, None) == _abi.EINVAL
    draws = (ctypes.c_int32 * 4)()
    prm = _abi.Params(0.01, 1, 0)
    assert L.imask_draws(ctypes.byref(prm), ctypes.byref(lv), 0, -1, draws) == _abi.EINVAL
    assert L.imask_draws(ctypes.byref(prm), ctypes.byref(lv), 0, 4, draws) == _abi.OK
    # the timed steps: negative counts, a missing output array, a null state
    reg = _abi.Reg(_abi.REG_TIKHONOV, 0.01, 0.0, 1e-3, 10)
    st = _abi.State()
    tms = (ctypes.c_float * 4)()
    assert L.imask_step_timed(gr, ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), a, ctypes.byref(st), -1,
                              tms, None) == _abi.EINVAL
    assert L.imask_step_timed(gr, ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), a, ctypes.byref(st), 4,
                              None, None) == _abi.EINVAL
    assert L.imask_step_timed(gr, ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), a, ctypes.byref(st), 4,
                              tms, None) == _abi.EINVAL


def test_measurement_blocks_validated():
    L = _abi.lib()
    g = _abi.Geometry(64, 10, 12, 0.0, 0.0)
    base = L.imask_phi_floats(ctypes.byref(g), ctypes.byref(im.Levels((0, 1), (0.5, 0.5)).c()))
    assert L.imask_phi_floats(ctypes.byref(g), ctypes.byref(im.Levels((0, 1), (0.5, 0.5), 0, 3).c())) == 3 * base
    assert L.imask_phi_floats(ctypes.byref(g), ctypes.byref(im.Levels((0, 1), (0.5, 0.5), 0, 11).c())) == 0
    assert L.imask_phi_floats(ctypes.byref(g), ctypes.byref(im.Levels((0, 1), (0.5, 0.5), 0, -2).c())) == 0
    lv = im.Levels((0, 1), (0.5, 0.5), 0, 3).c()
    reg = _abi.Reg(_abi.REG_TIKHONOV, 0.01, 0.0, 1e-3, 10)
    s = _abi.State()
    s.x[0], s.x[1], s.y[0], s.y[1] = 16, 32, 48, 64
    s.phi, s.psi, s.work, s.xbar = 80, 96, 112, 128
    b = (ctypes.c_void_p * 1)(16)
    for prm in (_abi.Params(0.01, 1, 0, _abi.SCHEDULE_SEQUENTIAL, 1.0),
                _abi.Params(0.01, 1, 0, _abi.SCHEDULE_PARALLEL, 1.0, _abi.DRAW_INDEPENDENT, 1)):
        assert L.imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), b,
                            ctypes.byref(s), 1, None) == _abi.ENOTSUP
    listed = im.Geometry(64, 10, 12, angles=tuple(0.1 * a for a in range(10))).c()
    prm = _abi.Params(0.01, 1, 0)
    assert L.imask_step(1, ctypes.byref(listed), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), b,
                        ctypes.byref(s), 1, None) == _abi.ENOTSUP
    bad = im.Levels((0, 1), (0.5, 0.5), 0, 11).c()
    assert L.imask_step(1, ctypes.byref(g), ctypes.byref(bad), ctypes.byref(reg), ctypes.byref(prm), b,
                        ctypes.byref(s), 1, None) == _abi.EINVAL
    out = (ctypes.c_int32 * 64)()
    assert L.imask_block_draws(ctypes.byref(prm), ctypes.byref(lv), 5, 64, out) == _abi.OK
    assert list(out) == oracle.block_draws(1, 0, 5, 64, 3)


def test_fan_geometry_validated():
    """Fan beam: source distance in (2E, 1e4 E], detector distance in
    [0, 1e4 E], spacing and offset bounds taken in magnified pixels, and no
    measurement blocks over listed views."""
    L = _abi.lib()
    E = 1.5

    def ok(**kw):
        gc = im.Geometry(64, 12, 40, extent=E, **kw).c()
        return L.imask_workspace_bytes(ctypes.byref(gc)) > 0

    par = L.imask_workspace_bytes(ctypes.byref(im.Geometry(64, 12, 40, extent=E).c()))
    fan = L.imask_workspace_bytes(ctypes.byref(im.Geometry(64, 12, 40, extent=E, src_dist=4.0, det_dist=2.0).c()))
    assert fan > par > 0  # the ray and view tables
    assert ok(src_dist=2 * E * 1.0001) and not ok(src_dist=2 * E) and not ok(src_dist=-4.0)
    assert ok(src_dist=1e4 * E) and not ok(src_dist=1.0001e4 * E)
    assert not ok(src_dist=4.0, det_dist=-0.1) and not ok(src_dist=4.0, det_dist=1.0001e4 * E)
    assert not ok(src_dist=float("nan")) and not ok(src_dist=4.0, det_dist=float("inf"))
    assert not ok(det_dist=float("nan"))  # checked for parallel beam too
    mag_pix = 2 * E / 64 * (4.0 + 2.0) / 4.0
    for sp, off, good in [(mag_pix / 64, 0.0, True), (mag_pix / 65, 0.0, False), (64 * mag_pix, 0.0, True),
                          (65 * mag_pix, 0.0, False), (0.0, 4 * E * 1.5, True), (0.0, -4 * E * 1.5 * 1.001, False)]:
        assert ok(src_dist=4.0, det_dist=2.0, det_spacing=sp, det_offset=off) == good, (sp, off)
    g = im.Geometry(64, 10, 12, src_dist=3.0, det_dist=1.0, angles=tuple(0.3 * a for a in range(10))).c()
    lv = im.Levels((0, 1), (0.5, 0.5), 0, 3).c()
    reg = _abi.Reg(_abi.REG_TIKHONOV, 0.01, 0.0, 1e-3, 10)
    s = _abi.State()
    s.x[0], s.x[1], s.y[0], s.y[1] = 16, 32, 48, 64
    s.phi, s.psi, s.work = 80, 96, 112
    b = (ctypes.c_void_p * 1)(16)
    prm = _abi.Params(0.01, 1, 0)
    assert L.imask_step(1, ctypes.byref(g), ctypes.byref(lv), ctypes.byref(reg), ctypes.byref(prm), b,
                        ctypes.byref(s), 1, None) == _abi.ENOTSUP


def test_partial_image_buffer_sizing():
    """The transposes' partial-image buffer holds up to 64 N^2 floats while
    that stays within 32 MiB (parallel beam) or 256 MiB (fan beam), never
    fewer than 16 N^2: the fan workspace exceeds the parallel one by the
    difference, and the parallel one grows by it from 16 N^2, give or take
    the small ray, view and table entries, the band partial sinograms and the
    alignment (under 64 KiB here)."""
    L = _abi.lib()

    def ws(n, fan):
        g = im.Geometry(n, 8, 16, src_dist=4.0 if fan else 0.0, det_dist=2.0).c()
        return L.imask_workspace_bytes(ctypes.byref(g))

    def part(n, cap):
        return max(16 * n * n, min(64 * n * n, cap))

    for n, par_images, fan_images in ((64, 64, 64), (512, 32, 64), (1024, 16, 64), (2048, 16, 16),
                                      (4096, 16, 16)):
        assert part(n, 1 << 23) == par_images * n * n and part(n, 1 << 26) == fan_images * n * n
        diff = ws(n, True) - ws(n, False)
        assert abs(diff - (fan_images - par_images) * n * n * 4) <= 65536, (n, diff)
    # the parallel workspace against one with 16 N^2: grows by the extra images
    assert abs(ws(512, False) - ws(1024, False) / 4 - 16 * 512 * 512 * 4) <= 65536


def test_noalloc_transpose_validates_before_any_device_call():
    """The workspace-free transpose checks its arguments and whether the
    geometry fits its static array before it looks up the array or launches
    anything (so these calls need no GPU)."""
    L = _abi.lib()
    p = ctypes.c_void_p(16)

    def call(g, lvl=0, sino=p, out=p):
        return L.imask_backproject_noalloc(ctypes.byref(g.c()), lvl, sino, out, None)

    assert call(im.Geometry(64, 90, 92), sino=None) == _abi.EINVAL
    assert call(im.Geometry(64, 90, 92), out=None) == _abi.EINVAL
    assert call(im.Geometry(64, 90, 92), lvl=6) == _abi.EINVAL
    assert call(im.Geometry(63, 90, 92)) == _abi.EINVAL
    assert call(im.Geometry(64, 3, 92, angles=(0.1, 0.2, 0.3))) == _abi.ENOTSUP
    assert call(im.Geometry(64, 90, 92, src_dist=4.0, det_dist=2.0)) == _abi.ENOTSUP
    # P + N^2 + 16 (lmax + 1) n_angles floats against the 48 MiB array, with
    # P = max(16 N^2, min(64 N^2, 2^23)) partial-image floats: N = 512 and
    # 8 levels leave room for 30720 angles
    assert call(im.Geometry(1024, 90, 92)) == _abi.ESIZE
    assert call(im.Geometry(512, 30721, 768)) == _abi.ESIZE
    assert (1 << 23) + 512 * 512 + 16 * 8 * 30720 <= _abi.NOALLOC_SCRATCH_BYTES // 4


def test_tiles_table_validates_and_round_trips():
    """imask_set_tiles keeps one entry per (grid side, angles, bins), refuses
    unsupported shapes, and a NULL entry restores the defaults."""
    from paper_2412_10249_amd import autotune

    L = _abi.lib()
    assert autotune.get_tiles(256, 384, 384) == {"bp": [0, 0], "bp_wg": 0, "fwd_lds_kb": 0}
    autotune.set_tiles(256, 384, 384, (4, 4), 2048, 96)
    assert autotune.get_tiles(256, 384, 384) == {"bp": [4, 4], "bp_wg": 2048, "fwd_lds_kb": 96}
    assert autotune.get_tiles(256, 384, 385)["bp_wg"] == 0  # another geometry keeps the defaults
    for bad in [(3, 3, 0, 0), (2, 8, 32, 0), (2, 8, 0, 200), (8, 8, 0, 0)]:
        t = _abi.Tiles(*bad)
        assert L.imask_set_tiles(256, 384, 384, ctypes.byref(t)) == _abi.EINVAL, bad
    assert autotune.get_tiles(256, 384, 384)["bp"] == [4, 4]  # a refused call changes nothing
    autotune.reset_tiles(256, 384, 384)
    assert autotune.get_tiles(256, 384, 384) == {"bp": [0, 0], "bp_wg": 0, "fwd_lds_kb": 0}


def test_tuned_forward_budget_keeps_the_workspace_size():
    """A tuned forward band budget never needs more bands than the default,
    so a workspace's size (and layout) does not depend on the tiles."""
    from paper_2412_10249_amd import autotune

    L = _abi.lib()
    g = im.Geometry(256, 384, 384).c()
    before = L.imask_workspace_bytes(ctypes.byref(g))
    for kb in (78, 96, 128, 156):
        autotune.set_tiles(256, 384, 384, (0, 0), 0, kb)
        assert L.imask_workspace_bytes(ctypes.byref(g)) == before
    autotune.reset_tiles(256, 384, 384)


def test_batch_entry_points_validate_before_any_device_call():
    L = _abi.lib()
    n = 2
    G = (_abi.Geometry * n)(im.Geometry(64, 90, 92).c(), im.Geometry(32, 48, 48).c())
    Lv = (_abi.Levels * n)(im.Levels((0, 1, 2), (1 / 3,) * 3).c(), im.Levels((0,), (1.0,)).c())
    assert L.imask_batch_bytes(n, G, Lv) > 0
    assert L.imask_batch_bytes(0, G, Lv) == 0
    Gf = (_abi.Geometry * 1)(im.Geometry(64, 90, 92, src_dist=4.0, det_dist=2.0).c())
    assert L.imask_batch_bytes(1, Gf, Lv) == 0
    buf = ctypes.c_void_p(256)
    assert L.imask_batch_step(1, Gf, Lv, buf, 1, None) == _abi.ENOTSUP
    assert L.imask_batch_step(n, G, Lv, None, 1, None) == _abi.EINVAL
    assert L.imask_batch_step(n, G, Lv, buf, -1, None) == _abi.EINVAL
    assert L.imask_batch_state(0, Lv, buf, None, None) == _abi.EINVAL
