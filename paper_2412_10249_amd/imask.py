"""PyTorch-facing binding of libimask: tensors in, tensors out.

Each function checks shapes/dtypes, passes raw device pointers and the
current HIP stream to the C ABI, and raises ImaskError on a nonzero return.
No arithmetic of the method happens here.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi
from ._abi import ImaskError, check, lib


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, shape, name: str) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ImaskError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ImaskError(f"{name} must be contiguous float32")
    if tuple(t.shape) != tuple(shape):
        raise ImaskError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


@dataclass(frozen=True)
class Geometry:
    """CT geometry: N x N image on [-E,E]^2 (E = extent) and n_det bins.
    Parallel beam (src_dist = 0): n_angles angles a*pi/n_angles or the listed
    ones (radians); spacing <= 0 selects the full-resolution pixel size 2E/N.
    Fan beam (src_dist = D > 2E): n_angles source positions 2 pi a/n_angles
    (or listed) at distance D, a flat detector det_dist beyond the centre;
    spacing <= 0 selects the magnified pixel size 2E/N (D + det_dist)/D."""
    n: int
    n_angles: int
    n_det: int
    det_spacing: float = 0.0
    det_offset: float = 0.0
    extent: float = 1.0
    angles: tuple = None
    src_dist: float = 0.0
    det_dist: float = 0.0

    def __post_init__(self):
        if self.angles is not None:
            a = tuple(float(t) for t in self.angles)
            if len(a) != self.n_angles:
                raise ImaskError(f"{len(a)} angles listed for n_angles = {self.n_angles}")
            object.__setattr__(self, "angles", a)
            object.__setattr__(self, "_carr", (ctypes.c_double * len(a))(*a))

    def c(self) -> _abi.Geometry:
        # the struct points into this object's angle array: keep self alive
        ang = ctypes.cast(self._carr, ctypes.POINTER(ctypes.c_double)) if self.angles is not None else None
        return _abi.Geometry(self.n, self.n_angles, self.n_det, self.det_spacing, self.det_offset, self.extent, ang,
                             self.src_dist, self.det_dist)

    @property
    def sino_shape(self):
        return (self.n_angles, self.n_det)

    @property
    def image_shape(self):
        return (self.n, self.n)


@dataclass(frozen=True)
class Levels:
    """Resolution set (log2 factors, first 0), probabilities p, and the
    number of measurement blocks combined with the image sketches (1: none)."""
    log2f: tuple
    p: tuple
    full_mode: int = _abi.FULL_PAPER
    n_blocks: int = 1

    def c(self) -> _abi.Levels:
        lv = _abi.Levels()
        lv.r = len(self.log2f)
        for k, (l, pk) in enumerate(zip(self.log2f, self.p)):
            lv.log2f[k] = int(l)
            lv.p[k] = float(pk)
        lv.full_mode = int(self.full_mode)
        lv.n_blocks = int(self.n_blocks)
        return lv

    @property
    def r(self) -> int:
        return len(self.log2f)

    @staticmethod
    def uniform(log2f, full_mode: int = _abi.FULL_PAPER, n_blocks: int = 1) -> "Levels":
        r = len(log2f)
        return Levels(tuple(log2f), tuple([1.0 / r] * r), full_mode, n_blocks)


@dataclass(frozen=True)
class Regularizer:
    kind: int = _abi.REG_TIKHONOV
    lam: float = 1e-2
    tv_weight: float = 0.0
    tv_eps: float = 1e-3
    tv_inner: int = 10

    def c(self) -> _abi.Reg:
        return _abi.Reg(self.kind, self.lam, self.tv_weight, self.tv_eps, self.tv_inner)


@dataclass(frozen=True)
class Params:
    """Step size, draw stream, the schedule (Alg. 1's parallel update or the
    ImaSk-Seq variant of Sec. 5 with extrapolation theta) and the draw mode
    (one index per iteration, or independent primal/dual indices with the
    dual one from dual_stream_id).  check_finite: after each call, test x and
    y for NaN/infinity (one synchronisation) and raise ImaskError if found."""
    sigma: float
    seed: int = 42
    stream_id: int = 0
    schedule: int = _abi.SCHEDULE_PARALLEL
    theta: float = 1.0
    draw_mode: int = _abi.DRAW_COMMON
    dual_stream_id: int = 0
    check_finite: bool = False

    def c(self) -> _abi.Params:
        return _abi.Params(self.sigma, self.seed, self.stream_id, self.schedule, self.theta, self.draw_mode,
                           self.dual_stream_id, int(bool(self.check_finite)), 0)


def workspace(g: Geometry, device="cuda") -> torch.Tensor:
    nbytes = lib().imask_workspace_bytes(ctypes.byref(g.c()))
    if nbytes == 0:
        raise ImaskError("invalid geometry")
    w = torch.empty(nbytes, dtype=torch.uint8, device=device)
    check(lib().imask_prepare(ctypes.byref(g.c()), _ptr(w), nbytes, _stream()), "imask_prepare")
    return w


def project(g: Geometry, log2f: int, x: torch.Tensor, work: torch.Tensor, out: torch.Tensor | None = None):
    """sino = R_l T_l x."""
    _need(x, g.image_shape, "x")
    if out is None:
        out = torch.empty(g.sino_shape, dtype=torch.float32, device=x.device)
    _need(out, g.sino_shape, "out")
    check(lib().imask_project(ctypes.byref(g.c()), log2f, _ptr(work), _ptr(x), _ptr(out), _stream()),
          "imask_project")
    return out


def backproject(g: Geometry, log2f: int, sino: torch.Tensor, work: torch.Tensor, out: torch.Tensor | None = None):
    """x = T_l^T R_l^T sino (exact transpose of project)."""
    _need(sino, g.sino_shape, "sino")
    if out is None:
        out = torch.empty(g.image_shape, dtype=torch.float32, device=sino.device)
    _need(out, g.image_shape, "out")
    check(lib().imask_backproject(ctypes.byref(g.c()), log2f, _ptr(work), _ptr(sino), _ptr(out), _stream()),
          "imask_backproject")
    return out


def backproject_noalloc(g: Geometry, log2f: int, sino: torch.Tensor, out: torch.Tensor):
    """backproject without a workspace: the library's static per-GPU array
    holds the transpose's constants and partial images.  `out` is the
    caller's (nothing is allocated here either)."""
    _need(sino, g.sino_shape, "sino")
    _need(out, g.image_shape, "out")
    check(lib().imask_backproject_noalloc(ctypes.byref(g.c()), log2f, _ptr(sino), _ptr(out), _stream()),
          "imask_backproject_noalloc")
    return out


def resample(x: torch.Tensor, log2f: int, mode: int, levels: Levels | None = None):
    n = x.shape[-1]
    nl = n >> log2f
    if mode == _abi.RESTRICT:
        _need(x, (n, n), "x")
        out_shape = (nl, nl)
    elif mode in (_abi.PROLONG, _abi.RESTRICT_ADJ):
        _need(x, (x.shape[0], x.shape[0]), "x")
        n = x.shape[0] << log2f
        out_shape = (n, n)
    else:
        _need(x, (n, n), "x")
        out_shape = (n, n)
    out = torch.empty(out_shape, dtype=torch.float32, device=x.device)
    lv = ctypes.byref(levels.c()) if levels is not None else None
    check(lib().imask_resample(n, log2f, mode, lv, _ptr(x), _ptr(out), _stream()), "imask_resample")
    return out


def sketch_apply(g: Geometry, levels: Levels, k: int, inp: torch.Tensor, adjoint: bool, work: torch.Tensor):
    """K_k inp (adjoint=False) or K_k^T inp (adjoint=True)."""
    if adjoint:
        _need(inp, g.sino_shape, "in")
        out = torch.empty(g.image_shape, dtype=torch.float32, device=inp.device)
    else:
        _need(inp, g.image_shape, "in")
        out = torch.empty(g.sino_shape, dtype=torch.float32, device=inp.device)
    check(lib().imask_sketch_apply(ctypes.byref(g.c()), ctypes.byref(levels.c()), k, int(adjoint), _ptr(work),
                                   _ptr(inp), _ptr(out), _stream()), "imask_sketch_apply")
    return out


def time_kernel(g: Geometry, which: int, log2f: int, inp: torch.Tensor, work: torch.Tensor, reps: int = 10) -> float:
    """Average launch duration (s) of one projector kernel, HIP events on the current stream."""
    if which == _abi.KERNEL_FORWARD:
        _need(inp, g.image_shape, "in")
        out = torch.empty(g.sino_shape, dtype=torch.float32, device=inp.device)
    else:
        _need(inp, g.sino_shape, "in")
        out = torch.empty(1, dtype=torch.float32, device=inp.device)
    ms = ctypes.c_double()
    check(lib().imask_time_kernel(ctypes.byref(g.c()), which, log2f, _ptr(work), _ptr(inp), _ptr(out), reps,
                                  _stream(), ctypes.byref(ms)), "imask_time_kernel")
    return ms.value / 1e3


def step_constants(g: Geometry, levels: Levels, mu: float, work: torch.Tensor, iters: int = 60, seed: int = 7):
    """(L^2, Lbar^2, Lbar_p^2) of Sec. 3.4 by power iterations on the GPU operators."""
    nbytes = lib().imask_constants_scratch_bytes(ctypes.byref(g.c()))
    if nbytes == 0:
        raise ImaskError("invalid geometry")
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=work.device)
    out = (ctypes.c_double * 3)()
    check(lib().imask_step_constants(ctypes.byref(g.c()), ctypes.byref(levels.c()), mu, iters, seed, _ptr(work),
                                     _ptr(scratch), out, _stream()), "imask_step_constants")
    return out[0], out[1], out[2]


def sigma_thm3(L2: float, Lbar2: float, Lbarp2: float, pmin: float, grid: int = 200):
    """(sigma, theta) from Thm. 3 minimised over a (c, rho) grid."""
    sig, th = ctypes.c_double(), ctypes.c_double()
    check(lib().imask_sigma_thm3(L2, Lbar2, Lbarp2, pmin, grid, ctypes.byref(sig), ctypes.byref(th)),
          "imask_sigma_thm3")
    return sig.value, th.value


def sigma_balamurugan(L2: float, Lbar2: float) -> float:
    """sigma_B = 1/(L^2 + 3 Lbar^2), the comparison step of Sec. 3.6."""
    out = ctypes.c_double()
    check(lib().imask_sigma_balamurugan(L2, Lbar2, ctypes.byref(out)), "imask_sigma_balamurugan")
    return out.value


def draws(params: Params, levels: Levels, k0: int, count: int) -> np.ndarray:
    out = (ctypes.c_int32 * max(count, 1))()
    check(lib().imask_draws(ctypes.byref(params.c()), ctypes.byref(levels.c()), k0, count, out), "imask_draws")
    return np.frombuffer(out, dtype=np.int32, count=count).copy()


def block_draws(params: Params, levels: Levels, k0: int, count: int) -> np.ndarray:
    """Measurement blocks of draws k0 .. k0+count-1 (all 0 without blocks)."""
    out = (ctypes.c_int32 * max(count, 1))()
    check(lib().imask_block_draws(ctypes.byref(params.c()), ctypes.byref(levels.c()), k0, count, out),
          "imask_block_draws")
    return np.frombuffer(out, dtype=np.int32, count=count).copy()


@dataclass
class Problem:
    """Device-resident ImaSk state for one reconstruction (Alg. 1 INPUT)."""
    geom: Geometry
    levels: Levels
    reg: Regularizer
    params: Params
    b: torch.Tensor
    device: str = "cuda"
    compact_tables: bool = False  # Remark 1: psi holds the average, ztab the snapshots
    x: list = field(default_factory=list)
    y: list = field(default_factory=list)
    phi: torch.Tensor | None = None
    psi: torch.Tensor | None = None
    work: torch.Tensor | None = None
    xbar: torch.Tensor | None = None  # extrapolated point (sequential schedule)
    tvd: list = field(default_factory=list)  # TV dual pair, two ping-pong buffers (REG_TV)
    ztab: torch.Tensor | None = None  # compact dual tables: restricted iterate snapshots
    k: int = 0
    epochs: float = 0.0
    cur: int = 0

    def __post_init__(self):
        g = self.geom
        _need(self.b, g.sino_shape, "b")
        dev = self.b.device
        nphi = lib().imask_phi_floats(ctypes.byref(g.c()), ctypes.byref(self.levels.c()))
        if nphi == 0:
            raise ImaskError("invalid geometry or level set")
        self.x = [torch.zeros(g.image_shape, device=dev) for _ in range(2)]
        self.y = [torch.zeros(g.sino_shape, device=dev) for _ in range(2)]
        self.phi = torch.zeros(nphi, device=dev)
        if self.compact_tables:
            self.psi = torch.zeros(g.sino_shape, device=dev)
            self.ztab = torch.zeros(nphi, device=dev)
        else:
            self.psi = torch.zeros((self.levels.r,) + g.sino_shape, device=dev)
        self.work = workspace(g, dev)
        if self.params.schedule == _abi.SCHEDULE_SEQUENTIAL:
            self.xbar = torch.zeros(g.image_shape, device=dev)
        if self.reg.kind == _abi.REG_TV:
            self.tvd = [torch.zeros((2,) + g.image_shape, device=dev) for _ in range(2)]

    # -- C struct round trip
    def _cstate(self) -> _abi.State:
        s = _abi.State()
        s.x[0], s.x[1] = self.x[0].data_ptr(), self.x[1].data_ptr()
        s.y[0], s.y[1] = self.y[0].data_ptr(), self.y[1].data_ptr()
        s.phi, s.psi, s.work = self.phi.data_ptr(), self.psi.data_ptr(), self.work.data_ptr()
        s.k, s.epochs, s.cur = self.k, self.epochs, self.cur
        s.xbar = self.xbar.data_ptr() if self.xbar is not None else None
        if self.tvd:
            s.tvd[0], s.tvd[1] = self.tvd[0].data_ptr(), self.tvd[1].data_ptr()
        s.ztab = self.ztab.data_ptr() if self.ztab is not None else None
        return s

    def _absorb(self, s: _abi.State) -> None:
        self.k, self.epochs, self.cur = int(s.k), float(s.epochs), int(s.cur)

    @property
    def x_cur(self) -> torch.Tensor:
        return self.x[self.cur]

    @property
    def y_cur(self) -> torch.Tensor:
        return self.y[self.cur]

    def step(self, n_steps: int = 1) -> None:
        s = self._cstate()
        bp = (ctypes.c_void_p * 1)(self.b.data_ptr())
        rc = lib().imask_step(1, ctypes.byref(self.geom.c()), ctypes.byref(self.levels.c()),
                              ctypes.byref(self.reg.c()), ctypes.byref(self.params.c()), bp,
                              ctypes.byref(s), n_steps, _stream())
        self._absorb(s)  # steps taken before an error (ENONFINITE) are kept
        check(rc, "imask_step")

    def step_timed(self, n_steps: int):
        """n_steps steps in one library call; returns each step's GPU time
        in ms (HIP events between the steps; a diagnostic)."""
        s = self._cstate()
        bp = (ctypes.c_void_p * 1)(self.b.data_ptr())
        ms = (ctypes.c_float * max(1, n_steps))()
        rc = lib().imask_step_timed(ctypes.byref(self.geom.c()), ctypes.byref(self.levels.c()),
                                    ctypes.byref(self.reg.c()), ctypes.byref(self.params.c()), bp[0],
                                    ctypes.byref(s), n_steps, ms, _stream())
        self._absorb(s)
        check(rc, "imask_step_timed")
        return [float(ms[i]) for i in range(n_steps)]

    def solve(self, budget: float, kind: int = _abi.BUDGET_ITERS) -> None:
        s = self._cstate()
        bp = (ctypes.c_void_p * 1)(self.b.data_ptr())
        rc = lib().imask_solve(1, ctypes.byref(self.geom.c()), ctypes.byref(self.levels.c()),
                               ctypes.byref(self.reg.c()), ctypes.byref(self.params.c()), bp,
                               ctypes.byref(s), float(budget), kind, _stream())
        self._absorb(s)
        check(rc, "imask_solve")

    def phi_tables(self, block: int = 0):
        """The table as a list of images: sketch 0 full size, k > 0 coarse
        (with measurement blocks, the tables of one block)."""
        per = sum((self.geom.n >> l) ** 2 for l in self.levels.log2f)
        out, off = [], block * per
        for l in self.levels.log2f:
            nl = self.geom.n >> l
            out.append(self.phi[off:off + nl * nl].view(nl, nl))
            off += nl * nl
        return out

    def state_dict(self) -> dict:
        d = {"x": self.x_cur.clone(), "y": self.y_cur.clone(), "phi": self.phi.clone(),
             "psi": self.psi.clone(), "k": self.k, "epochs": self.epochs}
        if self.xbar is not None:
            d["xbar"] = self.xbar.clone()
        if self.tvd:
            d["tvd"] = self.tvd[self.cur].clone()
        if self.ztab is not None:
            d["ztab"] = self.ztab.clone()
        return d

    def load_state_dict(self, d: dict) -> None:
        self.cur = 0
        self.x[0].copy_(d["x"])
        self.y[0].copy_(d["y"])
        self.phi.copy_(d["phi"])
        self.psi.copy_(d["psi"])
        if self.xbar is not None:
            self.xbar.copy_(d["xbar"])
        if self.tvd:
            self.tvd[0].copy_(d["tvd"])
        if self.ztab is not None:
            self.ztab.copy_(d["ztab"])
        self.k, self.epochs = int(d["k"]), float(d["epochs"])


def step_many(problems: list, n_steps: int = 1) -> None:
    """One imask_step call advancing several independent problems."""
    n = len(problems)
    if n == 0:
        return
    G = (_abi.Geometry * n)(*[p.geom.c() for p in problems])
    L = (_abi.Levels * n)(*[p.levels.c() for p in problems])
    R = (_abi.Reg * n)(*[p.reg.c() for p in problems])
    P = (_abi.Params * n)(*[p.params.c() for p in problems])
    B = (ctypes.c_void_p * n)(*[p.b.data_ptr() for p in problems])
    S = (_abi.State * n)(*[p._cstate() for p in problems])
    rc = lib().imask_step(n, G, L, R, P, B, S, n_steps, _stream())
    for p, s in zip(problems, S):
        p._absorb(s)
    check(rc, "imask_step")
