"""ctypes shim over ``liborc.so`` (built from ``imask_oracle.c``).

Every function takes and returns float64 numpy arrays shaped like the paper's
objects: images are (N_l, N_l), sinograms are (n_angles, n_det).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "imask_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

MODE_PAPER = 0
MODE_UNBIASED = 1
REG_TIKHONOV = 0
REG_SMOOTH_TV = 1
REG_TV = 2

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U64 = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        geo = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
               ctypes.c_double, ctypes.c_double]
        L.orc_project.argtypes = geo + [ctypes.c_int, _D, _D]
        L.orc_backproject.argtypes = geo + [ctypes.c_int, _D, _D]
        L.orc_count_samples.argtypes = geo + [ctypes.c_int]
        L.orc_count_samples.restype = ctypes.c_longlong
        L.orc_restrict.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_prolong.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_compensate.argtypes = [ctypes.c_int, ctypes.c_int, _I32, _D, _D, _D]
        sk = geo + [ctypes.c_int, _I32, _D, ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_sketch_fwd.argtypes = sk
        L.orc_sketch_adj.argtypes = sk
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_thresholds.argtypes = [ctypes.c_int, _D, _U64]
        L.orc_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                ctypes.c_int, _D, _I32]
        L.orc_tv_value.argtypes = [ctypes.c_int, _D, ctypes.c_double]
        L.orc_tv_value.restype = ctypes.c_double
        L.orc_tv_gradient.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D]
        L.orc_tv_fgp.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_int, _D, _D, _D]
        L.orc_tv_fgp.restype = None
        L.orc_tv_prox.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, _D]
        L.orc_imask_run.argtypes = geo + [ctypes.c_int, _I32, _D, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint64, _D, ctypes.c_int,
                                          _D, _D, _D, _D, _D, _I32, _D]
        L.orc_imask_run.restype = ctypes.c_int
        L.orc_imask_seq_run.argtypes = geo + [ctypes.c_int, _I32, _D, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                              ctypes.c_uint64, _D, ctypes.c_int,
                                              _D, _D, _D, _D, _D, _D, _I32, _D]
        L.orc_imask_seq_run.restype = ctypes.c_int
        L.orc_imask_compact_run.argtypes = geo + [ctypes.c_int, _I32, _D, ctypes.c_int,
                                                  ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_double, ctypes.c_int,
                                                  ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                                  ctypes.c_uint64, _D, ctypes.c_int,
                                                  _D, _D, _D, _D, _D, _D, _I32, _D]
        L.orc_imask_compact_run.restype = ctypes.c_int
        L.orc_imask_indep_run.argtypes = geo + [ctypes.c_int, _I32, _D, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_int,
                                                ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                                ctypes.c_uint64, _D, ctypes.c_int,
                                                _D, _D, _D, _D, _D, _I32, _I32, _D]
        L.orc_imask_indep_run.restype = ctypes.c_int
        L.orc_block_rows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32, _I32]
        L.orc_block_rows.restype = None
        L.orc_block_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                      ctypes.c_int, _I32]
        L.orc_block_draws.restype = None
        L.orc_imask_blocks_run.argtypes = geo + [ctypes.c_int, _I32, _D, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_int,
                                                 ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                                 ctypes.c_uint64, _D, ctypes.c_int,
                                                 _D, _D, _D, _D, _D, _I32, _I32, _D]
        L.orc_imask_blocks_run.restype = ctypes.c_int
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass(frozen=True)
class Geometry:
    """2-D CT geometry: N x N image on [-E,E]^2 (E = extent), n_det bins of
    spacing ds centred at s0.

    Parallel beam (src_dist = 0): n_angles angles a*pi/n_angles or the given
    list (radians); default spacing the full-res pixel size 2E/N.
    Fan beam (src_dist = D > 0): n_angles source positions at angle
    2 pi a/n_angles (or the list), distance D from the centre, and a flat
    detector at distance det_dist beyond the centre; default spacing the
    pixel size magnified onto the detector, 2E/N (D + det_dist)/D."""
    n: int
    n_angles: int
    n_det: int
    ds: float = 0.0
    s0: float = 0.0
    extent: float = 1.0
    angles: tuple = None
    src_dist: float = 0.0
    det_dist: float = 0.0

    def __post_init__(self):
        if self.angles is not None:
            a = tuple(float(t) for t in self.angles)
            assert len(a) == self.n_angles
            object.__setattr__(self, "angles", a)
            object.__setattr__(self, "_ang", _f64(a))

    @property
    def fan(self) -> bool:
        return self.src_dist > 0

    @property
    def spacing(self) -> float:
        if self.ds > 0:
            return self.ds
        h = 2.0 * self.extent / self.n
        return h * (self.src_dist + self.det_dist) / self.src_dist if self.fan else h

    def theta(self) -> np.ndarray:
        if self.angles is not None:
            return np.array(self.angles)
        return np.arange(self.n_angles) * np.pi / self.n_angles

    def args(self):
        ang = _dp(self._ang) if self.angles is not None else None
        return (self.n, self.n_angles, self.n_det, self.spacing, self.s0, self.extent, ang, self.src_dist,
                self.det_dist)


@dataclass
class Levels:
    """Resolution set: log2 downsampling factors (first one 0) and the
    sampling probabilities p of each sketch."""
    log2f: list
    p: list
    mode: int = MODE_PAPER

    @property
    def r(self) -> int:
        return len(self.log2f)

    def carrays(self):
        lf = np.ascontiguousarray(self.log2f, dtype=np.int32)
        pp = _f64(self.p)
        return lf, pp


def project(g: Geometry, lvl: int, z) -> np.ndarray:
    z = _f64(z)
    assert z.shape == (g.n >> lvl, g.n >> lvl)
    out = np.empty((g.n_angles, g.n_det))
    lib().orc_project(*g.args(), lvl, _dp(z), _dp(out))
    return out


def backproject(g: Geometry, lvl: int, sino) -> np.ndarray:
    s = _f64(sino)
    assert s.shape == (g.n_angles, g.n_det)
    nl = g.n >> lvl
    out = np.empty((nl, nl))
    lib().orc_backproject(*g.args(), lvl, _dp(s), _dp(out))
    return out


def count_samples(g: Geometry, lvl: int) -> int:
    return int(lib().orc_count_samples(*g.args(), lvl))


def restrict(x, lvl: int) -> np.ndarray:
    x = _f64(x)
    n = x.shape[0]
    out = np.empty((n >> lvl, n >> lvl))
    lib().orc_restrict(n, lvl, _dp(x), _dp(out))
    return out


def prolong(z, lvl: int) -> np.ndarray:
    z = _f64(z)
    n = z.shape[0] << lvl
    out = np.empty((n, n))
    lib().orc_prolong(n, lvl, _dp(z), _dp(out))
    return out


def compensate(x, lv: Levels) -> np.ndarray:
    x = _f64(x)
    lf, pp = lv.carrays()
    out = np.empty_like(x)
    lib().orc_compensate(x.shape[0], lv.r, lf.ctypes.data_as(_I32), _dp(pp), _dp(x), _dp(out))
    return out


def sketch_fwd(g: Geometry, lv: Levels, k: int, x) -> np.ndarray:
    x = _f64(x)
    lf, pp = lv.carrays()
    out = np.empty((g.n_angles, g.n_det))
    lib().orc_sketch_fwd(*g.args(), lv.r, lf.ctypes.data_as(_I32), _dp(pp), lv.mode, k,
                         _dp(x), _dp(out))
    return out


def sketch_adj(g: Geometry, lv: Levels, k: int, y) -> np.ndarray:
    y = _f64(y)
    lf, pp = lv.carrays()
    out = np.empty((g.n, g.n))
    lib().orc_sketch_adj(*g.args(), lv.r, lf.ctypes.data_as(_I32), _dp(pp), lv.mode, k,
                         _dp(y), _dp(out))
    return out


def splitmix64(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64(seed, k))


def thresholds(p) -> np.ndarray:
    pp = _f64(p)
    out = np.empty(len(pp), dtype=np.uint64)
    lib().orc_thresholds(len(pp), _dp(pp), out.ctypes.data_as(_U64))
    return out


def draws(seed: int, stream: int, k0: int, count: int, p) -> np.ndarray:
    pp = _f64(p)
    out = np.empty(count, dtype=np.int32)
    lib().orc_draws(seed, stream, k0, count, len(pp), _dp(pp), out.ctypes.data_as(_I32))
    return out


def tv_value(u, eps: float) -> float:
    u = _f64(u)
    return float(lib().orc_tv_value(u.shape[0], _dp(u), eps))


def tv_gradient(u, eps: float) -> np.ndarray:
    u = _f64(u)
    out = np.empty_like(u)
    lib().orc_tv_gradient(u.shape[0], _dp(u), eps, _dp(out))
    return out


def tv_prox(v, u0, tau: float, lam: float, w: float, eps: float, J: int) -> np.ndarray:
    v, u0 = _f64(v), _f64(u0)
    out = np.empty_like(v)
    lib().orc_tv_prox(v.shape[0], _dp(v), _dp(u0), tau, lam, w, eps, J, _dp(out))
    return out


def tv_fgp(b, gamma: float, J: int, p=None):
    """prox of gamma TV + nonnegativity at b by J dual fast gradient
    projection steps from the dual pair p (2, N, N; zeros if None).
    Returns (u, p_after)."""
    b = _f64(b)
    n = b.shape[0]
    pp = np.zeros((2, n, n)) if p is None else np.array(p, dtype=np.float64, copy=True)
    u = np.empty_like(b)
    lib().orc_tv_fgp(n, _dp(b), gamma, J, _dp(pp[0]), _dp(pp[1]), _dp(u))
    return u, pp


@dataclass
class Reg:
    """Regulariser: TIKHONOV R = lam/2 |x|^2; SMOOTH_TV
    R = w TV_eps + lam/2 |x|^2 with J FISTA iterations; TV (the paper's
    prior) R = w TV + chi_{>=0} + lam/2 |x|^2 with J dual FGP iterations
    warm-started at the state's dual pair; mu = lam."""
    kind: int = REG_TIKHONOV
    lam: float = 1e-2
    tv_weight: float = 0.0
    tv_eps: float = 1e-3
    tv_inner: int = 10


@dataclass
class State:
    x: np.ndarray
    y: np.ndarray
    phi: np.ndarray  # (r, N, N)
    psi: np.ndarray  # (r, n_angles, n_det)
    k: int = 0
    epochs: float = 0.0
    draws: list = field(default_factory=list)
    xbar: np.ndarray | None = None  # extrapolated point (ImaSk-Seq only)
    tvd: np.ndarray | None = None   # TV dual pair (2, N, N) of REG_TV's prox
    dual_draws: list = field(default_factory=list)  # dual indices (independent draws only)

    @staticmethod
    def zeros(g: Geometry, lv: Levels) -> "State":
        return State(np.zeros((g.n, g.n)), np.zeros((g.n_angles, g.n_det)),
                     np.zeros((lv.r, g.n, g.n)), np.zeros((lv.r, g.n_angles, g.n_det)),
                     xbar=np.zeros((g.n, g.n)), tvd=np.zeros((2, g.n, g.n)))

    def copy(self) -> "State":
        return State(self.x.copy(), self.y.copy(), self.phi.copy(), self.psi.copy(),
                     self.k, self.epochs, list(self.draws),
                     None if self.xbar is None else self.xbar.copy(),
                     None if self.tvd is None else self.tvd.copy(), list(self.dual_draws))

    def ensure(self, g: Geometry) -> None:
        if self.xbar is None:
            self.xbar = self.x.copy()
        if self.tvd is None:
            self.tvd = np.zeros((2, g.n, g.n))


def imask_run(g: Geometry, lv: Levels, reg: Reg, sigma: float, seed: int, stream: int,
              b, n_iter: int, state: State | None = None) -> State:
    """Alg. 1 (ImaSk) for n_iter iterations from `state` (zeros if None)."""
    st = State.zeros(g, lv) if state is None else state.copy()
    st.ensure(g)
    b = _f64(b)
    lf, pp = lv.carrays()
    dr = np.empty(max(n_iter, 1), dtype=np.int32)
    ep = np.array([st.epochs])
    rc = lib().orc_imask_run(*g.args(), lv.r, lf.ctypes.data_as(_I32), _dp(pp), lv.mode,
                             reg.kind, reg.lam, reg.tv_weight, reg.tv_eps, reg.tv_inner,
                             sigma, seed, stream, st.k, _dp(b), n_iter,
                             _dp(st.x), _dp(st.y), _dp(st.phi), _dp(st.psi), _dp(st.tvd),
                             dr.ctypes.data_as(_I32), _dp(ep))
    if rc != 0:
        raise ValueError("oracle rejected the level set")
    st.k += n_iter
    st.epochs = float(ep[0])
    st.draws.extend(int(v) for v in dr[:n_iter])
    return st


def block_rows(n_angles: int, n_blocks: int, j: int) -> tuple:
    """Angles [a0, a1) of measurement block j (contiguous blocks)."""
    a0, a1 = ctypes.c_int32(), ctypes.c_int32()
    lib().orc_block_rows(n_angles, n_blocks, j, ctypes.byref(a0), ctypes.byref(a1))
    return a0.value, a1.value


def block_draws(seed: int, stream: int, k0: int, count: int, n_blocks: int) -> list:
    out = np.empty(max(count, 1), dtype=np.int32)
    lib().orc_block_draws(seed, stream, k0, count, n_blocks, out.ctypes.data_as(_I32))
    return [int(v) for v in out[:count]]


@dataclass
class BlocksState(State):
    """State of Alg. 1 over image sketches x measurement blocks: phi has one
    full image per (sketch i, block j) pair, index i * n_blocks + j."""
    blocks: list = field(default_factory=list)

    @staticmethod
    def zeros(g: Geometry, lv: Levels, n_blocks: int = 1) -> "BlocksState":
        return BlocksState(np.zeros((g.n, g.n)), np.zeros((g.n_angles, g.n_det)),
                           np.zeros((lv.r * n_blocks, g.n, g.n)), np.zeros((lv.r, g.n_angles, g.n_det)),
                           xbar=np.zeros((g.n, g.n)), tvd=np.zeros((2, g.n, g.n)))

    def copy(self) -> "BlocksState":
        c = BlocksState(self.x.copy(), self.y.copy(), self.phi.copy(), self.psi.copy(), self.k, self.epochs,
                        list(self.draws), None if self.xbar is None else self.xbar.copy(),
                        None if self.tvd is None else self.tvd.copy())
        c.blocks = list(self.blocks)
        return c


def imask_blocks_run(g: Geometry, lv: Levels, reg: Reg, sigma: float, seed: int, stream: int, n_blocks: int,
                     b, n_iter: int, state: BlocksState | None = None) -> BlocksState:
    """Alg. 1 over the product sketches K_ij = S E_j K_i (S = n_blocks
    contiguous angle blocks, uniform block draws), n_iter iterations."""
    st = BlocksState.zeros(g, lv, n_blocks) if state is None else state.copy()
    st.ensure(g)
    b = _f64(b)
    lf, pp = lv.carrays()
    dr = np.empty(max(n_iter, 1), dtype=np.int32)
    bl = np.empty(max(n_iter, 1), dtype=np.int32)
    ep = np.array([st.epochs])
    rc = lib().orc_imask_blocks_run(*g.args(), lv.r, lf.ctypes.data_as(_I32), _dp(pp), lv.mode, n_blocks,
                                    reg.kind, reg.lam, reg.tv_weight, reg.tv_eps, reg.tv_inner,
                                    sigma, seed, stream, st.k, _dp(b), n_iter,
                                    _dp(st.x), _dp(st.y), _dp(st.phi), _dp(st.psi), _dp(st.tvd),
                                    dr.ctypes.data_as(_I32), bl.ctypes.data_as(_I32), _dp(ep))
    if rc != 0:
        raise ValueError("oracle rejected the level set or block count")
    st.k += n_iter
    st.epochs = float(ep[0])
    st.draws.extend(int(v) for v in dr[:n_iter])
    st.blocks.extend(int(v) for v in bl[:n_iter])
    return st


def imask_seq_run(g: Geometry, lv: Levels, reg: Reg, sigma: float, theta: float, seed: int, stream: int,
                  b, n_iter: int, state: State | None = None) -> State:
    """ImaSk-Seq (Sec. 5) for n_iter iterations from `state` (zeros if None)."""
    st = State.zeros(g, lv) if state is None else state.copy()
    st.ensure(g)
    b = _f64(b)
    lf, pp = lv.carrays()
    dr = np.empty(max(n_iter, 1), dtype=np.int32)
    ep = np.array([st.epochs])
    rc = lib().orc_imask_seq_run(*g.args(), lv.r, lf.ctypes.data_as(_I32), _dp(pp), lv.mode,
                                 reg.kind, reg.lam, reg.tv_weight, reg.tv_eps, reg.tv_inner,
                                 sigma, theta, seed, stream, st.k, _dp(b), n_iter,
                                 _dp(st.x), _dp(st.xbar), _dp(st.y), _dp(st.phi), _dp(st.psi), _dp(st.tvd),
                                 dr.ctypes.data_as(_I32), _dp(ep))
    if rc != 0:
        raise ValueError("oracle rejected the level set")
    st.k += n_iter
    st.epochs = float(ep[0])
    st.draws.extend(int(v) for v in dr[:n_iter])
    return st


def imask_indep_run(g: Geometry, lv: Levels, reg: Reg, sigma: float, seed: int, stream: int, dual_stream: int,
                    b, n_iter: int, state: State | None = None) -> State:
    """Alg. 1 with independent primal (stream) and dual (dual_stream) draws;
    state.draws gets the primal indices, state.dual_draws the dual ones."""
    st = State.zeros(g, lv) if state is None else state.copy()
    st.ensure(g)
    b = _f64(b)
    lf, pp = lv.carrays()
    dr = np.empty(max(n_iter, 1), dtype=np.int32)
    dd = np.empty(max(n_iter, 1), dtype=np.int32)
    ep = np.array([st.epochs])
    rc = lib().orc_imask_indep_run(*g.args(), lv.r, lf.ctypes.data_as(_I32), _dp(pp), lv.mode,
                                   reg.kind, reg.lam, reg.tv_weight, reg.tv_eps, reg.tv_inner,
                                   sigma, seed, stream, dual_stream, st.k, _dp(b), n_iter,
                                   _dp(st.x), _dp(st.y), _dp(st.phi), _dp(st.psi), _dp(st.tvd),
                                   dr.ctypes.data_as(_I32), dd.ctypes.data_as(_I32), _dp(ep))
    if rc != 0:
        raise ValueError("oracle rejected the level set")
    st.k += n_iter
    st.epochs = float(ep[0])
    st.draws.extend(int(v) for v in dr[:n_iter])
    st.dual_draws.extend(int(v) for v in dd[:n_iter])
    return st


@dataclass
class CompactState:
    """State of Alg. 1 with Remark 1's compact dual tables: z (r, N, N) holds
    the iterate at each sketch's last refresh, psibar the table average."""
    x: np.ndarray
    y: np.ndarray
    phi: np.ndarray
    z: np.ndarray
    psibar: np.ndarray
    tvd: np.ndarray
    k: int = 0
    epochs: float = 0.0
    draws: list = field(default_factory=list)

    @staticmethod
    def zeros(g: Geometry, lv: Levels) -> "CompactState":
        return CompactState(np.zeros((g.n, g.n)), np.zeros((g.n_angles, g.n_det)), np.zeros((lv.r, g.n, g.n)),
                            np.zeros((lv.r, g.n, g.n)), np.zeros((g.n_angles, g.n_det)), np.zeros((2, g.n, g.n)))

    def copy(self) -> "CompactState":
        return CompactState(self.x.copy(), self.y.copy(), self.phi.copy(), self.z.copy(), self.psibar.copy(),
                            self.tvd.copy(), self.k, self.epochs, list(self.draws))


def imask_compact_run(g: Geometry, lv: Levels, reg: Reg, sigma: float, seed: int, stream: int,
                      b, n_iter: int, state: CompactState | None = None) -> CompactState:
    """Alg. 1 with Remark 1's compact dual tables for n_iter iterations."""
    st = CompactState.zeros(g, lv) if state is None else state.copy()
    b = _f64(b)
    lf, pp = lv.carrays()
    dr = np.empty(max(n_iter, 1), dtype=np.int32)
    ep = np.array([st.epochs])
    rc = lib().orc_imask_compact_run(*g.args(), lv.r, lf.ctypes.data_as(_I32), _dp(pp), lv.mode,
                                     reg.kind, reg.lam, reg.tv_weight, reg.tv_eps, reg.tv_inner,
                                     sigma, seed, stream, st.k, _dp(b), n_iter,
                                     _dp(st.x), _dp(st.y), _dp(st.phi), _dp(st.z), _dp(st.psibar), _dp(st.tvd),
                                     dr.ctypes.data_as(_I32), _dp(ep))
    if rc != 0:
        raise ValueError("oracle rejected the level set")
    st.k += n_iter
    st.epochs = float(ep[0])
    st.draws.extend(int(v) for v in dr[:n_iter])
    return st


def dense_matrix(fwd, n_in_shape, n_out: int) -> np.ndarray:
    """Explicit matrix of a linear map by applying it to unit vectors."""
    n_in = int(np.prod(n_in_shape))
    A = np.empty((n_out, n_in))
    e = np.zeros(n_in)
    for q in range(n_in):
        e[q] = 1.0
        A[:, q] = np.ravel(fwd(e.reshape(n_in_shape)))
        e[q] = 0.0
    return A
