"""Helpers shared by the GPU tests (device transfer, relative errors)."""
import json
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def f32(a) -> np.ndarray:
    """The float32-rounded input, as float64, so both sides see the same values."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def golden(name: str) -> dict:
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def say(msg: str) -> None:
    print(msg, flush=True)


U32 = 2.0 ** -24  # unit roundoff of float32


def elementwise_ok(got, exp, absref, n_terms: int, floor: float = 1e-6):
    """Element-by-element rounding bound for a projector output.

    Each output element is an FP32 sum of at most n_terms products whose
    absolute values add up to absref (the operator applied to the absolute
    input: every Joseph weight is nonnegative).  The classical bound of an
    n-term floating-point sum, gamma_n = n u / (1 - n u) times that sum,
    covers the accumulation in any order; `floor` times max(absref) covers
    the fixed-point coordinate (weights within 1e-6 of FP64's) and the FP32
    inputs.  Returns (ok, worst ratio of |got - exp| to the bound)."""
    got = np.asarray(got, dtype=np.float64)
    exp = np.asarray(exp, dtype=np.float64)
    absref = np.asarray(absref, dtype=np.float64)
    nu = n_terms * U32
    bound = nu / (1.0 - nu) * absref + floor * float(absref.max())
    worst = float(np.max(np.abs(got - exp) / np.maximum(bound, 1e-300)))
    return worst <= 1.0, worst


def max_rel(got, exp) -> float:
    """max |got - exp| / max |exp|: the element-by-element companion of rel()."""
    got = np.asarray(got, dtype=np.float64)
    exp = np.asarray(exp, dtype=np.float64)
    return float(np.max(np.abs(got - exp)) / max(float(np.max(np.abs(exp))), 1e-300))
