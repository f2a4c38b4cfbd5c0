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
