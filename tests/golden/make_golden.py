"""Writes the stored expected values under tests/golden/ using only the
oracle (oracle/) and the seeded input module (synth/).

  cfg1_sigma.json  step size for the 64x64 parity workload (90 angles,
                   92 bins, levels 64/32/16 with p = 1/3, Tikhonov
                   lambda = 1e-2): the normalised constants L^2, Lbar^2,
                   Lbar_p^2 by the power method on the oracle's sketches
                   (both full-resolution modes) and sigma from Thm. 3
                   (Sec. 3.6) minimised over a (c, rho) grid.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import steps  # noqa: E402


def cfg1_sigma():
    g = oracle.Geometry(64, 90, 92)
    out = {"workload": "64x64, 90 angles, 92 bins, levels (0,1,2), p=1/3, Tikhonov lambda=1e-2"}
    for mode, name in ((oracle.MODE_PAPER, "paper"), (oracle.MODE_UNBIASED, "unbiased")):
        lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, mode)
        L2, lb, lp = steps.constants_power(lambda k, x: oracle.sketch_fwd(g, lv, k, x),
                                           lambda k, y: oracle.sketch_adj(g, lv, k, y),
                                           lv.p, 1e-2, (64, 64), (90, 92), iters=300)
        sigma, theta, c, rho = steps.sigma_thm3(L2, lb, lp, min(lv.p), 200, 200)
        out[name] = {"L2": L2, "Lbar2": lb, "Lbarp2": lp, "sigma": sigma, "theta": theta, "c": c, "rho": rho,
                     "sigma_B": steps.sigma_balamurugan(L2, lb)}
    return out


if __name__ == "__main__":
    res = cfg1_sigma()
    with open(os.path.join(HERE, "cfg1_sigma.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))
