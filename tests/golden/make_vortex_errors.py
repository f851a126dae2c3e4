"""Writes vortex_errors_oracle.json: the FP64 oracle's density errors
against the exact isentropic vortex (Sec. 4.1) on the refinement levels the
GPU convergence test uses.  Calls only oracle/ (and the input generators in
workloads/).

    python tests/golden/make_vortex_errors.py      # a few minutes on one core
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.exact import vortex_state  # noqa: E402
from oracle.ssd import SSD  # noqa: E402
from workloads import cases as C  # noqa: E402
from workloads import meshes as M  # noqa: E402

# (N, dt0, levels): SSP-RK3 to T with step dt0 / f on vortex_mesh(f), omega = 1
T = 0.5
RUNS = [(3, 0.01, (1, 2, 4)), (4, 0.004, (1, 2))]


def errors(N, f, dt0):
    case = C.vortex_case(omega=1.0)
    s = SSD(M.vortex_mesh(f), case, N)
    x, y = s.sp_coords(0.0)
    Q = vortex_state(x, y, 0.0, case)
    n = int(round(T / (dt0 / f)))
    Q = s.run(Q, 0.0, T / n, n)
    xT, yT = s.sp_coords(s.theta(T))
    e = Q[0] - vortex_state(xT, yT, T, case)[0]
    w = s.ops.w
    W = (w[:, None] * w[None, :])[:, :, None] * np.moveaxis(s.geo.detJ, 0, 2)
    return float((W * np.abs(e)).sum() / W.sum()), float(np.sqrt((W * e * e).sum() / W.sum()))


def main():
    out = {"_source": "FP64 oracle (oracle/ssd.py), density error against the exact vortex, "
                      "SSP-RK3 to t = 0.5, dt = dt0 / f on vortex_mesh(f), omega = 1",
           "T": T, "runs": []}
    for N, dt0, levels in RUNS:
        for f in levels:
            l1, l2 = errors(N, f, dt0)
            print(f"N={N} f={f}: L1 {l1:.6e} L2 {l2:.6e}", flush=True)
            out["runs"].append({"N": N, "f": f, "dt0": dt0, "L1": l1, "L2": l2})
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                           "vortex_errors_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
