"""Writes paper_vortex_errors_oracle.json: the FP64 oracle's density errors
against the exact isentropic vortex of the paper's own test (Sec. 4.1,
Tables 1-2: epsilon = 1, U = rho = 1, Mach 0.3 with p = 1 / (gamma M^2),
mean flow at arctan(1/2), inner disk r < 2 rotating at omega = 1, errors at
t = 2 when the vortex centre reaches the sliding interface) on the vortex
mesh family at refinements f = 1, 2, 3 (384, 1,536 and 3,456 cells),
SSP-RK3 with dt = dt0 / f.  Calls only oracle/ (and the input generators
in workloads/); the levels run in parallel processes.

    python tests/golden/make_paper_vortex_errors.py      # about 40 minutes
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

T = 2.0
# (N, dt0, levels): stable steps with margin (CFL about 0.1 per point spacing)
RUNS = [(3, 0.004, (1, 2, 3)), (4, 0.0016, (1, 2, 3))]


def errors(args):
    N, f, dt0 = args
    from threadpoolctl import threadpool_limits

    from oracle.exact import vortex_state
    from oracle.ssd import SSD
    from workloads import cases as C
    from workloads import meshes as M
    case = C.paper_vortex_case()
    s = SSD(M.vortex_mesh(f), case, N)
    x, y = s.sp_coords(0.0)
    Q = vortex_state(x, y, 0.0, case)
    n = int(round(T / (dt0 / f)))
    with threadpool_limits(1):
        Q = s.run(Q, 0.0, T / n, n)
    xT, yT = s.sp_coords(s.theta(T))
    e = Q[0] - vortex_state(xT, yT, T, case)[0]
    w = s.ops.w
    W = (w[:, None] * w[None, :])[:, :, None] * np.moveaxis(s.geo.detJ, 0, 2)
    l1 = float((W * np.abs(e)).sum() / W.sum())
    l2 = float(np.sqrt((W * e * e).sum() / W.sum()))
    print(f"N={N} f={f} cells={s.E}: L1 {l1:.6e} L2 {l2:.6e}", flush=True)
    return {"N": N, "f": f, "cells": int(s.E), "dt0": dt0, "steps": n, "L1": l1, "L2": l2}


def main():
    jobs = [(N, f, dt0) for N, dt0, levels in RUNS for f in levels]
    jobs.sort(key=lambda j: -(j[1] ** 3) * j[0])      # longest first
    with Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        runs = pool.map(errors, jobs, chunksize=1)
    runs.sort(key=lambda r: (r["N"], r["f"]))
    out = {"_source": "FP64 oracle (oracle/ssd.py), density error against the exact vortex of "
                      "Sec. 4.1 (epsilon 1, Mach 0.3, mean flow at arctan(1/2), omega 1), "
                      "SSP-RK3 to t = 2, dt = dt0 / f on vortex_mesh(f)",
           "T": T, "runs": runs}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                           "paper_vortex_errors_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
