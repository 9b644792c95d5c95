"""Writes tests/golden/vortex_N9_16x16_t10_oracle_rho.npy: the FP64 oracle's nodal density of the
isentropic vortex (Sec. 5; N = 9, 16 x 16 cells on the periodic [0,10]^2, Rusanov flux, limiter on,
initial data by nodal interpolation, CFL time steps of the oracle's rule with the workload's factor,
the last one shortened to land on t = 10), read by the GPU test of the end-to-end L1 error.

Calls only the oracle (oracle/) and the initial-data module.  About 15 minutes on 8 threads:

    python tests/golden/make_vortex_oracle_t10.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O                     # noqa: E402
from paper_1406_7416_amd import workloads as W     # noqa: E402

T_END = 10.0


def main():
    wl = W.vortex(16, 9)
    o = O.Oracle(wl)
    u0, _ = o.project(wl.ic, 0)
    o.set_state(u0)
    steps = 0
    while o.time < T_END * (1 - 1e-14):
        o.step(min(o.cfl_dt(), T_END - o.time))
        steps += 1
    rho = o.state()[0]
    np.save(os.path.join(HERE, "vortex_N9_16x16_t10_oracle_rho.npy"), rho)
    print(f"{steps} steps, t = {o.time}")


if __name__ == "__main__":
    main()
