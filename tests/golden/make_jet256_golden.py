"""Writes tests/golden/jet256_fp64_500steps.txt from the CPU oracle alone.

Workload: the synthetic M = 1.4 jet on the 256 x 128 x 128 curvilinear grid, FP64,
seed 0, boundary conditions applied to the initial field, then 500 five-stage Runge-Kutta
steps at CFL 0.5 (paper, Time Marching Method; Boundary Conditions). Stored:

* ke: the volume-weighted kinetic energy after every step (500 values);
* the running statistics of (rho, u, v, w, p) sampled every 10 steps (50 samples), reduced
  over the azimuth (the statistics the paper's Numerical Results could not converge):
  centreline mean and r.m.s. axial velocity at every axial station, and radial profiles of
  the mean and r.m.s. axial velocity and the mean density and pressure at stations
  i = 16, 64, 128, 192, 240.

Every value is written with 17 significant digits. Nothing here calls the GPU library.

    python tests/golden/make_jet256_golden.py        (about 15-30 minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic as sy  # noqa: E402
from oracle.stats import RunningStats, jet_products  # noqa: E402

GRID = (256, 128, 128)
STEPS = 500
EVERY = 10
STATIONS = (16, 64, 128, 192, 240)
OUT = os.path.join(HERE, "jet256_fp64_500steps.txt")


def main():
    p, xyz, q = sy.make_case("jet", GRID, seed=0)
    o = oracle.Oracle(p, xyz)
    x = o.apply_bc(q)
    st = RunningStats(p.shape, p.gamma)
    ke = []
    t0 = time.perf_counter()
    for n in range(1, STEPS + 1):
        x, _ = o.step(x, 1, cfl=0.5)
        ke.append(o.diagnostics(x)[0])
        if n % EVERY == 0:
            st.add(x)
            print(f"step {n} ke {ke[-1]:.17g} elapsed {time.perf_counter() - t0:.0f} s",
                  flush=True)
    mean, rms = st.mean_rms()
    prod = jet_products(mean, rms, STATIONS)
    with open(OUT + ".tmp", "w") as f:
        f.write("# Jet 256x128x128 FP64, seed 0, CFL 0.5, 500 Runge-Kutta steps, written by the\n")
        f.write("# CPU oracle (tests/golden/make_jet256_golden.py). Paper: Time Marching Method,\n")
        f.write("# Boundary Conditions; statistics as the Numerical Results section needs them.\n")
        f.write(f"# samples every {EVERY} steps: {st.n}\n")
        f.write("ke " + " ".join(f"{v:.17g}" for v in ke) + "\n")
        for name, arr in prod.items():
            f.write(name + " " + " ".join(f"{v:.17g}" for v in np.asarray(arr)) + "\n")
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
