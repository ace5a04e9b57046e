"""Write the FP64 oracle's density after 10 Strang steps of the 32^3 x 32^3
workload (seeded initial condition, drifting 4-mode potential), the reference
for the FP16/BF16 storage error at the precision form's stated size.

Calls only the oracle and the seeded input generators:
    python tests/golden/make_density_32x32.py      (about 10-20 min on 8 cores)
Writes tests/golden/density_32x32_10steps.npz: rho (FP64 [32,32,32]), mass
(in-domain, FP64) and outflow (total tallied outflow, FP64).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2110_15867_amd import inputs  # noqa: E402

STEPS = 10


def main():
    w = inputs.workload(2)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    f = inputs.initial_f32(w).astype(np.float64)   # the FP32 initial condition both sides start from
    pot = inputs.potential(w)
    outflow = np.zeros(int(np.prod(w.n)))
    t0 = time.time()
    for n in range(STEPS):
        gn = inputs.accel_field(w, pot, n * w.dt)
        gnp1 = inputs.accel_field(w, pot, (n + 1) * w.dt)
        f = oracle.step(og, f, gn, gnp1, w.dt, outflow=outflow)
        print(f"step {n + 1}/{STEPS} done, {time.time() - t0:.0f} s", flush=True)
    rho, _, mass = oracle.moments(og, f)
    np.savez(os.path.join(HERE, "density_32x32_10steps.npz"), rho=rho, mass=np.float64(mass),
             outflow=np.float64(outflow.sum()))
    print("mass", mass, "outflow", outflow.sum())


if __name__ == "__main__":
    main()
