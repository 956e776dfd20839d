"""Seeded synthetic workloads of the benchmark and the parity tests.

Plain data only (grid shapes, particles per cell, temperatures, drifts, seeds
and box lists): no step of the method is computed here.  The workloads stand in
for the paper's test problems (Sect. 3: thermal plasma, counter-streaming
beams, Harris sheet; Sect. 5: scans in the number of superparticles per cell),
which used no public dataset.
"""
from __future__ import annotations

import numpy as np

# thermal pair plasma, small case that the oracle runs in seconds
THERMAL16 = dict(name="thermal pair plasma 16^3", dims=(16, 16, 16), ppc=8, theta=0.1, n_x=10.0,
                 dt=0.5, steps=100, seed=1)

# thermal pair plasma, the benchmark workload
THERMAL64 = dict(name="thermal pair plasma 64^3", dims=(64, 64, 64), ppc=64, theta=0.1, n_x=10.0,
                 dt=0.5, steps=2000, seed=2)

# two counter-streaming cold pair beams along x (filamentation)
FILAMENT = dict(name="counter-streaming pair beams 256x256x4", dims=(256, 256, 4), ppc_per_beam=32,
                gamma=3.0, theta=0.01, n_x=20.0, rho0=128.0, dt=0.5, steps=3000, seed=3)

# periodic double Harris sheet (B along y, gradient along x, drifts along z)
HARRIS = dict(name="double Harris sheet 512x256x4", dims=(512, 256, 4), ppc=64, mass_ratio=25.0,
              theta_e=1.0, gu_e=0.68, chi=1.0, n_x=15.0, rho0=128.0, background=0.1, dt=0.5,
              steps=2000, seed=4)

# scaled-down shapes of the same workloads, small enough for element-wise
# parity with the oracle over ten steps
BEAMS_SMALL = dict(name="counter-streaming pair beams 32x32x4", dims=(32, 32, 4), ppc_per_beam=4,
                   gamma=3.0, theta=0.01, n_x=20.0, rho0=16.0, dt=0.5, seed=3)
HARRIS_SMALL = dict(name="double Harris sheet 64x32x4", dims=(64, 32, 4), ppc=4, mass_ratio=25.0,
                    theta_e=1.0, gu_e=0.68, chi=1.0, n_x=4.0, rho0=8.0, background=0.1, dt=0.5, seed=4)
ENSEMBLE_SMALL = dict(name="ensemble of 6 thermal boxes", n_boxes=6, edge=(6, 14), ppc=(1, 8),
                      theta=(0.05, 1.0), n_x=10.0, dt=0.5, seed=6)

# ensemble of independent thermal boxes, log-uniform sizes and densities
ENSEMBLE = dict(name="ensemble of 256 thermal boxes", n_boxes=256, edge=(8, 32), ppc=(4, 256),
                theta=(0.05, 1.0), n_x=10.0, dt=0.5, steps=500, seed=5)


def ensemble_boxes(spec=ENSEMBLE, n_boxes=None):
    """Box list of the ensemble workload: edge ~ round(exp U[ln 8, ln 32]),
    pairs per cell ~ round(exp U[ln 4, ln 256]), theta ~ U[0.05, 1]."""
    rng = np.random.default_rng(spec["seed"])
    n = spec["n_boxes"] if n_boxes is None else n_boxes
    lo, hi = spec["edge"]
    plo, phi = spec["ppc"]
    tlo, thi = spec["theta"]
    out = []
    for b in range(n):
        edge = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        ppc = int(round(np.exp(rng.uniform(np.log(plo), np.log(phi)))))
        theta = float(rng.uniform(tlo, thi))
        out.append(dict(dims=(edge, edge, edge), ppc=ppc, theta=theta, seed=1000 + b))
    return out
