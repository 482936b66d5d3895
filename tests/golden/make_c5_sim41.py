"""Writes c5_sim41_oracle.json: the oracle's forward sensitivity of sim 41 of
the batched footing set (81,608 particles; the sim whose central-difference
gradient departs most from the adjoint) over the first 11 load steps:
reaction curve R at its drawn (E, phi), the target curve Rt at its target
(E, phi), dR/d(E, phi) per step, and the gradient of the squared misfit
sum_k (R_k - Rt_k)^2.  Calls only the oracle and the input generator.
Run from the repository root: python tests/golden/make_c5_sim41.py"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2507_09435_amd import workloads as W  # noqa: E402

SIM, STEPS = 41, 11


def main():
    sims, targets = W.make_c5(nsim=64, n_steps=30)
    w = sims[SIM]
    P = w.prob
    nodes, rd = w.footing_nodes(), P.dim - 1
    bcs = [w.bc(k) for k in range(STEPS)]
    R, dR, _ = O.simulate_sensitivity(P, w.particles, bcs, nodes, rd, tol=1e-12, line_search=4)
    st_t = w.particles.copy()
    st_t.E = np.full(st_t.np, targets[SIM][0])
    st_t.phi = np.full(st_t.np, targets[SIM][1])
    Rt, _, _ = O.simulate_sensitivity(P, st_t, bcs, nodes, rd, tol=1e-12, line_search=4)
    g = (2.0 * (R - Rt)[:, None] * dR).sum(axis=0)
    out = {"sim": SIM, "steps": STEPS, "particles": int(w.particles.np), "E": float(w.particles.E[0]),
           "phi": float(w.particles.phi[0]), "target": [float(targets[SIM][0]), float(targets[SIM][1])],
           "R": R.tolist(), "Rt": Rt.tolist(), "dR_dE": dR[:, 0].tolist(), "dR_dphi": dR[:, 1].tolist(),
           "dL_dE": float(g[0]), "dL_dphi": float(g[1])}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_sim41_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
