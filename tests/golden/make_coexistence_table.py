"""Write lbm_inputs/coexistence_tau.json: the bulk densities a flat
liquid-vapour interface settles at under the velocity-shift Shan–Chen
scheme (Sec. II.A, Eqs. ueq and uhydro), as a function of G and tau.

With the velocity shift the coexistence densities depend on tau (at
G = -5.5: 2.307 / 0.104 at tau = 1, 2.272 / 0.074 at tau = 0.8), so drops and
threads started at the tau-free mechanical-stability values condense or
evaporate before they do anything else.  The input recipes start them here
instead.  Each entry is the planar scheme on a 1 x 64 lattice (Table I's
set-up) with the interface at r = 32, free-slip planes, 20 000 steps from a
tanh profile between the mechanical-stability densities; a pair of nulls
marks a (G, tau) at which the interface does not stay finite.

Run from the repository root:  python tests/golden/make_coexistence_table.py
(calls only the CPU oracle; about 80 s)."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from lbm_inputs import coexistence_densities, node_coords, tanh_profile  # noqa: E402

G_GRID = [round(-6.0 + 0.1 * k, 1) for k in range(11)]
TAU_GRID = [round(0.6 + 0.05 * k, 2) for k in range(9)]
STEPS, NR = 20000, 64


def flat_interface(G, tau):
    rg, rl = coexistence_densities(G)
    p = O.make_params(1, NR, G=G, tau=tau, wall=1, axisym=0)
    _, r = node_coords(1, NR)
    rho = tanh_profile(r, NR / 2.0, rl, rg, 2.0)
    f = O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), STEPS)
    rr, _, _ = O.moments(p, f)
    if not np.isfinite(rr).all():
        return None, None
    return float(rr[-1, 0]), float(rr[0, 0])


def main():
    table = {"G": G_GRID, "tau": TAU_GRID, "rho_g": [], "rho_l": [],
             "recipe": f"planar 1 x {NR}, interface at r = {NR // 2}, free-slip, {STEPS} steps (oracle)"}
    for G in G_GRID:
        row_g, row_l = [], []
        for tau in TAU_GRID:
            g, l = flat_interface(G, tau)
            row_g.append(g)
            row_l.append(l)
            print(f"G={G} tau={tau}: rho_l={l} rho_g={g}", flush=True)
        table["rho_g"].append(row_g)
        table["rho_l"].append(row_l)
    out = os.path.join(ROOT, "lbm_inputs", "coexistence_tau.json")
    with open(out, "w") as fh:
        json.dump(table, fh, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
