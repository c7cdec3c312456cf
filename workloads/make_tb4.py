"""Write workloads/data/tb4_model.json: the stored random four-band model.

Rule: the first seed >= 0 whose minimum direct gap between band 2 and band 3
(the highest valence and lowest conduction band) on a 240 x 240 grid is at
least 0.5 eV, with on-site splitting H0 = diag(D, D, -D, -D), D = 1 eV.
Run:  python -m workloads.make_tb4
"""

import json
import os

import numpy as np

from .models import HARTREE_EV, draw_tb4_hoppings, mp_grid, tb4_hamiltonian

DELTA_EV = 1.0
MIN_GAP_EV = 0.5
SCAN_GRID = 240


def min_direct_gap_ev(tx, ty, delta_ev=DELTA_EV, nk=SCAN_GRID):
    a = 1.0
    kpts = mp_grid(nk, nk, a, 0.5)
    gap = np.inf
    for chunk in np.array_split(kpts, 16):
        hk, _ = tb4_hamiltonian(chunk, a, tx / HARTREE_EV, ty / HARTREE_EV, delta_ev / HARTREE_EV)
        e = np.linalg.eigvalsh(hk)
        gap = min(gap, float((e[:, 2] - e[:, 1]).min()))
    return gap * HARTREE_EV


def main():
    seed = 0
    while True:
        tx, ty = draw_tb4_hoppings(seed)
        g = min_direct_gap_ev(tx, ty)
        if g >= MIN_GAP_EV:
            break
        seed += 1
    out = {
        "rule": "first seed >= 0 with min direct gap (band 2 -> 3) >= 0.5 eV on a 240x240 grid",
        "seed": seed,
        "delta_ev": DELTA_EV,
        "min_direct_gap_ev": g,
        "tx_re": tx.real.tolist(), "tx_im": tx.imag.tolist(),
        "ty_re": ty.real.tolist(), "ty_im": ty.imag.tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "tb4_model.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"seed {seed}: min direct gap {g:.4f} eV -> {path}")


if __name__ == "__main__":
    main()
