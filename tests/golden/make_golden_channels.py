"""Write the stored oracle results of the channel-wise compression at full size
(calls only oracle/ and workloads/).

Output (tests/golden/):
  tb4_36x36_channels.json        exciton-shift table of channel-wise truncation and the chosen fraction
  tb4_36x36_channel_series.npz   FP64 oracle P, J, occ (4000 steps) with the channel-wise kernel at
                                 the chosen fraction

The fixed-error criterion is the one of make_golden.py (the paper's accuracy
criterion for its 5 % point, Sec. "SVD acceleration of TD-aGW": the first
bright exciton of the Tamm-Dancoff Hamiltonian dE + K moves by at most 0.04 eV),
here over the fraction kept per off-diagonal channel (Eq. svd-channel-wise,
the diagonal channels kept whole, as in the paper's "K^{diag-ch} + 5 % K^{off-ch}").
Run:  python -m tests.golden.make_golden_channels   (about ten minutes on 8 cores)
"""

from __future__ import annotations

import json
import os
import time

import numpy as np

import oracle as O
from tests.golden.make_golden import SHIFT_EV, first_bright
from workloads import HARTREE_EV, get_config

HERE = os.path.dirname(os.path.abspath(__file__))
FRACTIONS = [0.01, 0.02, 0.05, 0.1, 0.2]


def assemble(f, nk, npair):
    """Dense matrix of the channel-wise kernel (block (p, q) at rows p::P, columns q::P)."""
    n = nk * npair
    kt = np.zeros((n, n), dtype=np.complex128)
    for p in range(npair):
        kt[p::npair, p::npair] = f["diag"][p]
        for q in range(npair):
            if q != p:
                s, vh, _ = f["off"][(p, q)]
                kt[p::npair, q::npair] = s @ vh
    return kt


def main():
    cfg = get_config(1)
    m = cfg.model()
    nk, npair = m.nk, (m.nb - m.nv) * m.nv
    t0 = time.time()
    k = O.build_kernel(m, cfg.r0, "eh")
    e_dense, _ = first_bright(m, k)
    print(f"dense first bright exciton {e_dense * HARTREE_EV:.4f} eV, {time.time() - t0:.0f} s", flush=True)
    rows, chosen = [], None
    for frac in FRACTIONS:
        f = O.compress_channelwise(k, nk, npair, "fraction", frac)
        e, _ = first_bright(m, assemble(f, nk, npair))
        ranks = sorted({int(r) for (p, q), r in f["ranks"].items() if p != q})
        kept = sum(int(r) for (p, q), r in f["ranks"].items() if p != q)
        # stored complex elements: whole diagonal channels + S and V^H of the off-diagonal ones
        stored = npair * nk * nk + 2 * nk * kept
        row = {"fraction": frac, "ranks": ranks, "shift_ev": (e - e_dense) * HARTREE_EV,
               "stored_fraction_of_dense": stored / float((nk * npair) ** 2)}
        rows.append(row)
        print(row, f"{time.time() - t0:.0f} s", flush=True)
        if chosen is None and abs(row["shift_ev"]) <= SHIFT_EV:
            chosen = (frac, f)
    frac, f = chosen
    out = O.propagate(m, O.ChannelOp(f, nk, npair), "eh", cfg.fields, cfg.dt)
    print(f"propagation at fraction {frac} in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "tb4_36x36_channel_series.npz"), P=out["P"], J=out["J"], occ=out["occ"])
    info = {"workload": cfg.name, "criterion": {"bright_exciton_shift_ev": SHIFT_EV},
            "dense_first_bright_ev": e_dense * HARTREE_EV, "table": rows,
            "chosen": {"fraction": frac, "ranks": {f"{p},{q}": int(r) for (p, q), r in f["ranks"].items()}}}
    with open(os.path.join(HERE, "tb4_36x36_channels.json"), "w") as fh:
        json.dump(info, fh, indent=1)


if __name__ == "__main__":
    main()
