"""Write the stored oracle results used at full size (calls only oracle/ and workloads/).

Output (tests/golden/):
  tb4_36x36_fixed_error.json   rank table of the fixed-error criterion and the chosen rank
  tb4_36x36_oracle_series.npz  FP64 oracle P, J, occ of the 36x36 four-band workload
                               (4000 steps): dense kernel (dense_*), dense kernel rounded
                               to complex64 (pert_*), compressed kernel at the chosen rank
                               (low_*) and at the exciton-shift point alone (paper_*)

Fixed-error criterion: among kept fractions of the singular values of K_off
in FRACTIONS, the smallest whose FP64 compressed kernel
  (1) moves the first bright exciton of the Tamm-Dancoff Hamiltonian dE + K
      by at most 0.04 eV (the paper's accuracy criterion for its 5 % point,
      Sec. "SVD acceleration of TD-aGW"), and
  (2) keeps the relative L2 error of P(t) against the dense FP64 run within
      5e-2 over the first half of the run (t <= t0).
The strong-field run of this workload is chaotic after the pulse peak (a
6e-8 perturbation of K grows to ~3e-4 in P(t) by the end, recorded as the
sensitivity), so the L2 criterion is taken where trajectories are still
predictable.  The smallest fraction meeting (1) alone is stored as well.
Run:  python -m tests.golden.make_golden   (several minutes on 8 cores)
"""

from __future__ import annotations

import json
import os
import time

import numpy as np
import scipy.linalg

import oracle as O
from workloads import HARTREE_EV, get_config

HERE = os.path.dirname(os.path.abspath(__file__))
FRACTIONS = [0.005, 0.01, 0.02, 0.03, 0.05, 0.075, 0.1, 0.15, 0.2]
SHIFT_EV = 0.04
EPS_P_L2 = 5e-2
NLOW = 40


def first_bright(model, kmat, nlow=NLOW):
    """Lowest exciton of dE + K (cv block) with oscillator strength >= 1e-2 of the
    strongest among the nlow lowest states, |<A^S | e.d_cv>|^2, field along x."""
    amat, lab = O.linear_operator(model, kmat, "eh")
    ev, vec = scipy.linalg.eigh(amat, subset_by_index=[0, nlow - 1])
    kn, n, m = lab[:, 0], lab[:, 1], lab[:, 2]
    osc = np.abs(vec.conj().T @ model.dip[0][kn, n, m]) ** 2
    i = int(np.argmax(osc >= 1e-2 * osc.max()))
    return float(ev[i]), float(ev[0])


def main():
    cfg = get_config(1)
    m = cfg.model()
    t0 = time.time()
    k = O.build_kernel(m, cfg.r0, "eh")
    print(f"kernel {k.shape} in {time.time() - t0:.0f} s", flush=True)
    kdiag, koff = O.split_diag(k)
    u, s, vh = O.svd_offdiag(koff, "eigh")
    print(f"svd in {time.time() - t0:.0f} s", flush=True)
    n = k.shape[0]
    e_dense, e_low_dense = first_bright(m, k)
    ref = O.propagate(m, O.DenseOp(k), "eh", cfg.fields, cfg.dt)
    print(f"dense propagation in {time.time() - t0:.0f} s", flush=True)
    half = int(cfg.fields.nsteps[0]) // 2 + 1

    def errs(out):
        def l2(key, sl):
            a, b = out[key][sl], ref[key][sl]
            return float(np.linalg.norm(a - b) / np.linalg.norm(b - ref[key][0]))
        return {"err_P_l2_first_half": l2("P", slice(0, half)), "err_P_l2_full": l2("P", slice(None)),
                "err_J_l2_first_half": l2("J", slice(0, half)), "err_J_l2_full": l2("J", slice(None))}

    # sensitivity: the same dense run with K rounded to complex64
    k32 = k.astype(np.complex64).astype(np.complex128)
    pert = O.propagate(m, O.DenseOp(k32), "eh", cfg.fields, cfg.dt)
    nq = int(cfg.fields.nsteps[0])
    scale = np.abs(ref["P"]).max()
    sens = {f"err_P_max_to_step_{q}": float(np.abs(pert["P"][:q + 1] - ref["P"][:q + 1]).max() / scale)
            for q in (nq // 4, nq // 2, 3 * nq // 4, nq)}
    print("sensitivity", sens, f"{time.time() - t0:.0f} s", flush=True)
    rows = []
    chosen = paper = None
    series_low = series_paper = None
    for frac in FRACTIONS:
        r = O.choose_rank(s, "fraction", frac)
        fac = {"kdiag": kdiag, "US": u[:, :r] * s[None, :r], "Vh": vh[:r]}
        ktil = np.diag(kdiag) + fac["US"] @ fac["Vh"]
        e_b, e_0 = first_bright(m, ktil)
        out = O.propagate(m, O.LowRankOp.from_factors(fac), "eh", cfg.fields, cfg.dt)
        row = {"fraction": frac, "rank": int(r), "bright_exciton_ev": e_b * HARTREE_EV,
               "shift_ev": (e_b - e_dense) * HARTREE_EV, **errs(out)}
        rows.append(row)
        print(row, f"{time.time() - t0:.0f} s", flush=True)
        if paper is None and abs(row["shift_ev"]) <= SHIFT_EV:
            paper = row
            series_paper = out
        if chosen is None and abs(row["shift_ev"]) <= SHIFT_EV and row["err_P_l2_first_half"] <= EPS_P_L2:
            chosen = row
            series_low = out
    rel_cut = int(O.choose_rank(s, "rel_cut", 1e-3))
    info = {
        "workload": cfg.name, "n": int(n),
        "criterion": {"bright_exciton_shift_ev": SHIFT_EV, "err_P_l2_first_half": EPS_P_L2},
        "sensitivity_k_rounded_to_c64": sens,
        "dense_bright_exciton_ev": e_dense * HARTREE_EV, "dense_lowest_exciton_ev": e_low_dense * HARTREE_EV,
        "rank_rel_cut_1e-3": rel_cut, "table": rows, "chosen": chosen, "shift_only": paper,
    }
    with open(os.path.join(HERE, "tb4_36x36_fixed_error.json"), "w") as f:
        json.dump(info, f, indent=1)
    np.savez_compressed(os.path.join(HERE, "tb4_36x36_oracle_series.npz"),
                        dense_P=ref["P"], dense_J=ref["J"], dense_occ=ref["occ"],
                        pert_P=pert["P"], pert_J=pert["J"], pert_occ=pert["occ"],
                        low_P=series_low["P"], low_J=series_low["J"], low_occ=series_low["occ"],
                        low_rank=np.array([chosen["rank"]]), low_fraction=np.array([chosen["fraction"]]),
                        paper_P=series_paper["P"], paper_J=series_paper["J"], paper_occ=series_paper["occ"],
                        paper_rank=np.array([paper["rank"]]), paper_fraction=np.array([paper["fraction"]]))
    print(json.dumps(info, indent=1))


if __name__ == "__main__":
    main()
