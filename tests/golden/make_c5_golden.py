"""Write the stored oracle results of the large-lattice workload (square 20x20, U=8, beta=10,
dtau=0.1, 100 slices) that the GPU tests compare against: the CPU oracle (reference mode, fresh G
rebuilt from scratch at every stabilisation point) sweeps two sampled chains from their seeded
fields once, at the stabilisation intervals 5 and 10 slices.

Calls only oracle/ and dqmc_inputs (the seeded inputs).  Run from the repository root:
    python tests/golden/make_c5_golden.py
It takes a few minutes of CPU time.
"""
import base64
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import dqmc_inputs as di  # noqa: E402
from oracle import Model, OracleChains  # noqa: E402

WORKLOAD = "square20x20_U8_b10"
CHAINS = (0, 37)              # sampled chain indices of the workload's seeds
INTERVALS = (5, 10)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_square20x20_U8_b10_one_sweep.json")


def pack(fields: np.ndarray) -> str:
    return base64.b64encode(np.packbits((fields > 0).ravel())).decode()


def main():
    w = di.WORKLOADS[WORKLOAD]
    rec = {"workload": WORKLOAD, "n_sites": w.n_sites, "n_slices": w.n_slices, "U": w.U,
           "beta": w.beta, "dtau": w.dtau, "sweeps": 1, "chains": {}}
    for c in CHAINS:
        seed = w.seeds(1, c)
        f0 = w.fields(1, c)
        for ns in INTERVALS:
            t0 = time.perf_counter()
            oc = OracleChains(Model(w.hopping(), w.U, w.dtau, w.n_slices, ns), f0, seed)
            oc.sweep(1)
            o = oc.measure()[0]
            key = f"{c}_ns{ns}"
            rec["chains"][key] = {
                "chain": c, "seed": int(seed[0]), "stab_every": ns,
                "fields_bits_b64": pack(oc.fields()[0]),
                "double_occ": o["double_occ"], "density": o["density"], "kinetic": o["kinetic"],
                "logdet_up": o["logdet_up"], "logdet_dn": o["logdet_dn"], "max_drift": o["max_drift"],
                "accepted": o["accepted"], "near_ties": o["near_ties"], "flags": o["flags"]}
            print(key, f"{time.perf_counter() - t0:.1f} s", {k: v for k, v in rec["chains"][key].items()
                                                              if k != "fields_bits_b64"}, flush=True)
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
