"""Write tests/golden/*.json from the CPU oracle only (never from the GPU path).

cas8.json: the (8e,8o) synthetic active space (seed 0, L = 24): dense FCI
ground-state energy and the number of connected determinant pairs of the
full space (diagonal included).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import hci_synth as hs  # noqa: E402
import oracle as O  # noqa: E402


def main():
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    sp = hs.full_space(w.norb, w.nalpha, w.nbeta)
    e, c = O.lowest_eigenpair(h, g, sp)
    nnz = int(O.row_counts(w.norb, sp).sum())
    out = {"workload": "cas8", "e_fci": e, "nnz": nnz, "n_det": int(len(sp)),
           "generator": "tests/golden/make_golden.py (oracle only)"}
    with open(os.path.join(HERE, "cas8.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
