"""Writes mol20_grad_rows.json: oracle gradient rows of three atoms of the
20-atom gradient workload (seeded synth.mol20, Schwarz threshold 1e-11, no
primitive screening), E = 1/2 tr(PJ) - 1/4 tr(PK) at fixed P (SI eqs.
si_dE_J, si_dE_K).  Calls only the CPU oracle.

    python tests/golden/make_grad_rows.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2406_14920_amd import synth  # noqa: E402

ATOMS = (0, 9, 19)


def main():
    mol = synth.mol20()
    B = oracle.OBasis(mol)
    t = time.time()
    Q = B.schwarz()
    print("schwarz %.1fs" % (time.time() - t), flush=True)
    rows = {}
    for A in ATOMS:
        t = time.time()
        g = oracle.grad(mol, only_atom=A, Q=Q, tau_prim=0.0)
        rows[str(A)] = [float(v) for v in g[A]]
        print("atom %d: %s  %.1fs" % (A, g[A], time.time() - t), flush=True)
    out = {"workload": "synth.mol20() (seed 14924): 20 atoms, 420 spherical bf",
           "schwarz_thresh": mol.tau_schwarz, "prim_thresh": 0.0,
           "source": "oracle.grad(mol, only_atom=A, tau_prim=0.0); SI eqs. si_dE_J, si_dE_K",
           "rows": rows}
    with open(os.path.join(HERE, "mol20_grad_rows.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
