"""Writes tests/golden/c3_cell5_sampled.npz: FP64 oracle values for sampled
outputs of the largest cell of the batched workload (8 atoms, N_aux = 1040,
3x3x3 k grid, 16 occupied of 312 bands, 32 frequencies; cell 5, seed 3005),
with the triples formed one auxiliary atom at a time.

Calls only the oracle and the seeded input generator:
  for q in Q: chi0 rows 0..15 at frequency indices W_IDX, W^c rows 0..15 at
  W_IDX (q = 0 with the Gamma head/wing treatment), and the Sigma^c
  contribution of that q for the k points K_IDX (all QP bands, all
  frequencies).  About 20 minutes on eight host cores.
Run: python tests/golden/make_c3_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth.systems import make_config  # noqa: E402
from oracle.pipeline import Oracle  # noqa: E402

CELL = 5
Q = (0, 4)
W_IDX = np.array([0, 16, 31])
K_IDX = np.array([0, 13, 26])
ROWS = 16


def main():
    t0 = time.time()
    s = make_config(3, CELL)
    print(f"cell generated after {time.time() - t0:.1f} s", flush=True)
    o = Oracle(s, per_atom=True)
    print(f"oracle tables after {time.time() - t0:.1f} s", flush=True)
    out = dict(CELL=np.array(CELL), Q=np.array(Q), W_IDX=W_IDX, K_IDX=K_IDX, ROWS=np.array(ROWS), seed=np.array(s.seed))
    for q in Q:
        B = o.B(q)
        print(f"q={q}: triples after {time.time() - t0:.1f} s", flush=True)
        chi = o.chi0(q, B)
        print(f"q={q}: chi0 after {time.time() - t0:.1f} s", flush=True)
        Wc = o.wc(q, chi=chi, B=B, gamma=True)
        del B
        sq, _ = o.sigma_q(q, Wc, ks=list(K_IDX))
        out[f"chi_q{q}"] = chi[W_IDX, :ROWS, :]
        out[f"wc_q{q}"] = Wc[W_IDX, :ROWS, :]
        out[f"sigma_q{q}"] = sq
        del chi, Wc
        print(f"q={q} done after {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "c3_cell5_sampled.npz"), **out)
    print("wrote c3_cell5_sampled.npz")


if __name__ == "__main__":
    main()
