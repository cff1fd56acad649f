"""Writes tests/golden/c2_sampled.npz: FP64 oracle values for sampled outputs of
the Si-like 2-atom workload (N_aux = 260, 6x6x6 k grid, 32 frequencies).

Calls only the oracle and the seeded input generator:
  for q in Q: chi0 rows 0..15 at frequency indices W_IDX, W^c rows 0..15 at
  W_IDX (q = 0 with the Gamma head/wing treatment), and the Sigma^c
  contribution of that q for the k points K_IDX (all QP bands, all frequencies).
Run: python tests/golden/make_c2_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth.systems import make_config  # noqa: E402
from oracle.pipeline import Oracle  # noqa: E402

Q = (0, 1, 107)
W_IDX = np.array([0, 15, 31])
K_IDX = np.array([0, 1, 50, 107, 215])
ROWS = 16


def main():
    t0 = time.time()
    s = make_config(2)
    o = Oracle(s)
    out = dict(Q=np.array(Q), W_IDX=W_IDX, K_IDX=K_IDX, ROWS=np.array(ROWS), seed=np.array(s.seed))
    for q in Q:
        B = o.B(q)
        chi = o.chi0(q, B)
        Wc = o.wc(q, chi=chi, B=B, gamma=True)
        sq, _ = o.sigma_q(q, Wc, ks=list(K_IDX))
        out[f"chi_q{q}"] = chi[W_IDX, :ROWS, :]
        out[f"wc_q{q}"] = Wc[W_IDX, :ROWS, :]
        out[f"sigma_q{q}"] = sq
        print(f"q={q} done after {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "c2_sampled.npz"), **out)
    print("wrote c2_sampled.npz")


if __name__ == "__main__":
    main()
