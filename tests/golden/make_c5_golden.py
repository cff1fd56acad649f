"""Writes tests/golden/c5_sampled.npz: FP64 oracle values for sampled outputs of
the 16-atom workload (N_b 624, N_aux 2080, 3x3x3 k grid, 32 occupied bands,
48 frequencies) at one q: chi~ and W^c rows ROWS at the frequency indices
W_IDX, and their diagonals.

The cell's LRI coefficients (50 GB) are never held whole: the oracle takes
them atom by atom from the generator's stream, forms the triples one
auxiliary atom at a time, and sums the response one k at a time (B of one k
is 0.6 GB).  Peak host memory about 50 GB (the Bloch-transformed
coefficients at +k and -k); about 15 minutes on eight host cores.

Calls only the oracle and the seeded input generator.
Run: python tests/golden/make_c5_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth.systems import lri_blocks, make_config  # noqa: E402
from oracle.pipeline import Oracle  # noqa: E402

Q = 5
W_IDX = np.array([0, 24, 47])
ROWS = np.array([0, 129, 130, 2079])   # first and last function, and an atom boundary


def main():
    t0 = time.time()
    s = make_config(5, materialize_lri=False)
    print(f"cell (without its coefficients) after {time.time() - t0:.1f} s", flush=True)

    def blocks():
        for A, blk in enumerate(lri_blocks(s.spec, s.seed)):
            yield blk
            print(f"  atom {A} transformed after {time.time() - t0:.1f} s", flush=True)

    o = Oracle(s, per_atom=True, lri_blocks=blocks())
    om = o.omega[W_IDX]
    chi = None
    for k in range(s.n_k):
        part = o.chi0(Q, omega=om, ks=[k])
        chi = part if chi is None else chi + part
        print(f"  k={k}: response terms after {time.time() - t0:.1f} s", flush=True)
    Wc = o.wc(Q, chi=chi)
    np.savez_compressed(os.path.join(HERE, "c5_sampled.npz"), Q=np.array(Q), W_IDX=W_IDX, ROWS=ROWS,
                        seed=np.array(s.seed), chi_rows=chi[:, ROWS, :], wc_rows=Wc[:, ROWS, :],
                        chi_diag=np.einsum("wii->wi", chi), wc_diag=np.einsum("wii->wi", Wc))
    print(f"wrote c5_sampled.npz after {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
