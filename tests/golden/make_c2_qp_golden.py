"""Writes tests/golden/c2_qp.npz: the FP64 oracle's whole pass over the
Si-like 2-atom workload (N_aux = 260, 6x6x6 k grid, 32 frequencies, QP bands
0..7): Sigma^c_n(k, i w) summed over all 216 q (Eq. GW_selfe_element with
W -> W^c, the q = 0 term with the Gamma head/wing treatment of Sec. III B),
and the QP energies and renormalisation factors from its Pade continuation.

Calls only the oracle and the seeded input generator.  The q terms are
summed by forked worker processes over disjoint q sets (one BLAS thread each,
sharing the parent's read-only oracle tables; the partial sums are added in
q-set order), about 2 hours on seven host cores.
Run: python tests/golden/make_c2_qp_golden.py [--workers 7]
"""
import argparse
import multiprocessing as mp
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("MKL_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth.systems import make_config  # noqa: E402
from oracle.pipeline import Oracle  # noqa: E402
from oracle import grids, continuation  # noqa: E402


_O = None   # the oracle of the cell, built before the workers fork


def partial(qs):
    """Sum of the Sigma^c contributions of the q in qs."""
    t0 = time.time()
    o = _O
    s = o.sys
    sp = s.spec
    sigma = np.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=np.complex128)
    for i, q in enumerate(qs):
        B = o.B(q)
        chi = o.chi0(q, B)
        Wc = o.wc(q, chi=chi, B=B, gamma=True)
        sq, _ = o.sigma_q(q, Wc)
        sigma += sq
        print(f"q={q} ({i + 1} of {len(qs)} in this set) done after {time.time() - t0:.1f} s", flush=True)
    return sigma


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=7)
    a = ap.parse_args()
    global _O
    t0 = time.time()
    s = make_config(2)
    o = Oracle(s)
    _O = o
    sp = s.spec
    sets = [list(range(w, s.n_k, a.workers)) for w in range(a.workers)]
    with mp.get_context("fork").Pool(a.workers) as pool:
        parts = pool.map(partial, sets)
    sigma = np.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=np.complex128)
    for p in parts:
        sigma += p
    eps_qp = s.eig[:, sp.qp_lo:sp.qp_lo + sp.n_qp]
    nodes = grids.pade_nodes(sp.n_freq, o.n_par)
    E, Z, ok = continuation.qp_energies(sigma, o.omega, eps_qp, s.e_static, s.mu, nodes)
    np.savez_compressed(os.path.join(HERE, "c2_qp.npz"), sigma=sigma, E=E, Z=Z, converged=ok,
                        seed=np.array(s.seed), n_par=np.array(o.n_par))
    print(f"wrote c2_qp.npz after {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
