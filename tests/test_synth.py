"""Host logic of the seeded input generator (no GPU)."""
import numpy as np

from synth.systems import eigenvalues_of, make_config, make_custom, window_of, transition_window


def test_eigenvalues_of_matches_the_generator():
    for s in (make_config(1), make_custom(n_atoms=2, nb_per_atom=4, naux_per_atom=9, nk=(3, 1, 2), n_occ=2,
                                          n_freq=6, seed=43)):
        e = eigenvalues_of(s.spec, s.seed)
        assert np.array_equal(e, s.eig)
        assert window_of(e, s.spec.n_occ) == transition_window(s)
