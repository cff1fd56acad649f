"""Host logic of the seeded input generator (no GPU)."""
import numpy as np

from synth.systems import eigenvalues_of, make_config, make_custom, window_of, transition_window


def test_eigenvalues_of_matches_the_generator():
    for s in (make_config(1), make_custom(n_atoms=2, nb_per_atom=4, naux_per_atom=9, nk=(3, 1, 2), n_occ=2,
                                          n_freq=6, seed=43)):
        e = eigenvalues_of(s.spec, s.seed)
        assert np.array_equal(e, s.eig)
        assert window_of(e, s.spec.n_occ) == transition_window(s)


def test_streamed_coefficients_equal_the_materialised_array():
    """lri_blocks yields the coefficients make_system draws, atom by atom; a
    cell drawn without them has every other array unchanged."""
    from synth.systems import lri_blocks, make_system
    for s in (make_config(1), make_custom(n_atoms=3, nb_per_atom=5, naux_per_atom=7, nk=(2, 2, 1), n_occ=3,
                                          n_freq=6, seed=41)):
        flat = np.concatenate([b.reshape(-1) for b in lri_blocks(s.spec, s.seed)])
        assert np.array_equal(flat, s.lri)
        bare = make_system(s.spec, s.seed, materialize_lri=False)
        assert bare.lri is None and np.array_equal(bare.lri_off, s.lri_off)
        for f in ("eig", "evec", "V", "p", "R", "lattice"):
            assert np.array_equal(getattr(bare, f), getattr(s, f)), f
