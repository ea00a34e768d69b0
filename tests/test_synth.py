"""The seeded input generators: determinism, subset regeneration and the
unitarity of the synthetic reflectors."""
import numpy as np

import synth


def test_gaussian_column_subset_matches_full():
    full = synth.gaussian(50, 200, 9, "z")
    cols = [0, 63, 64, 130, 199]
    assert np.array_equal(synth.gaussian(50, 200, 9, "z", cols=cols), full[:, cols])
    assert np.array_equal(synth.gaussian(50, 200, 9, "z"), full)
    assert abs(np.mean(np.abs(full) ** 2) - 1) < 0.05


def test_unitary_reflectors_are_unitary():
    lengths = np.array([2, 5, 64, 64, 17, 3])
    for dt in ["d", "z"]:
        V, tau = synth.unitary_reflectors(lengths, 64, 5, dt)
        for k, L in enumerate(lengths):
            v = V[k, :L]
            assert v[0] == 1 and np.all(V[k, L:] == 0)
            H = np.eye(L) - tau[k] * np.outer(v, np.conj(v))
            assert np.linalg.norm(np.conj(H.T) @ H - np.eye(L)) < 1e-14 * L
            assert 1 - 1e-12 <= (tau[k] * np.vdot(v, v)).real <= 2 + 1e-12


def test_band_matrix_layout_and_shift():
    ab = synth.band_matrix(10, 3, 1, "z", diag_shift=True)
    assert ab.shape == (4, 10) and np.all(ab[0].imag == 0)
    assert np.all(ab[3, 7:] == 0)
    B = synth.dense_from_band(ab)
    assert np.allclose(B, np.conj(B.T))
    assert np.all(np.abs(np.tril(B, -4)) == 0)


def test_batched_sizes():
    n = synth.batched_sizes()
    assert len(n) == 64 and set(np.unique(n)) <= set(512 * np.arange(1, 9))
