"""Seeded synthetic inputs: reproducible, chunk-independent and shaped as stated."""
import numpy as np

from paper_2505_03755_amd import synth


def test_cholesky_rows_reproducible_and_chunk_independent():
    a = synth.cholesky_vectors(6, 9, 20.0, seed=0)
    b = synth.cholesky_vectors(6, 9, 20.0, seed=0)
    np.testing.assert_array_equal(a, b)
    tail = synth.cholesky_vectors(3, 9, 20.0, seed=0, p0=3)
    np.testing.assert_array_equal(a[3:], tail)
    assert a.shape == (6, synth.npair(9))
    c = synth.cholesky_vectors(6, 9, 20.0, seed=1)
    assert not np.array_equal(a, c)


def test_cholesky_envelope_decays_with_distance_from_diagonal():
    nao, L = 64, 4.0
    B = synth.cholesky_vectors(400, nao, L)
    il, jl = np.tril_indices(nao)
    d = il - jl
    near = B[:, d == 0].std()
    far = B[:, d == 8].std()
    # std ratio exp(-8/4) = 0.135; generous statistical bounds
    assert 0.10 < far / near < 0.17


def test_orbitals_orthonormal_and_sign_fixed():
    C = synth.orbitals(17)
    np.testing.assert_allclose(C.T @ C, np.eye(17), atol=1e-13)
    np.testing.assert_array_equal(C, synth.orbitals(17))


def test_two_body_density_has_eightfold_symmetry():
    G = synth.two_body_density(5)
    for p in ["vuwx", "uvxw", "vuxw", "wxuv", "xwuv", "wxvu", "xwvu"]:
        np.testing.assert_allclose(np.einsum("uvwx->" + p, G), G, atol=1e-15)


def test_fragment_densities_orthonormal():
    Cs = synth.fragment_densities(20, 5, 3, frag=2)
    for C in Cs:
        np.testing.assert_allclose(C.T @ C, np.eye(5), atol=1e-13)


def test_coulomb_metric_is_spd_with_the_requested_condition():
    M = synth.coulomb_metric(50, 1e5, seed=3)
    assert np.array_equal(M, M.T)
    w = np.linalg.eigvalsh(M)
    assert w[0] > 0
    assert np.isclose(w[-1] / w[0], 1e5, rtol=1e-6)
    assert np.array_equal(M, synth.coulomb_metric(50, 1e5, seed=3))
