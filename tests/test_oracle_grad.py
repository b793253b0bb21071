"""Pins for the gradient oracle: central finite differences (h = 1e-5), redundant rotations,
occupied-rotation invariance, and the vector-Jacobian product against finite differences."""
import numpy as np
import pytest

from oracle import df_grad as G
from oracle import df_oracle as O
from paper_2505_03755_amd import synth


@pytest.fixture(scope="module")
def prob():
    nao, naux, nocc, nac = 10, 7, 3, 3
    B = synth.cholesky_vectors(naux, nao, 4.0, seed=3)
    C0 = synth.orbitals(nao, seed=3)
    h = synth.symmetric_matrix(nao, seed=3)
    Gam = synth.two_body_density(nac, seed=3)
    return nao, naux, nocc, nac, B, C0, h, Gam


def fd_kappa(prob, kappa, step=1e-5):
    nao, naux, nocc, nac, B, C0, h, Gam = prob
    g = np.zeros_like(kappa)
    for i in range(nao):
        for j in range(nao):
            d = np.zeros_like(kappa)
            d[i, j] = step
            ep = G.energy(B, nao, G.rotate(C0, kappa + d), nocc, nac, h, Gam)
            em = G.energy(B, nao, G.rotate(C0, kappa - d), nocc, nac, h, Gam)
            g[i, j] = (ep - em) / (2 * step)
    return g


@pytest.mark.parametrize("scale", [0.0, 0.05])
def test_orbital_gradient_vs_finite_differences(prob, scale):
    nao = prob[0]
    kappa = scale * np.random.default_rng(4).standard_normal((nao, nao))
    g = G.orbital_gradient(prob[4], nao, prob[5], kappa, prob[2], prob[3], prob[6], prob[7])
    fd = fd_kappa(prob, kappa)
    np.testing.assert_allclose(g, fd, rtol=0, atol=2e-7 * np.abs(fd).max())
    np.testing.assert_allclose(g, -g.T, atol=1e-12 * np.abs(g).max())


def test_redundant_rotations_vanish(prob):
    nao, naux, nocc, nac, B, C0, h, Gam = prob
    g = G.orbital_gradient(B, nao, C0, np.zeros((nao, nao)), nocc, nac, h, Gam)
    scale = np.abs(g).max()
    assert np.abs(g[:nocc, :nocc]).max() <= 1e-12 * scale        # occupied-occupied
    assert np.abs(g[nocc + nac:, nocc + nac:]).max() == 0.0      # virtual-virtual
    assert np.abs(g[:nocc, nocc + nac:]).max() > 1e-3 * scale    # occupied-virtual is not redundant


def test_energy_invariant_under_occupied_rotation(prob):
    nao, naux, nocc, nac, B, C0, h, Gam = prob
    k = np.zeros((nao, nao))
    k[:nocc, :nocc] = np.random.default_rng(9).standard_normal((nocc, nocc))
    e0 = G.energy(B, nao, C0, nocc, nac, h, Gam)
    e1 = G.energy(B, nao, G.rotate(C0, k), nocc, nac, h, Gam)
    assert abs(e1 - e0) <= 1e-12 * abs(e0)


def test_energy_terms_consistent(prob):
    nao, naux, nocc, nac, B, C0, h, Gam = prob
    t = G.energy_terms(B, nao, C0, nocc, nac, h, Gam)
    assert abs(t["J"] - t["J_from_v"]) <= 1e-12 * abs(t["J"])       # tr(DJ) = sum_P v_P^2
    assert t["K"] < 0                                                # K is positive semidefinite


def test_gradient_in_C_vs_finite_differences(prob):
    nao, naux, nocc, nac, B, C0, h, Gam = prob
    C = C0 + 0.1 * np.random.default_rng(1).standard_normal(C0.shape)   # not orthonormal: a plain function of C
    g = G.energy_gradient_C(B, nao, C, nocc, nac, h, Gam)
    dirs = synth.directions(6, C.shape, seed=2)
    for d in dirs:
        step = 1e-5
        fd = (G.energy(B, nao, C + step * d, nocc, nac, h, Gam) - G.energy(B, nao, C - step * d, nocc, nac, h, Gam)) / (2 * step)
        assert abs(fd - np.sum(g * d)) <= 1e-7 * max(1.0, abs(fd))


def test_vjp_vs_finite_differences(prob):
    nao, naux, nocc, nac, B, C0, h, Gam = prob
    rng = np.random.default_rng(5)
    Cocc, Cact = C0[:, :nocc], C0[:, nocc:nocc + nac]
    gJ, gK = rng.standard_normal((nao, nao)), rng.standard_normal((nao, nao))
    geri = rng.standard_normal((nac,) * 4)
    dCo, dCa = G.step_vjp(B, nao, Cocc, Cact, gJ, gK, geri)
    for _ in range(4):
        Do, Da = rng.standard_normal(Cocc.shape), rng.standard_normal(Cact.shape)
        step = 1e-5
        Fp = G.forward(B, nao, Cocc + step * Do, Cact + step * Da)
        Fm = G.forward(B, nao, Cocc - step * Do, Cact - step * Da)
        fd = sum(np.sum(g * (p - m)) for g, p, m in zip((gJ, gK, geri), Fp, Fm)) / (2 * step)
        lin = np.sum(dCo * Do) + np.sum(dCa * Da)
        assert abs(fd - lin) <= 1e-7 * max(1.0, abs(fd))
