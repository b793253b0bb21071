"""Pins of the one-pass oracle (oracle/df_stream.py).

  * J, K C_occ, K, (uv|wx), the (pu|vw) rows against the brute-force 4-index route on micro
    sizes (Eq. v_emb and the transformed blocks from the explicit-loop unpack);
  * the energy terms against their 4-index definitions (tr(D J) = sum (ij|kl) D_ij D_kl, tr(D K) =
    sum (ik|jl) D_ij D_kl);
  * dE/dC against central finite differences of the brute-force energy in C;
  * dE/dkappa: the closed form at kappa = 0 and SciPy's Frechet adjoint elsewhere agree with
    finite differences of the energy in kappa;
  * the result does not depend on the block size the rows come in.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import brute
from oracle import df_oracle as O
from oracle import df_stream as S
from paper_2505_03755_amd import synth


def brute_energy(B, nao, C, nocc, nac, h, Gam):
    eri = brute.eri4(B, nao)
    Cocc, Cact = C[:, :nocc], C[:, nocc:nocc + nac]
    D = Cocc @ Cocc.T
    J = brute.coulomb(eri, D)
    K = brute.exchange(eri, D)
    act = brute.transform4(eri, Cact, Cact, Cact, Cact)
    return (np.sum(D * h) + 0.5 * np.sum(D * J) - 0.25 * np.sum(D * K) + 0.5 * np.sum(act * Gam)), J, K, eri


@pytest.fixture(scope="module")
def prob():
    nao, naux, nocc, nac = 9, 11, 3, 3
    B = synth.cholesky_vectors(naux, nao, 4.0, seed=5)
    C = synth.orbitals(nao, seed=5)
    h = synth.symmetric_matrix(nao, seed=5)
    Gam = synth.two_body_density(nac, seed=5)
    return nao, naux, nocc, nac, B, C, h, Gam


@pytest.mark.parametrize("chunk", [1, 4, 11])
def test_pass_against_bruteforce(prob, chunk):
    nao, naux, nocc, nac, B, C, h, Gam = prob
    p_rows = [0, 4, 8]
    r = S.step_pass(S.host_chunks(B, chunk), naux, nao, C, nocc, nac, h, Gam, p_rows=p_rows, want_K=True,
                    k_rows=[8, 0, 5])
    E, J, K, eri = brute_energy(B, nao, C, nocc, nac, h, Gam)
    np.testing.assert_allclose(r["K_rows"], K[[8, 0, 5]], atol=1e-12 * np.abs(K).max())
    Cocc, Cact = C[:, :nocc], C[:, nocc:nocc + nac]
    np.testing.assert_allclose(r["J"], J, atol=1e-12 * np.abs(J).max())
    np.testing.assert_allclose(r["K"], K, atol=1e-12 * np.abs(K).max())
    np.testing.assert_allclose(r["KC"], K @ Cocc, atol=1e-12 * np.abs(K).max())
    np.testing.assert_allclose(r["eri"], brute.transform4(eri, Cact, Cact, Cact, Cact), atol=1e-12 * np.abs(eri).max())
    pa = brute.transform4(eri, C[:, p_rows], Cact, Cact, Cact)
    np.testing.assert_allclose(r["papa_rows"], pa, atol=1e-12 * np.abs(eri).max())
    D = Cocc @ Cocc.T
    np.testing.assert_allclose(r["v"], np.einsum("pij,ij->p", brute.dense_B(B, nao), D), atol=1e-12)
    assert abs(r["E"] - E) <= 1e-12 * abs(E)
    assert abs(r["E_J"] - 0.5 * np.einsum("ij,ijkl,kl->", D, eri, D)) <= 1e-12 * abs(E)
    assert abs(r["E_K"] + 0.25 * np.einsum("ij,ikjl,kl->", D, eri, D)) <= 1e-12 * abs(E)


def test_block_size_does_not_matter(prob):
    nao, naux, nocc, nac, B, C, h, Gam = prob
    a = S.step_pass(S.host_chunks(B, 2), naux, nao, C, nocc, nac, h, Gam, p_rows=[1])
    b = S.step_pass(S.host_chunks(B, 7), naux, nao, C, nocc, nac, h, Gam, p_rows=[1])
    for k in ("J", "KC", "eri", "papa_rows", "G"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-13 * np.abs(b[k]).max())
    assert abs(a["E"] - b["E"]) <= 1e-13 * abs(b["E"])


def test_blocks_must_cover_p_in_order(prob):
    nao, naux, nocc, nac, B, C, h, Gam = prob
    with pytest.raises(ValueError):
        S.step_pass(iter([(0, B[:4]), (5, B[5:])]), naux, nao, C, nocc, nac, h, Gam)
    with pytest.raises(ValueError):
        S.step_pass(iter([(0, B[:4])]), naux, nao, C, nocc, nac, h, Gam)


def test_gradient_in_C_against_finite_differences(prob):
    nao, naux, nocc, nac, B, C, h, Gam = prob
    G = S.step_pass(S.host_chunks(B, 4), naux, nao, C, nocc, nac, h, Gam)["G"]
    step = 1e-5
    fd = np.zeros_like(C)
    for i in range(nao):
        for j in range(nocc + nac):
            d = np.zeros_like(C)
            d[i, j] = step
            fd[i, j] = (brute_energy(B, nao, C + d, nocc, nac, h, Gam)[0]
                        - brute_energy(B, nao, C - d, nocc, nac, h, Gam)[0]) / (2 * step)
    np.testing.assert_allclose(G, fd, rtol=0, atol=2e-7 * np.abs(fd).max())


@pytest.mark.parametrize("scale", [0.0, 0.05])
def test_orbital_gradient_against_finite_differences(prob, scale):
    nao, naux, nocc, nac, B, C0, h, Gam = prob
    kappa = scale * np.random.default_rng(6).standard_normal((nao, nao))
    rot = lambda k: C0 @ scipy.linalg.expm(k - k.T)
    G = S.step_pass(S.host_chunks(B, 5), naux, nao, rot(kappa), nocc, nac, h, Gam)["G"]
    g = S.orbital_gradient_from_G(C0, kappa, G)
    rng = np.random.default_rng(7)
    for _ in range(6):
        d = rng.standard_normal((nao, nao))
        d /= np.linalg.norm(d)
        step = 1e-5
        fd = (brute_energy(B, nao, rot(kappa + step * d), nocc, nac, h, Gam)[0]
              - brute_energy(B, nao, rot(kappa - step * d), nocc, nac, h, Gam)[0]) / (2 * step)
        assert abs(np.sum(g * d) - fd) <= 1e-7 * np.linalg.norm(g)
    np.testing.assert_allclose(g, -g.T, atol=1e-12 * np.abs(g).max())
