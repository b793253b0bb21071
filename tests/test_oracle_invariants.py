"""Oracle invariants and special cases that hold at any size."""
import math

import numpy as np
import pytest

from oracle import df_oracle as O
from paper_2505_03755_amd import synth


@pytest.fixture(scope="module")
def small():
    nao, naux, nocc, nac = 40, 70, 11, 5
    B = synth.cholesky_vectors(naux, nao, 10.0, seed=7)
    C = synth.orbitals(nao, seed=7)
    return nao, naux, nocc, nac, B, C


def test_symmetry_and_psd(small):
    nao, naux, nocc, nac, B, C = small
    J, K, v = O.jk(B, nao, C[:, :nocc])
    np.testing.assert_allclose(J, J.T, atol=1e-12)
    np.testing.assert_allclose(K, K.T, atol=1e-12)
    ev = np.linalg.eigvalsh((K + K.T) / 2)
    assert ev.min() > -1e-10 * ev.max()


def test_trace_identities(small):
    nao, naux, nocc, nac, B, C = small
    Cocc = C[:, :nocc]
    D = Cocc @ Cocc.T
    J, K, v = O.jk(B, nao, Cocc)
    # tr(DJ) = sum_P v_P^2 (from Eqs. J_1 and J_2)
    assert math.isclose(O.fsum_dot(D, J), math.fsum((v * v).tolist()), rel_tol=1e-12)
    # tr(DK) = sum_P ||Cocc^T B_P Cocc||_F^2
    Bd = O.unpack(B, nao)
    s = math.fsum(float(np.sum((Cocc.T @ Bd[P] @ Cocc) ** 2)) for P in range(naux))
    assert math.isclose(O.fsum_dot(D, K), s, rel_tol=1e-12)


def test_occupied_rotation_invariance(small):
    nao, naux, nocc, nac, B, C = small
    Cocc = C[:, :nocc]
    U = np.linalg.qr(np.random.default_rng(3).standard_normal((nocc, nocc)))[0]
    J1, K1, v1 = O.jk(B, nao, Cocc)
    J2, K2, v2 = O.jk(B, nao, Cocc @ U)
    np.testing.assert_allclose(J2, J1, atol=1e-11 * np.abs(J1).max())
    np.testing.assert_allclose(K2, K1, atol=1e-11 * np.abs(K1).max())
    np.testing.assert_allclose(v2, v1, atol=1e-11 * np.abs(v1).max())


def test_identity_density_special_case(small):
    nao, naux, nocc, nac, B, C = small
    Bd = O.unpack(B, nao)
    J, K, v = O.jk(B, nao, np.eye(nao))
    np.testing.assert_allclose(v, np.trace(Bd, axis1=1, axis2=2), atol=1e-12)
    np.testing.assert_allclose(J, np.einsum("p,pij->ij", np.trace(Bd, axis1=1, axis2=2), Bd), atol=1e-10)
    np.testing.assert_allclose(K, np.einsum("pik,pkj->ij", Bd, Bd), atol=1e-10)


def test_single_aux_closed_form():
    nao = 23
    B = synth.cholesky_vectors(1, nao, 5.0, seed=2)
    C = synth.orbitals(nao, seed=2)[:, :6]
    b = O.unpack(B, nao)[0]
    D = C @ C.T
    J, K, v = O.jk(B, nao, C)
    np.testing.assert_allclose(J, np.sum(b * D) * b, atol=1e-12)
    np.testing.assert_allclose(K, b @ D @ b, atol=1e-12)


def test_two_k_routes_agree(small):
    nao, naux, nocc, nac, B, C = small
    Cocc = C[:, :nocc]
    K1 = O.exchange(B, nao, Cocc)
    K2 = O.exchange_paper_route(B, nao, Cocc @ Cocc.T)
    np.testing.assert_allclose(K1, K2, rtol=0, atol=1e-13 * np.abs(K1).max())


def test_active_eri_symmetry_and_gram(small):
    nao, naux, nocc, nac, B, C = small
    Cact = C[:, nocc:nocc + nac]
    eri, buv = O.active_eri(B, nao, Cact)
    for p in ["vuwx", "uvxw", "vuxw", "wxuv", "xwuv", "wxvu", "xwvu"]:
        np.testing.assert_allclose(np.einsum("uvwx->" + p, eri), eri, atol=1e-12)
    G = eri.reshape(nac * nac, nac * nac)
    ev = np.linalg.eigvalsh(G)
    assert ev.min() > -1e-10 * ev.max()
    assert np.linalg.matrix_rank(G, tol=1e-9 * ev.max()) <= min(naux, nac * (nac + 1) // 2)


def test_papa_symmetry_and_active_slice(small):
    nao, naux, nocc, nac, B, C = small
    Cact = C[:, nocc:nocc + nac]
    pa = O.papa(B, nao, C, Cact)
    np.testing.assert_allclose(pa, pa.transpose(0, 1, 3, 2), atol=1e-12)
    eri, _ = O.active_eri(B, nao, Cact)
    np.testing.assert_allclose(pa[nocc:nocc + nac], eri, atol=1e-12)
    full = O.papa_full(B, nao, C, Cact, C)
    G = full.reshape(nao * nac, nao * nac)
    np.testing.assert_allclose(G, G.T, atol=1e-11)
    np.testing.assert_allclose(full[:, :, nocc:nocc + nac, :], pa.transpose(0, 1, 2, 3), atol=1e-11)


def test_chunking_does_not_change_results(small):
    nao, naux, nocc, nac, B, C = small
    a = O.jk(B, nao, C[:, :nocc], chunk=7)
    b = O.jk(B, nao, C[:, :nocc], chunk=240)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, atol=1e-12 * np.abs(y).max())
