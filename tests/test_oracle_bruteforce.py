"""Oracle vs the brute-force 4-index route on micro sizes.

The brute-force route forms (mu nu|lam sig) = sum_P b^P_{mu nu} b^P_{lam sig}
(Eq. cholesky) with an explicit-loop unpack, then applies the 4-index
definitions of J and K (Eq. v_emb), of the MO-basis ERI blocks (Eqs. ppaa,
papa) and of the (pa|aa) and (aa|aa) patterns (Eqs. MO_conv, flas).
"""
import numpy as np
import pytest

from oracle import brute, df_oracle as O

SIZES = [(1, 1), (2, 3), (3, 5), (7, 1), (7, 5), (12, 17), (13, 48)]


def _inputs(nao, naux, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((naux, O.npair(nao)))
    C = np.linalg.qr(rng.standard_normal((nao, nao)))[0]
    return B, C, rng


@pytest.mark.parametrize("nao,naux", SIZES)
def test_unpack_matches_explicit_loop(nao, naux):
    B, _, _ = _inputs(nao, naux, 1)
    np.testing.assert_array_equal(O.unpack(B, nao), brute.dense_B(B, nao))


@pytest.mark.parametrize("nao,naux", SIZES)
def test_jk_vs_bruteforce(nao, naux):
    B, C, rng = _inputs(nao, naux, 2)
    nocc = max(1, nao // 3)
    Cocc = C[:, :nocc]
    eri = brute.eri4(B, nao)
    J, K, v = O.jk(B, nao, Cocc)
    D = Cocc @ Cocc.T
    scale = max(1.0, np.abs(J).max())
    np.testing.assert_allclose(J, brute.coulomb(eri, D), rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(K, brute.exchange(eri, D), rtol=0, atol=1e-12 * max(1.0, np.abs(K).max()))
    # signed weights: gamma = C diag(w) C^T (a general symmetric density)
    w = rng.standard_normal(nocc)
    Jw, Kw, _ = O.jk(B, nao, Cocc, w)
    G = (Cocc * w) @ Cocc.T
    np.testing.assert_allclose(Jw, brute.coulomb(eri, G), rtol=0, atol=1e-12 * max(1.0, np.abs(Jw).max()))
    np.testing.assert_allclose(Kw, brute.exchange(eri, G), rtol=0, atol=1e-12 * max(1.0, np.abs(Kw).max()))
    np.testing.assert_allclose(O.exchange_paper_route(B, nao, G), Kw, rtol=0, atol=1e-12 * max(1.0, np.abs(Kw).max()))


@pytest.mark.parametrize("nao,naux", SIZES)
def test_jk_many_vs_bruteforce(nao, naux):
    """Several densities with one unpack per P block (a block size that splits the P range
    unevenly): each J, K, v against the 4-index definitions of its own density."""
    B, C, rng = _inputs(nao, naux, 3)
    eri = brute.eri4(B, nao)
    Cs = [np.linalg.qr(rng.standard_normal((nao, k)))[0] for k in (1, max(1, nao // 2), nao)]
    J, K, v = O.jk_many(B, nao, Cs, chunk=2)
    dense = brute.dense_B(B, nao)
    for k, Ck in enumerate(Cs):
        D = Ck @ Ck.T
        np.testing.assert_allclose(J[k], brute.coulomb(eri, D), rtol=0, atol=1e-12 * max(1.0, np.abs(J[k]).max()))
        np.testing.assert_allclose(K[k], brute.exchange(eri, D), rtol=0, atol=1e-12 * max(1.0, np.abs(K[k]).max()))
        np.testing.assert_allclose(v[k], np.einsum("pij,ij->p", dense, D), rtol=0, atol=1e-12 * max(1.0, np.abs(v[k]).max()))


@pytest.mark.parametrize("nao,naux", SIZES)
def test_half_and_second_transform_vs_explicit(nao, naux):
    B, C, _ = _inputs(nao, naux, 3)
    Bd = brute.dense_B(B, nao)
    Cr = C[:, : max(1, nao // 2)]
    X = O.half_transform(B, nao, Cr)
    ref = np.zeros_like(X)
    for P in range(naux):
        for m in range(nao):
            for c in range(Cr.shape[1]):
                ref[P, m, c] = sum(Bd[P, m, n] * Cr[n, c] for n in range(nao))
    np.testing.assert_allclose(X, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))
    Y = O.second_transform(X, C)
    ref2 = np.einsum("mp,Pmc->Ppc", C, ref)
    np.testing.assert_allclose(Y, ref2, rtol=0, atol=1e-12 * max(1.0, np.abs(ref2).max()))


@pytest.mark.parametrize("nao,naux", SIZES)
def test_active_eri_and_papa_vs_bruteforce(nao, naux):
    B, C, _ = _inputs(nao, naux, 4)
    nac = max(1, min(4, nao - 1))
    nocc = nao - nac
    Cact = C[:, nocc:nocc + nac]
    eri4 = brute.eri4(B, nao)
    eri, buv = O.active_eri(B, nao, Cact)
    ref = brute.transform4(eri4, Cact, Cact, Cact, Cact)
    np.testing.assert_allclose(eri, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))
    # (p u|v w) over all MOs p
    pa = O.papa(B, nao, C, Cact)
    refp = brute.transform4(eri4, C, Cact, Cact, Cact)
    np.testing.assert_allclose(pa, refp, rtol=0, atol=1e-12 * max(1.0, np.abs(refp).max()))
    # Eq. papa: (p u|q v) and Eq. ppaa: (p q|u v)
    Cq = C[:, : max(1, nao // 2)]
    full = O.papa_full(B, nao, C, Cact, Cq)
    reff = brute.transform4(eri4, C, Cact, Cq, Cact)
    np.testing.assert_allclose(full, reff, rtol=0, atol=1e-12 * max(1.0, np.abs(reff).max()))
    pp = O.ppaa(B, nao, C, Cq, Cact)
    refq = brute.transform4(eri4, C, Cq, Cact, Cact)
    np.testing.assert_allclose(pp, refq, rtol=0, atol=1e-12 * max(1.0, np.abs(refq).max()))


def test_identity_active_columns_give_raw_eri_entries():
    nao, naux = 9, 6
    B, _, _ = _inputs(nao, naux, 5)
    idx = [1, 4, 8]
    Cact = np.eye(nao)[:, idx]
    eri, _ = O.active_eri(B, nao, Cact)
    eri4 = brute.eri4(B, nao)
    np.testing.assert_allclose(eri, eri4[np.ix_(idx, idx, idx, idx)], rtol=0, atol=1e-13)


@pytest.mark.parametrize("nao,naux", [(1, 1), (3, 5), (7, 4), (12, 3)])
def test_second_transform_against_explicit_loops(nao, naux):
    """Eq. (ao2mo_2) after Eq. (ao2mo_1): Y[P, p, c] = sum_mu C2[mu, p] sum_nu b^P_{mu nu} C[nu, c], by
    explicit loops over the brute-force unpacked b^P; and its contraction over P equals the
    4-index transform of (mu nu|lam sig) (so the P index is not transposed with another)."""
    B, C, rng = _inputs(nao, naux, 41)
    ncol, n2 = max(1, nao // 2), max(1, nao - 1)
    Cr, C2 = C[:, :ncol], rng.standard_normal((nao, n2))
    Y = O.second_transform(O.half_transform(B, nao, Cr), C2)
    Bd = brute.dense_B(B, nao)
    ref = np.zeros((naux, n2, ncol))
    for P in range(naux):
        for p in range(n2):
            for c in range(ncol):
                s = 0.0
                for mu in range(nao):
                    for nu in range(nao):
                        s += C2[mu, p] * Bd[P, mu, nu] * Cr[nu, c]
                ref[P, p, c] = s
    np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))
    eri = brute.transform4(brute.eri4(B, nao), C2, Cr, C2, Cr)
    np.testing.assert_allclose(np.einsum("Ppc,Pqd->pcqd", Y, Y), eri, rtol=0, atol=1e-11 * max(1.0, np.abs(eri).max()))
