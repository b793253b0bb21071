"""Pins of the oracle that forms b^P from the three-centre integrals and the metric (Eq. cholesky),
and of its change of orbital basis."""
import numpy as np
import pytest

from oracle import brute
from oracle import df_build as OB
from oracle import df_oracle as O


def spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    return (Q * np.geomspace(1.0, 1.0 / cond, n)) @ Q.T


def test_reproduces_the_fitted_eri():
    """sum_P b^P b^P equals (mu nu|P)(P|Q)^-1(Q|lam sig) formed with a general (LU) solve."""
    naux, nao = 40, 9
    metric = spd(naux, 1e4, 1)
    E = np.random.default_rng(2).standard_normal((naux, O.npair(nao)))
    B = OB.cholesky_vectors(metric, E)
    ref = E.T @ np.linalg.solve(metric, E)
    assert np.allclose(B.T @ B, ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    # and the factor itself: L L^T = (P|Q), L lower with a positive diagonal
    L = OB.metric_cholesky(metric)
    assert np.allclose(L @ L.T, metric, rtol=0, atol=1e-13)
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) > 0)
    # L B = E (the substitution is solved, not transposed)
    assert np.allclose(L @ B, E, rtol=0, atol=1e-12 * np.abs(E).max())


def test_identity_and_diagonal_metric():
    naux, nao = 12, 5
    E = np.random.default_rng(3).standard_normal((naux, O.npair(nao)))
    assert np.array_equal(OB.cholesky_vectors(np.eye(naux), E), E)
    d = np.linspace(0.5, 4.0, naux)
    assert np.allclose(OB.cholesky_vectors(np.diag(d), E), E / np.sqrt(d)[:, None], rtol=1e-15, atol=0)


def test_hand_worked_example():
    """(P|Q) = [[4, 2], [2, 5]] = L L^T with L = [[2, 0], [1, 2]]; one pair with E = (2, 5):
    b_1 = 2/2 = 1, b_2 = (5 - 1*1)/2 = 2."""
    B = OB.cholesky_vectors(np.array([[4.0, 2.0], [2.0, 5.0]]), np.array([[2.0], [5.0]]))
    assert np.allclose(B, [[1.0], [2.0]], rtol=0, atol=1e-15)


def test_embedding_against_four_index_transform():
    naux, nao, ne = 6, 7, 4
    rng = np.random.default_rng(4)
    B = rng.standard_normal((naux, O.npair(nao)))
    M = rng.standard_normal((nao, ne))
    Be = OB.embed(B, nao, M)
    assert Be.shape == (naux, O.npair(ne))
    ref = brute.transform4(brute.eri4(B, nao), M, M, M, M)
    assert np.allclose(brute.eri4(Be, ne), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # rows of b^P themselves: the identity basis leaves B unchanged, a permutation permutes it
    assert np.allclose(OB.embed(B, nao, np.eye(nao)), B, rtol=0, atol=0)
    perm = rng.permutation(nao)
    Bp = brute.dense_B(OB.embed(B, nao, np.eye(nao)[:, perm]), nao)
    assert np.array_equal(Bp, brute.dense_B(B, nao)[:, perm][:, :, perm])


def test_not_positive_definite_is_rejected():
    with pytest.raises(np.linalg.LinAlgError):
        OB.metric_cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
