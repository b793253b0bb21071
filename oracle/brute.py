"""Brute-force 4-index route, for tiny sizes only.

TEST INFRASTRUCTURE ONLY (see ``oracle/df_oracle.py``).  This module forms the
full density-fitted ERI tensor (mu nu|lam sig) = sum_P b^P_{mu nu} b^P_{lam sig}
(Eq. cholesky) and evaluates every quantity straight from its 4-index
definition (Eqs. v_emb, ppaa, papa and the index patterns of Eqs. MO_conv and
flas), with no density-fitting shortcut.  It is the independent route the
factored oracle is checked against.
"""
from __future__ import annotations

import numpy as np


def dense_B(B: np.ndarray, nao: int) -> np.ndarray:
    """Unpack with explicit loops over (i, j): b^P_{ij} = b^P_{ji} = B[P, i(i+1)/2 + j], i >= j."""
    naux = B.shape[0]
    out = np.zeros((naux, nao, nao))
    for P in range(naux):
        k = 0
        for i in range(nao):
            for j in range(i + 1):
                out[P, i, j] = B[P, k]
                out[P, j, i] = B[P, k]
                k += 1
    return out


def eri4(B: np.ndarray, nao: int) -> np.ndarray:
    """(mu nu|lam sig) = sum_P b^P_{mu nu} b^P_{lam sig}, shape (nao,)*4."""
    Bd = dense_B(B, nao)
    return np.einsum("pmn,pls->mnls", Bd, Bd)


def coulomb(eri: np.ndarray, D: np.ndarray) -> np.ndarray:
    """First term of Eq. (v_emb): J_{12} = g^{13}_{24} D_{34} = (1 2|3 4) D_{34}."""
    return np.einsum("mnls,ls->mn", eri, D)


def exchange(eri: np.ndarray, gamma: np.ndarray) -> np.ndarray:
    """Second term of Eq. (v_emb): K_{12} = g^{13}_{42} gamma_{34} = (1 4|3 2) gamma_{34}."""
    return np.einsum("adcb,cd->ab", eri, gamma)


def transform4(eri: np.ndarray, C1, C2, C3, C4) -> np.ndarray:
    """(p q|r s) = sum C1[mu,p] C2[nu,q] C3[lam,r] C4[sig,s] (mu nu|lam sig)."""
    t = np.einsum("mnls,mp->pnls", eri, C1)
    t = np.einsum("pnls,nq->pqls", t, C2)
    t = np.einsum("pqls,lr->pqrs", t, C3)
    return np.einsum("pqrs,st->pqrt", t, C4)
