"""Plain FP64 CPU oracle for forming the Cholesky vectors b^P.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this module; only the tests, the package's smoke() self-check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the GPU path.

Eq. (cholesky) writes the density-fitted ERIs as
    (mu nu|lam sig) ~ (mu nu|P) (P|Q)^-1 (Q|lam sig) = sum_P b^P_{mu nu} b^P_{lam sig}.
With the Coulomb metric factored as (P|Q) = L L^T (Cholesky, L lower triangular
with a positive diagonal), b = L^-1 E, E[Q, pair] = (Q|mu nu), satisfies it:
b^T b = E^T L^-T L^-1 E = E^T (P|Q)^-1 E.  The pairs are packed as everywhere
else: pair(i, j) = i(i+1)/2 + j for i >= j.

The same vectors in another orbital basis (the embedding orbitals of a fragment,
whose effective potentials are built exactly as in the AO basis; Sec.
"Calculation of effective potentials") are b^P_{ef} = (M^T b^P M)_{ef} for the
orbital coefficients M [nao][nemb], packed the same way.

Parity pins (tests/test_oracle_build.py): b^T b against (mu nu|P)(P|Q)^-1(Q|lam sig)
formed with a general linear solve; the identity and diagonal metrics in closed
form; a hand-worked 2 x 2 example; the embedded vectors against the brute-force
4-index transform.  Parity unpinned: none.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .df_oracle import mo_vectors, npair

__all__ = ["metric_cholesky", "cholesky_vectors", "embed"]


def metric_cholesky(metric: np.ndarray) -> np.ndarray:
    """L with (P|Q) = L L^T, lower triangular, positive diagonal (library Cholesky)."""
    return np.linalg.cholesky(np.asarray(metric, dtype=np.float64))


def cholesky_vectors(metric: np.ndarray, eri3: np.ndarray) -> np.ndarray:
    """b = L^-1 E by forward substitution: B[P, pair] with E[Q, pair] = (Q|mu nu)."""
    L = metric_cholesky(metric)
    return scipy.linalg.solve_triangular(L, np.asarray(eri3, dtype=np.float64), lower=True)


def embed(B: np.ndarray, nao: int, M: np.ndarray) -> np.ndarray:
    """Packed b^P in the basis of the columns of M: Be[P, pair(e, f)] = (M^T b^P M)_{ef}."""
    M = np.asarray(M, dtype=np.float64)
    ne = M.shape[1]
    Y = mo_vectors(B, nao, M, M)
    e, f = np.tril_indices(ne)
    out = np.empty((B.shape[0], npair(ne)))
    out[:] = Y[:, e, f]
    return out
