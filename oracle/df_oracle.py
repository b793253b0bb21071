"""Plain FP64 CPU oracle for the density-fitted contractions of DF-LASSCF.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link this module; only the tests, the
package's ``smoke()`` self-check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the GPU path.

Everything here is written as the plain definition of the quantity in the
paper (Agarawal et al., "Enabling Multireference Calculations on Multi-Metallic
Systems with Graphic Processing Units", arXiv 2505.03755), in float64 NumPy,
one auxiliary index P at a time (or in small chunks of P so that memory stays
bounded), with library matrix products as the only building blocks.

Conventions (see the Theory section of the paper):
  * Density fitting, Eq. (cholesky): (mu nu|lam sig) = sum_P b^P_{mu nu} b^P_{lam sig}.
  * The Cholesky vectors are stored packed, lower triangle, row major:
    B[P, i*(i+1)//2 + j] = b^P_{ij} for i >= j (Sec. "Analysis of computational
    bottlenecks": the vectors are kept in triangular form of size
    N_aux N_ao (N_ao+1)/2).
  * Densities are given by a factor:  D = C diag(w) C^T (w = 1 by default).

Parity pins: every function below is pinned by tests in ``tests/test_oracle_*``
against a brute-force 4-index ERI, closed forms, hand-derived golden values and
invariants.  Parity unpinned: none.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "npair", "unpack", "iter_unpacked", "density", "half_transform",
    "second_transform", "jvec", "coulomb", "exchange", "exchange_paper_route",
    "jk", "jk_many", "mo_vectors", "active_eri", "papa", "papa_full", "ppaa", "fsum_dot",
]

DEFAULT_CHUNK = 240   # the P-block size the paper keeps (PySCF default)


def npair(nao: int) -> int:
    """Number of packed pairs of an N_ao x N_ao symmetric matrix."""
    return nao * (nao + 1) // 2


def _unpack_rows(flat: np.ndarray, out: np.ndarray, nao: int) -> None:
    """Fill out[k] (zeros on entry) with the symmetric matrix of packed row flat[k]."""
    for i in range(nao):                # row i holds (i, 0), (i, 1), ..., (i, i)
        out[:, i, :i + 1] = flat[:, i * (i + 1) // 2:i * (i + 1) // 2 + i + 1]
    d = np.arange(nao)
    for m in out:                       # lower + its transpose (upper zero): the mirror; the
        m += m.T.copy()                 # doubled diagonal is halved again (both exact)
        m[d, d] *= 0.5


_POOL: ThreadPoolExecutor | None = None


def _pool() -> ThreadPoolExecutor:
    global _POOL
    if _POOL is None:
        _POOL = ThreadPoolExecutor(max(1, min(8, len(os.sched_getaffinity(0)))))
    return _POOL


def unpack(bp: np.ndarray, nao: int) -> np.ndarray:
    """Packed lower-triangular row(s) -> dense symmetric matrix/matrices.

    bp has shape (..., npair); entry i*(i+1)//2 + j holds element (i, j), i >= j.  Large batches
    are unpacked by several threads, each on its own rows (a copy: the values do not depend on it).
    """
    bp = np.asarray(bp, dtype=np.float64)
    if bp.shape[-1] != npair(nao):
        raise ValueError("packed length does not match nao")
    lead = bp.shape[:-1]
    flat = bp.reshape((-1, bp.shape[-1]))
    out = np.zeros((flat.shape[0], nao, nao))
    n = flat.shape[0]
    nw = min(_pool()._max_workers, n) if n * nao * nao >= (1 << 24) else 1
    if nw > 1:
        cuts = [n * k // nw for k in range(nw + 1)]
        list(_pool().map(lambda k: _unpack_rows(flat[cuts[k]:cuts[k + 1]], out[cuts[k]:cuts[k + 1]], nao),
                         range(nw)))
    else:
        _unpack_rows(flat, out, nao)
    return out.reshape(lead + (nao, nao))


def iter_unpacked(B: np.ndarray, nao: int, chunk: int = DEFAULT_CHUNK):
    """Yield (P0, P1, dense B_P for P in [P0, P1)) over the auxiliary index."""
    naux = B.shape[0]
    for p0 in range(0, naux, chunk):
        p1 = min(naux, p0 + chunk)
        yield p0, p1, unpack(B[p0:p1], nao)


def density(C: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """D = C diag(w) C^T (the factorised density)."""
    C = np.asarray(C, dtype=np.float64)
    if w is None:
        return C @ C.T
    return (C * np.asarray(w, dtype=np.float64)) @ C.T


def half_transform(B: np.ndarray, nao: int, C: np.ndarray, chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """Eq. (ao2mo_1): X[P, mu, c] = sum_nu b^P_{mu nu} C[nu, c].

    The untransformed AO index comes first, as in b^P_{e_2 p_1}.
    """
    C = np.asarray(C, dtype=np.float64)
    X = np.empty((B.shape[0], nao, C.shape[1]))
    for p0, p1, Bd in iter_unpacked(B, nao, chunk):
        X[p0:p1] = np.matmul(Bd, C)
    return X


def second_transform(X: np.ndarray, C2: np.ndarray) -> np.ndarray:
    """Eq. (ao2mo_2): Y[P, p, c] = sum_mu C2[mu, p] X[P, mu, c]."""
    return np.matmul(np.asarray(C2, dtype=np.float64).T[None], X)


def jvec(B: np.ndarray, nao: int, D: np.ndarray, chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """Eq. (J_1): v_P = sum_{ij} b^P_{ij} D_{ij}."""
    v = np.empty(B.shape[0])
    for p0, p1, Bd in iter_unpacked(B, nao, chunk):
        v[p0:p1] = np.einsum("pij,ij->p", Bd, D)
    return v


def coulomb(B: np.ndarray, nao: int, v: np.ndarray, chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """Eq. (J_2): J_{ij} = sum_P v_P b^P_{ij}."""
    J = np.zeros((nao, nao))
    for p0, p1, Bd in iter_unpacked(B, nao, chunk):
        J += np.tensordot(v[p0:p1], Bd, axes=(0, 0))
    return J


def exchange(B: np.ndarray, nao: int, C: np.ndarray, w: np.ndarray | None = None,
             chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """Factored exchange: K = sum_P (B_P C) diag(w) (B_P C)^T.

    With gamma = C diag(w) C^T this equals Eqs. (K_1)-(K_2) of the paper.
    """
    C = np.asarray(C, dtype=np.float64)
    wv = np.ones(C.shape[1]) if w is None else np.asarray(w, dtype=np.float64)
    K = np.zeros((nao, nao))
    for p0, p1, Bd in iter_unpacked(B, nao, chunk):
        X = np.matmul(Bd, C)                       # (chunk, nao, nocc)
        K += np.tensordot(X * wv, X, axes=([0, 2], [0, 2]))
    return K


def exchange_paper_route(B: np.ndarray, nao: int, gamma: np.ndarray,
                         chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """Eqs. (K_1)-(K_2) as written: v^P_{ik} = b^P_{ij} gamma_{jk};  K_{ij} = v^P_{ik} b^P_{jk}."""
    gamma = np.asarray(gamma, dtype=np.float64)
    K = np.zeros((nao, nao))
    for p0, p1, Bd in iter_unpacked(B, nao, chunk):
        V = np.matmul(Bd, gamma)                   # v^P_{ik}
        K += np.einsum("pik,pjk->ij", V, Bd)
    return K


def jk(B: np.ndarray, nao: int, Cocc: np.ndarray, w: np.ndarray | None = None,
       chunk: int = DEFAULT_CHUNK):
    """One "JK call" for one density D = Cocc diag(w) Cocc^T: returns (J, K, v).

    J = J[D] and K = K[D]; no spin factor is applied.
    """
    D = density(Cocc, w)
    v = jvec(B, nao, D, chunk)
    J = coulomb(B, nao, v, chunk)
    K = exchange(B, nao, Cocc, w, chunk)
    return J, K, v


def jk_many(B: np.ndarray, nao: int, Cs, chunk: int = DEFAULT_CHUNK):
    """The JK call of many densities D_k = C_k C_k^T at once, each b^P unpacked once: returns
    (J, K, v) with J, K [ndm, nao, nao], v [ndm, naux], each density's as in jk() (Eqs. J_1, J_2
    and the factored K)."""
    Cs = [np.asarray(C, dtype=np.float64) for C in Cs]
    ndm, naux = len(Cs), B.shape[0]
    Ds = [C @ C.T for C in Cs]
    J = np.zeros((ndm, nao, nao))
    K = np.zeros((ndm, nao, nao))
    v = np.empty((ndm, naux))
    for p0, p1, Bd in iter_unpacked(B, nao, chunk):
        for k in range(ndm):
            v[k, p0:p1] = np.einsum("pij,ij->p", Bd, Ds[k])      # Eq. (J_1)
            J[k] += np.tensordot(v[k, p0:p1], Bd, axes=(0, 0))    # Eq. (J_2)
            X = np.matmul(Bd, Cs[k])                              # b^P C_k
            K[k] += np.tensordot(X, X, axes=([0, 2], [0, 2]))     # sum_P (b^P C_k)(b^P C_k)^T
    return J, K, v


def mo_vectors(B: np.ndarray, nao: int, Cl: np.ndarray, Cr: np.ndarray,
               chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """Eqs. (ao2mo_1)-(ao2mo_2) with two coefficient sets: b^P_{pu} = (Cl^T B_P Cr)_{pu}."""
    Cl = np.asarray(Cl, dtype=np.float64)
    Cr = np.asarray(Cr, dtype=np.float64)
    out = np.empty((B.shape[0], Cl.shape[1], Cr.shape[1]))
    for p0, p1, Bd in iter_unpacked(B, nao, chunk):
        out[p0:p1] = np.matmul(Cl.T[None], np.matmul(Bd, Cr))
    return out


def active_eri(B: np.ndarray, nao: int, Cact: np.ndarray, chunk: int = DEFAULT_CHUNK):
    """Active-space ERIs (uv|wx) = sum_P b^P_{uv} b^P_{wx}; returns (eri, b_uv)."""
    buv = mo_vectors(B, nao, Cact, Cact, chunk)
    return np.tensordot(buv, buv, axes=(0, 0)), buv


def papa(B: np.ndarray, nao: int, Cp: np.ndarray, Cact: np.ndarray, chunk: int = DEFAULT_CHUNK):
    """The gradient pattern (p u|v w) = sum_P b^P_{pu} b^P_{vw}, shape (np, nac, nac, nac).

    This is the index pattern g^{p a}_{a a} the LASSCF orbital gradient needs
    once per cycle (Eq. MO_conv); it is the q-in-active slice of Eq. (papa).
    """
    bpu = mo_vectors(B, nao, Cp, Cact, chunk)
    bvw = mo_vectors(B, nao, Cact, Cact, chunk)
    return np.tensordot(bpu, bvw, axes=(0, 0))


def papa_full(B: np.ndarray, nao: int, Cp: np.ndarray, Cact: np.ndarray, Cq: np.ndarray,
              chunk: int = DEFAULT_CHUNK):
    """Eq. (papa): (p u|q v) = sum_P b^P_{pu} b^P_{qv}, shape (np, nac, nq, nac)."""
    bpu = mo_vectors(B, nao, Cp, Cact, chunk)
    bqv = mo_vectors(B, nao, Cq, Cact, chunk)
    return np.tensordot(bpu, bqv, axes=(0, 0))


def ppaa(B: np.ndarray, nao: int, Cp: np.ndarray, Cq: np.ndarray, Cact: np.ndarray,
         chunk: int = DEFAULT_CHUNK):
    """Eq. (ppaa): (p q|u v) = sum_P b^P_{pq} b^P_{uv}, shape (np, nq, nac, nac)."""
    bpq = mo_vectors(B, nao, Cp, Cq, chunk)
    buv = mo_vectors(B, nao, Cact, Cact, chunk)
    return np.tensordot(bpq, buv, axes=(0, 0))


def fsum_dot(a: np.ndarray, b: np.ndarray) -> float:
    """sum_i a_i b_i with the products rounded once each and summed exactly (math.fsum)."""
    return math.fsum((np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64)).ravel().tolist())
