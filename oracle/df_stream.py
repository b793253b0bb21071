"""One pass of the FP64 oracle over the auxiliary index, for workloads whose unpacked B does not fit.

TEST INFRASTRUCTURE ONLY (see ``oracle/df_oracle.py``); shares no code with the GPU path.

Every output of the differentiable DF step is a sum over the auxiliary index P of terms that
involve b^P alone (Eq. cholesky), so the oracle can take the packed rows of B block by block,
unpack each block, and add up the definitions below.  The caller hands the blocks in P order
(``chunks`` yields (P0, packed rows of P0 .. P0 + n - 1)), e.g. copied from device memory one
block at a time.  With C_occ, C_act the occupied and active columns of C and D = C_occ C_occ^T:

  v_P        = sum_{ij} b^P_ij D_ij                                  Eq. (J_1)
  J          = sum_P v_P b^P                                         Eq. (J_2)
  X_P        = b^P C_occ  (the half transform, Eq. ao2mo_1)
  K C_occ    = sum_P X_P (X_P^T C_occ)                               Eqs. (K_1)-(K_2), gamma = D
  tr(D K)    = sum_P || C_occ^T b^P C_occ ||_F^2
  K (full, optional) = sum_P X_P X_P^T, or rows of it: K[i, :] = sum_P X_P[i, :] X_P^T
  b_uv       = C_act^T b^P C_act,  (uv|wx) = sum_P b^P_uv b^P_wx      Eq. (ao2mo_2), the (aa|aa) block
  (pu|vw)    = sum_P b^P_pu b^P_vw for the requested rows p           the g^{pa}_{aa} pattern
  E          = tr(D h) + 1/2 tr(D J) - 1/4 tr(D K) + 1/2 sum (uv|wx) Gamma
  dE/dC_occ  = 2 (h + J - K/2) C_occ
  dE/dC_act  = 2 sum_P (b^P C_act) Z_P,  Z_P[u,v] = sum_wx Gamma_uvwx b^P_wx
(the energy and its derivatives as in ``oracle/df_grad.py``).  Scalar sums use math.fsum.
Parity pins: tests/test_oracle_stream.py (the brute-force 4-index route, closed forms, and
independence from the block size).  Parity unpinned: none.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import df_oracle as O


def host_chunks(B: np.ndarray, chunk: int = O.DEFAULT_CHUNK):
    """Blocks of rows of a packed B held in host memory."""
    for p0 in range(0, B.shape[0], chunk):
        yield p0, B[p0:p0 + chunk]


def step_pass(chunks, naux: int, nao: int, C: np.ndarray, nocc: int, nac: int, h: np.ndarray,
              Gamma: np.ndarray, p_rows=(), want_K: bool = False, k_rows=()) -> dict:
    """The quantities listed in the module docstring from one pass over the blocks of B.

    Returns a dict with v [naux], J, KC = K C_occ [nao, nocc], K (with want_K), K_rows = K[k_rows, :]
    [len(k_rows), nao], buv [naux, nac, nac],
    eri [nac]^4, papa_rows [len(p_rows), nac, nac, nac] ((pu|vw) for p in p_rows), the energy terms
    E_h, E_J, E_K, E_eri and E, and G = dE/dC [nao, nmo] (columns past nocc + nac zero)."""
    C = np.asarray(C, dtype=np.float64)
    Cocc, Cact = C[:, :nocc], C[:, nocc:nocc + nac]
    Cp = C[:, list(p_rows)]
    D = Cocc @ Cocc.T
    Gm = Gamma.reshape(nac * nac, nac * nac)
    v = np.empty(naux)
    J = np.zeros((nao, nao))
    KC = np.zeros((nao, nocc))
    K = np.zeros((nao, nao)) if want_K else None
    kr = list(k_rows)
    Kr = np.zeros((len(kr), nao))
    buv = np.empty((naux, nac, nac))
    bpu = np.empty((naux, len(p_rows), nac))
    Gact = np.zeros((nao, nac))
    trDK = []
    seen = 0
    for p0, rows in chunks:
        n = rows.shape[0]
        if p0 != seen:
            raise ValueError("blocks of B must come in P order without gaps")
        Bd = O.unpack(rows, nao)                                  # b^P, [n, nao, nao]
        vb = np.einsum("pij,ij->p", Bd, D)                         # Eq. (J_1)
        v[p0:p0 + n] = vb
        J += np.tensordot(vb, Bd, axes=(0, 0))                     # Eq. (J_2)
        X = np.tensordot(Bd, Cocc, axes=(2, 0))                   # X_P = b^P C_occ, [n, nao, nocc]
        M = np.tensordot(Cocc, X, axes=(0, 1)).transpose(1, 0, 2)  # M_P = C_occ^T b^P C_occ
        KC += np.tensordot(X, M, axes=([0, 2], [0, 2]))           # sum_P X_P M_P^T = sum_P X_P X_P^T C_occ
        trDK.extend((M * M).sum(axis=(1, 2)).tolist())
        if want_K:
            K += np.tensordot(X, X, axes=([0, 2], [0, 2]))
        if kr:
            Kr += np.tensordot(X[:, kr, :], X, axes=([0, 2], [0, 2]))   # sum_P X_P[i, :] X_P^T
        Xa = np.tensordot(Bd, Cact, axes=(2, 0))                  # b^P C_act
        bu = np.tensordot(Cact, Xa, axes=(0, 1)).transpose(1, 0, 2)   # b^P_uv
        buv[p0:p0 + n] = bu
        bpu[p0:p0 + n] = np.tensordot(Cp, Xa, axes=(0, 1)).transpose(1, 0, 2)   # b^P_pu, p in p_rows
        Z = (bu.reshape(n, nac * nac) @ Gm.T).reshape(n, nac, nac)  # Z_P[u,v] = sum_wx Gamma_uvwx b_wx
        Gact += 2.0 * np.einsum("pmv,pvu->mu", Xa, Z)
        seen += n
    if seen != naux:
        raise ValueError(f"the blocks cover {seen} of {naux} auxiliary rows")
    eri = np.tensordot(buv, buv, axes=(0, 0))
    papa_rows = np.tensordot(bpu, buv, axes=(0, 0))
    E_h = O.fsum_dot(D, h)
    E_J = 0.5 * O.fsum_dot(D, J)
    E_K = -0.25 * math.fsum(trDK)
    E_eri = 0.5 * O.fsum_dot(eri, Gamma)
    G = np.zeros_like(C)
    G[:, :nocc] = 2.0 * ((h + J) @ Cocc - 0.5 * KC)
    G[:, nocc:nocc + nac] = Gact
    out = {"v": v, "J": J, "KC": KC, "buv": buv, "eri": eri, "papa_rows": papa_rows, "E_h": E_h, "E_J": E_J,
           "E_K": E_K, "E_eri": E_eri, "E": math.fsum([E_h, E_J, E_K, E_eri]), "G": G}
    if want_K:
        out["K"] = K
    if kr:
        out["K_rows"] = Kr
    return out


def orbital_gradient_from_G(C0: np.ndarray, kappa: np.ndarray, G: np.ndarray) -> np.ndarray:
    """dE/dkappa for C = C0 exp(kappa - kappa^T) given G = dE/dC at that C: W - W^T with
    W = L_exp(-(kappa - kappa^T), C0^T G) (W = C0^T G at kappa = 0), as in df_grad.orbital_gradient."""
    R = kappa - kappa.T
    A = C0.T @ G
    W = A if not np.any(R) else scipy.linalg.expm_frechet(-R, A, compute_expm=False)
    return W - W.T
