"""FP64 CPU oracle for the differentiable DF step (energy, gradients, vector-Jacobian products).

TEST INFRASTRUCTURE ONLY (see ``oracle/df_oracle.py``); shares no code with the GPU path.

The model energy of the differentiable workload is

    E(kappa) = tr(D h) + 1/2 tr(D J[D]) - 1/4 tr(D K[D]) + 1/2 sum_{uvwx} (uv|wx) Gamma_{uvwx}

with C(kappa) = C0 exp(kappa - kappa^T), D = C_occ C_occ^T from the first N_occ columns of
C(kappa), (uv|wx) over the next N_ac columns, h symmetric and Gamma with the 8-fold symmetry of a
real two-body density.  J and K are the Coulomb and exchange builds of Eqs. (J_1)-(K_2) and
(uv|wx) the active-space ERIs, all through the density-fitting factorisation of Eq. (cholesky).

Derivatives (derived here from those definitions):
  dE/dC_occ = 2 (h + J - K/2) C_occ
  dE/dC_act = 2 sum_P (b^P C_act) Z_P,  Z_P[u,v] = sum_wx Gamma_uvwx (C_act^T b^P C_act)_wx
  dE/dkappa = W - W^T,  W = L_exp(-(kappa - kappa^T), C0^T G)   (adjoint of the Frechet
              derivative of exp; W = C0^T G at kappa = 0), G = [dE/dC_occ | dE/dC_act | 0].
The vector-Jacobian product of (J, K, eri) as functions of (C_occ, C_act) for cotangents
(gJ, gK, geri):
  dC_occ = 2 M C_occ + sum_P b^P S b^P C_occ,  M = sum_P <b^P, gJ> b^P,  S = gK + gK^T
  dC_act = sum_P (b^P C_act)(Z_P + Z_P^T),     Z_P[u,v] = sum_wx (geri_uvwx + geri_wxuv) b^P_wx
Final scalar reductions use math.fsum.  Parity pins: tests/test_oracle_grad.py (central finite
differences, the closed form at kappa = 0, redundant-rotation blocks, VJP against finite
differences of the forward).  Parity unpinned: none.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import df_oracle as O


def rotate(C0: np.ndarray, kappa: np.ndarray) -> np.ndarray:
    """C(kappa) = C0 exp(kappa - kappa^T)."""
    return C0 @ scipy.linalg.expm(kappa - kappa.T)


def energy(B, nao, C, nocc, nac, h, Gamma) -> float:
    """E for orbitals C (columns: occupied, active, rest)."""
    Cocc, Cact = C[:, :nocc], C[:, nocc:nocc + nac]
    D = Cocc @ Cocc.T
    J, K, _ = O.jk(B, nao, Cocc)
    eri, _ = O.active_eri(B, nao, Cact)
    terms = [O.fsum_dot(D, h), 0.5 * O.fsum_dot(D, J), -0.25 * O.fsum_dot(D, K), 0.5 * O.fsum_dot(eri, Gamma)]
    return math.fsum(terms)


def energy_terms(B, nao, C, nocc, nac, h, Gamma) -> dict:
    Cocc, Cact = C[:, :nocc], C[:, nocc:nocc + nac]
    D = Cocc @ Cocc.T
    J, K, v = O.jk(B, nao, Cocc)
    eri, _ = O.active_eri(B, nao, Cact)
    return {"h": O.fsum_dot(D, h), "J": 0.5 * O.fsum_dot(D, J), "K": -0.25 * O.fsum_dot(D, K),
            "eri": 0.5 * O.fsum_dot(eri, Gamma), "J_from_v": 0.5 * math.fsum((v * v).tolist())}


def energy_gradient_C(B, nao, C, nocc, nac, h, Gamma) -> np.ndarray:
    """G = dE/dC, shape (nao, nmo); columns past nocc + nac are zero."""
    Cocc, Cact = C[:, :nocc], C[:, nocc:nocc + nac]
    J, K, _ = O.jk(B, nao, Cocc)
    G = np.zeros_like(C)
    G[:, :nocc] = 2.0 * (h + J - 0.5 * K) @ Cocc
    if nac:
        buv = O.mo_vectors(B, nao, Cact, Cact)                  # b^P_uv
        Gm = Gamma.reshape(nac * nac, nac * nac)
        Z = (buv.reshape(-1, nac * nac) @ Gm.T).reshape(-1, nac, nac)   # Z_P[uv] = sum_wx Gamma_uvwx b_wx
        X = O.half_transform(B, nao, Cact)                      # b^P C_act
        G[:, nocc:nocc + nac] = 2.0 * np.einsum("pmv,pvu->mu", X, Z)
    return G


def orbital_gradient(B, nao, C0, kappa, nocc, nac, h, Gamma) -> np.ndarray:
    """dE/dkappa at kappa (the full N_mo x N_mo matrix; antisymmetric)."""
    R = kappa - kappa.T
    C = C0 @ scipy.linalg.expm(R)
    A = C0.T @ energy_gradient_C(B, nao, C, nocc, nac, h, Gamma)
    if not np.any(R):
        W = A
    else:
        W = scipy.linalg.expm_frechet(-R, A, compute_expm=False)
    return W - W.T


def forward(B, nao, Cocc, Cact):
    """(J, K, eri) as functions of (C_occ, C_act)."""
    J, K, _ = O.jk(B, nao, Cocc)
    eri, _ = O.active_eri(B, nao, Cact)
    return J, K, eri


def step_vjp(B, nao, Cocc, Cact, gJ, gK, geri):
    """Vector-Jacobian product of forward() for cotangents (gJ, gK, geri); returns (dCocc, dCact)."""
    nac = Cact.shape[1]
    dCocc = np.zeros_like(Cocc)
    dCact = np.zeros_like(Cact)
    if gJ is not None:
        u = O.jvec(B, nao, gJ)                     # <b^P, gJ>
        M = O.coulomb(B, nao, u)                   # sum_P u_P b^P
        dCocc += 2.0 * M @ Cocc
    if gK is not None:
        S = gK + gK.T
        dCocc += O.exchange_paper_route(B, nao, S) @ Cocc     # sum_P b^P S b^P C_occ
    if geri is not None and nac:
        G2 = geri.reshape(nac * nac, nac * nac)
        Gs = G2 + G2.T
        buv = O.mo_vectors(B, nao, Cact, Cact)
        Z = (buv.reshape(-1, nac * nac) @ Gs.T).reshape(-1, nac, nac)
        X = O.half_transform(B, nao, Cact)
        dCact += np.einsum("pmv,pvu->mu", X, Z + Z.transpose(0, 2, 1))
    return dCocc, dCact
