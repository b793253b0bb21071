"""Seeded synthetic inputs shaped like the paper's DF-LASSCF workloads.

This module only draws numbers; it holds none of the contraction arithmetic.
Both the tests (GPU path and CPU oracle alike) and the benchmark take their
inputs from here.

Recipe (shared by every workload):
  * Cholesky vectors B[P, pair], packed lower triangle, row major
    (pair(i, j) = i(i+1)/2 + j, i >= j), entries N(0, 1) * exp(-|i - j| / L),
    one independent stream per auxiliary row P, so the rows do not depend on
    how they are chunked.
  * Orbitals C = Q of the QR of a seeded N(0,1) N_ao x N_ao matrix, with the
    column signs fixed so that diag(R) > 0 (this makes Q unique).  The first
    N_occ columns are the doubly occupied orbitals, the next N_ac the active
    ones; all N_ao columns form the MO space p.
  * h: symmetric N(0,1) matrix (A + A^T)/2.  Gamma: an N(0,1) N_ac^4 tensor
    averaged over the 8 index permutations of a real 2-body density.
    kappa: 0.01 * N(0,1) N_mo x N_mo.

Streams: numpy ``default_rng(SeedSequence([seed, stream, index...]))`` with
stream 0 = B rows, 1 = C, 2 = h, 3 = Gamma, 4 = kappa, 5 = per-fragment
densities, 6 = finite-difference directions.

For the paper-scale workload (B is 27.7 GB) drawing B on the host is slow, so
``device_cholesky_vectors`` draws the same distribution on the GPU with
torch's counter-based generator; those values are not the host stream's, and
any check against the oracle copies the drawn values back.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["Workload", "WORKLOADS", "npair", "cholesky_vectors", "orbitals",
           "symmetric_matrix", "two_body_density", "kappa", "fragment_densities", "coulomb_metric",
           "device_cholesky_vectors", "directions"]


def npair(nao: int) -> int:
    return nao * (nao + 1) // 2


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def _envelope(nao: int, L: float) -> np.ndarray:
    il, jl = np.tril_indices(nao)
    return np.exp(-np.abs(il - jl).astype(np.float64) / float(L))


def cholesky_vectors(naux: int, nao: int, L: float, seed: int = 0, p0: int = 0) -> np.ndarray:
    """Rows P in [p0, p0 + naux) of the packed synthetic B, shape (naux, npair)."""
    env = _envelope(nao, L)
    out = np.empty((naux, env.size))
    for r in range(naux):
        out[r] = _rng(seed, 0, p0 + r).standard_normal(env.size)
        out[r] *= env
    return out


def orbitals(nao: int, seed: int = 0) -> np.ndarray:
    """Orthonormal N_ao x N_ao matrix with unique signs (diag(R) > 0)."""
    A = _rng(seed, 1).standard_normal((nao, nao))
    Q, R = np.linalg.qr(A)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return np.ascontiguousarray(Q * s)


def symmetric_matrix(n: int, seed: int = 0) -> np.ndarray:
    A = _rng(seed, 2).standard_normal((n, n))
    return (A + A.T) / 2


def two_body_density(nac: int, seed: int = 0) -> np.ndarray:
    """Random real N_ac^4 tensor with the 8-fold permutational symmetry of (uv|wx)."""
    G = _rng(seed, 3).standard_normal((nac,) * 4)
    perms = ["uvwx", "vuwx", "uvxw", "vuxw", "wxuv", "xwuv", "wxvu", "xwvu"]
    return sum(np.einsum("uvwx->" + p, G) for p in perms) / 8.0


def kappa(nmo: int, seed: int = 0, scale: float = 0.01) -> np.ndarray:
    return scale * _rng(seed, 4).standard_normal((nmo, nmo))


def fragment_densities(nemb: int, nocc: int, ndm: int, frag: int, seed: int = 0) -> np.ndarray:
    """ndm orthonormal factors C_k (nemb x nocc): thin-QR Q of seeded N(0,1) matrices."""
    out = np.empty((ndm, nemb, nocc))
    for k in range(ndm):
        A = _rng(seed, 5, frag, k).standard_normal((nemb, nocc))
        Q, R = np.linalg.qr(A)
        s = np.sign(np.diag(R))
        s[s == 0] = 1.0
        out[k] = Q * s
    return out


def coulomb_metric(naux: int, cond: float = 1e6, seed: int = 0) -> np.ndarray:
    """Symmetric positive definite N_aux x N_aux stand-in for the metric (P|Q): a seeded random
    orthogonal basis with eigenvalues spread geometrically from 1 down to 1/cond."""
    Q = np.linalg.qr(_rng(seed, 7).standard_normal((naux, naux)))[0]
    A = (Q * np.geomspace(1.0, 1.0 / cond, naux)) @ Q.T
    return (A + A.T) * 0.5


def directions(n_dir: int, shape, seed: int = 0) -> np.ndarray:
    """Unit-norm random directions (for finite-difference checks)."""
    A = _rng(seed, 6).standard_normal((n_dir,) + tuple(shape))
    return A / np.linalg.norm(A.reshape(n_dir, -1), axis=1).reshape((n_dir,) + (1,) * len(shape))


def device_cholesky_vectors(naux: int, nao: int, L: float, seed: int = 0, device="cuda",
                            rows_per_draw: int = 256):
    """Packed B drawn on the GPU (torch's Philox stream), same distribution as the host recipe."""
    import torch
    env = torch.from_numpy(_envelope(nao, L)).to(device)
    out = torch.empty((naux, env.numel()), dtype=torch.float64, device=device)
    g = torch.Generator(device=device)
    for r0 in range(0, naux, rows_per_draw):
        r1 = min(naux, r0 + rows_per_draw)
        g.manual_seed(int(seed) * 1_000_003 + r0)
        torch.randn((r1 - r0, env.numel()), generator=g, dtype=torch.float64, device=device,
                    out=out[r0:r1])
        out[r0:r1].mul_(env)
    return out


@dataclass(frozen=True)
class Workload:
    name: str
    nao: int
    naux: int
    nocc: int
    nac: int
    L: float
    seed: int = 0

    @property
    def nmo(self) -> int:
        return self.nao


# The workloads the benchmark and the parity tests use.  The decay length of the
# paper-scale case is not stated with it; it reuses the medium case's 40.
WORKLOADS = {
    "tiny": Workload("tiny", nao=120, naux=480, nocc=30, nac=8, L=20.0),
    "medium": Workload("medium", nao=600, naux=2400, nocc=150, nac=20, L=40.0),
    "paper": Workload("paper", nao=1200, naux=4800, nocc=300, nac=40, L=40.0),
}


@dataclass(frozen=True)
class Fragment:
    """One embedding-space subproblem of the batched fragment workload."""
    index: int
    nemb: int
    nac: int
    ndm: int = 64
    L: float = 20.0

    @property
    def naux(self) -> int:
        return 4 * self.nemb

    @property
    def nocc(self) -> int:
        return self.nemb // 4


# Eight uneven fragment subproblems (N_emb 80 .. 400, N_aux = 4 N_emb, 4-8 active orbitals,
# 64 densities of N_emb / 4 occupied columns each), the shapes of the fragment CASSCFs.
FRAGMENTS = tuple(Fragment(i, n, a) for i, (n, a) in enumerate(
    [(80, 4), (120, 4), (160, 6), (200, 6), (240, 6), (280, 8), (340, 8), (400, 8)]))


def fragment_problem(f: Fragment, seed: int = 0, ndm: int | None = None):
    """Host inputs of fragment f: packed B [naux, npair], ndm density factors [ndm, nemb, nocc] and
    orbitals C [nemb, nemb]; the active block is C[:, nocc:nocc + nac], the p space all of C."""
    ndm = f.ndm if ndm is None else ndm
    B = cholesky_vectors(f.naux, f.nemb, f.L, seed=seed * 101 + f.index)
    Cd = fragment_densities(f.nemb, f.nocc, ndm, f.index, seed=seed)
    C = orbitals(f.nemb, seed=seed * 101 + f.index)
    return B, Cd, C
