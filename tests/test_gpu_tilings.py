"""The tilings of the packed products against the FP64 oracle.

The half transform X_P = b^P C (Eq. ao2mo_1) and the adjoint's sum_P b^P Y_P are tiled in pieces
by their shape: 128 x 128 tiles on whole 128-row bands, a one-tile remainder of the columns on
one of five 128-row tile shapes (both in one launch), the rows past the last whole band on
64 x 176 tiles, or 64 x 176 / 128 x 96 / 128 x 48 tiles for the whole.  The shapes below take
every combination of pieces; for each the half transform (plain and accumulated onto what the
output holds), the step's J-vector from the half transform's epilogue and J (Eqs. J_1, J_2), K,
and the adjoint for random cotangents are compared with the oracle at the FP64 bar (1e-10
normwise and max relative).  N_aux is small and odd so the P splits are ragged.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import df_grad as G
from oracle import df_oracle as O
from paper_2505_03755_amd import dfmi, synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def close(gpu, ref, what, tol=TOL):
    g = gpu.detach().cpu().numpy()
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, (what, g.shape, r.shape)
    d = g - r
    assert np.linalg.norm(d) <= tol * np.linalg.norm(r), (what, np.linalg.norm(d) / np.linalg.norm(r))
    assert np.abs(d).max() <= tol * np.abs(r).max(), (what, np.abs(d).max() / np.abs(r).max())


# (nao, N_occ + N_ac columns) -> pieces of the half transform:
#   (130, 150): 128 x 128 + 128 x 48 remainder, rows 128-129 on 64 x 176 tiles
#   (130, 180): 128 x 128 + 128 x 64 remainder on all rows
#   (130, 200): 128 x 128 + 128 x 96 remainder
#   (130, 230): 128 x 128 + a second 128 x 128 column tile as the remainder
#   (130, 340): 128 x 128 (two column tiles) + 128 x 96, rows 128-129 on 64 x 176 tiles
#   (130, 100), (130, 70), (130, 64): one 128-row tile shape for the whole
#   (200, 150): 128 x 128 + 128 x 48 on all 200 rows
#   (130, 130): 128 x 48 tiles on one row of waves
SHAPES = [(130, 150), (130, 180), (130, 200), (130, 230), (130, 340), (130, 100), (130, 70), (130, 64),
          (200, 150), (130, 130)]
NAUX = 13


@pytest.mark.parametrize("nao,ncol", SHAPES)
def test_half_transform_tilings(nao, ncol):
    nac = 9
    nocc = ncol - nac
    B = synth.cholesky_vectors(NAUX, nao, 10.0, seed=nao + ncol)
    C = synth.orbitals(nao, seed=ncol)
    Cc = np.tile(C, (1, -(-ncol // nao)))[:, :ncol]      # ncol columns (more than nao when ncol > nao)
    Cocc, Cact = Cc[:, :nocc], Cc[:, nocc:]
    gB = dev(B)
    X = dfmi.half_transform(gB, nao, dev(Cc))
    Xr = O.half_transform(B, nao, Cc)
    X1 = dev(np.full(Xr.shape, 0.5))
    dfmi.half_transform(gB, nao, dev(Cc), out=X1, accumulate=True)
    out = dfmi.step(gB, nao, dev(Cocc), dev(Cact), dev(C), keep_x=True)
    torch.cuda.synchronize()
    close(X, Xr, "X")
    close(X1, Xr + 0.5, "X accumulated")
    J, K, v = O.jk(B, nao, Cocc)
    close(out["v"], v, "v from the half transform's epilogue")
    close(out["J"], J, "J")
    close(out["K"], K, "K")
    rng = np.random.default_rng(nao * ncol)
    gJ, gK = rng.standard_normal((nao, nao)), rng.standard_normal((nao, nao))
    ge = rng.standard_normal((nac,) * 4)
    dCo, dCa = dfmi.step_backward(gB, nao, dev(Cocc), dev(Cact), dev(gJ), dev(gK), dev(ge), out["Xocc"], out["Xact"])
    torch.cuda.synchronize()
    ref_o, ref_a = G.step_vjp(B, nao, Cocc, Cact, gJ, gK, ge)
    close(dCo, ref_o, "dC_occ (sum_P b^P Y_P on the tilings of N_occ columns)")
    close(dCa, ref_a, "dC_act")
