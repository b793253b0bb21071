"""GPU parity of df_ppaa, (pq|uv) of Eq. (ppaa), against the FP64 oracle's definition
sum_P b^P_pq b^P_uv (which forms b^P_pq; the library goes through the AO basis instead).

The output holds the (uv) index packed, u >= v; the oracle's [p][q][u][v] is brought to that
layout here.  Bar as in the other FP64 parity tests: normwise and max-entry 1e-10.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import df_oracle as O
from paper_2505_03755_amd import dfmi, synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def packed_uv(ref):
    """[p][q][u][v] -> [pair(u, v)][p][q] with pair(u, v) = u(u+1)/2 + v, u >= v."""
    nac = ref.shape[2]
    u, v = np.tril_indices(nac)
    return np.ascontiguousarray(ref[:, :, u, v].transpose(2, 0, 1))


def close(gpu, ref, tol=TOL, what=""):
    g = gpu.detach().cpu().numpy()
    assert g.shape == ref.shape, (what, g.shape, ref.shape)
    assert np.all(np.isfinite(g)), what
    d = g - ref
    rn, rm = np.linalg.norm(ref), np.abs(ref).max(initial=0.0)
    assert np.linalg.norm(d) <= tol * rn, (what, np.linalg.norm(d) / rn)
    assert np.abs(d).max() <= tol * rm, (what, np.abs(d).max() / rm)


def rand_inputs(nao, naux, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((naux, O.npair(nao))), np.linalg.qr(rng.standard_normal((nao, nao)))[0]


@pytest.mark.parametrize("nao,naux,nac,np_,nq", [(90, 29, 5, 70, 33), (37, 130, 1, 37, 0), (65, 17, 9, 3, 0),
                                                 (129, 61, 7, 129, 100)])
def test_ppaa_ragged_against_oracle(nao, naux, nac, np_, nq):
    B, C = rand_inputs(nao, naux, seed=nao + naux)
    Cp, Cact = C[:, :np_], C[:, nao - nac:]
    Cq = C[:, 5:5 + nq] if nq else None
    out = dfmi.ppaa(dev(B), nao, dev(Cp), dev(Cact), Cq=dev(Cq) if nq else None)
    torch.cuda.synchronize()
    ref = O.ppaa(B, nao, Cp, Cq if nq else Cp, Cact)
    close(out, packed_uv(ref), what=f"ppaa {nao} {naux} {nac} {np_} {nq}")


def test_ppaa_tiny_workload():
    wl = synth.WORKLOADS["tiny"]
    B = synth.cholesky_vectors(wl.naux, wl.nao, wl.L, seed=wl.seed)
    C = synth.orbitals(wl.nao, seed=wl.seed)
    Cact = C[:, wl.nocc:wl.nocc + wl.nac]
    out = dfmi.ppaa(dev(B), wl.nao, dev(C), dev(Cact))
    torch.cuda.synchronize()
    close(out, packed_uv(O.ppaa(B, wl.nao, C, C, Cact)), what="ppaa tiny")
    # with p, q active, (pq|uv) is the active-space (wx|uv)
    eri, _ = O.active_eri(B, wl.nao, Cact)
    a = slice(wl.nocc, wl.nocc + wl.nac)
    close(out[:, a, a], packed_uv(eri), what="active block")


def test_ppaa_medium_sampled_rows():
    """Medium workload (N_ao 600, N_aux 2400, N_ac 20): all of (pq|uv) on the GPU, sampled p rows
    against the oracle (its b^P_pq for those p only)."""
    wl = synth.WORKLOADS["medium"]
    B = synth.cholesky_vectors(wl.naux, wl.nao, wl.L, seed=wl.seed)
    C = synth.orbitals(wl.nao, seed=wl.seed)
    Cact = C[:, wl.nocc:wl.nocc + wl.nac]
    out = dfmi.ppaa(dev(B), wl.nao, dev(C), dev(Cact))
    torch.cuda.synchronize()
    rows = [0, 1, 149, 150, 169, 170, 598, 599]
    ref = O.ppaa(B, wl.nao, C[:, rows], C, Cact)
    close(out[:, rows, :], packed_uv(ref), what="ppaa medium rows")


def test_ppaa_zero_sizes():
    nao, naux = 40, 20
    B, C = rand_inputs(nao, naux, seed=3)
    out = dfmi.ppaa(dev(B), nao, dev(C), dev(np.zeros((nao, 0))))
    assert out.shape == (0, nao, nao)
    out = dfmi.ppaa(dev(B), nao, dev(np.zeros((nao, 0))), dev(C[:, :4]))
    assert out.shape == (10, 0, 0)
    torch.cuda.synchronize()


def test_ppaa_deterministic():
    nao, naux, nac = 70, 90, 6
    B, C = rand_inputs(nao, naux, seed=4)
    gB, gC, gA = dev(B), dev(C), dev(C[:, :nac])
    a = dfmi.ppaa(gB, nao, gC, gA)
    b = dfmi.ppaa(gB, nao, gC, gA)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
