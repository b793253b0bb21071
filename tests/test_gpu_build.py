"""GPU parity of df_build_cholesky (Eq. cholesky: (P|Q) = L L^T, b = L^-1 (Q|mu nu)) and of
df_embed_cholesky (b^P in another orbital basis) against the FP64 oracle.

Bar: normwise 1e-10.  The blocked factorisation and the substitution through inverted 128-wide
diagonal blocks differ from the oracle's LAPACK routines in rounding order only; their error
grows with the metric's condition number (about kappa^(1/2) eps for L and B), which is 1e6
here at most, so 1e-10 keeps a margin of several hundred.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import df_build as OB
from oracle import df_oracle as O
from paper_2505_03755_amd import dfmi, synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def rel(a, b):
    a = a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else np.asarray(a)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("naux,nao,cond", [(300, 20, 1e4), (128, 9, 1e6), (129, 13, 1e2), (57, 30, 1e6),
                                           (1, 4, 1.0), (520, 33, 1e6), (200, 1, 1e3), (256, 2, 1e5)])
def test_build_against_oracle(naux, nao, cond):
    metric = synth.coulomb_metric(naux, cond, seed=naux)
    E = synth.cholesky_vectors(naux, nao, 10.0, seed=naux + 1)
    L, B, info = dfmi.build_cholesky(dev(metric), dev(E), nao)
    assert int(info.item()) == 0
    assert rel(L, OB.metric_cholesky(metric)) <= TOL
    assert rel(B, OB.cholesky_vectors(metric, E)) <= TOL
    assert not torch.triu(L, 1).any()


def test_build_in_place_equals_out_of_place():
    naux, nao = 300, 24
    metric = dev(synth.coulomb_metric(naux, 1e5, seed=3))
    E = dev(synth.cholesky_vectors(naux, nao, 10.0, seed=4))
    L, B, _ = dfmi.build_cholesky(metric, E, nao)
    m2, e2 = metric.clone(), E.clone()
    L2, B2, _ = dfmi.build_cholesky(m2, e2, nao, in_place=True)
    torch.cuda.synchronize()
    assert L2.data_ptr() == m2.data_ptr() and B2.data_ptr() == e2.data_ptr()
    assert torch.equal(L, L2) and torch.equal(B, B2)


def test_not_positive_definite_reports_the_pivot():
    naux, nao = 200, 6
    w, Q = np.linalg.eigh(synth.coulomb_metric(naux, 1e3, seed=5))
    w[0] = -1e-2                                   # one negative eigenvalue
    bad = (Q * w) @ Q.T
    _, _, info = dfmi.build_cholesky(dev(bad), dev(synth.cholesky_vectors(naux, nao, 10.0, seed=6)), nao,
                                     check=False)
    k = int(info.item())
    assert 0 < k <= naux
    # the leading minors before the reported pivot are positive definite
    assert np.linalg.eigvalsh(bad[:k - 1, :k - 1])[0] > 0 if k > 1 else True
    with pytest.raises(ValueError):
        dfmi.build_cholesky(dev(bad), dev(synth.cholesky_vectors(naux, nao, 10.0, seed=6)), nao)


def test_built_vectors_feed_the_jk_call():
    """J and K from the built b^P equal the oracle's J and K from the oracle's b^P."""
    naux, nao, nocc = 260, 40, 9
    metric = synth.coulomb_metric(naux, 1e4, seed=8)
    E = synth.cholesky_vectors(naux, nao, 10.0, seed=9)
    _, B, _ = dfmi.build_cholesky(dev(metric), dev(E), nao)
    C = synth.orbitals(nao, seed=8)[:, :nocc]
    J, K, _ = dfmi.jk(B, nao, dev(C))
    Jr, Kr, _ = O.jk(OB.cholesky_vectors(metric, E), nao, C)
    assert rel(J, Jr) <= TOL and rel(K, Kr) <= TOL


@pytest.mark.parametrize("naux,nao,nemb", [(50, 40, 17), (33, 7, 7), (20, 65, 1), (64, 30, 45)])
def test_embed_against_oracle(naux, nao, nemb):
    B = synth.cholesky_vectors(naux, nao, 10.0, seed=nao)
    M = np.random.default_rng(nemb).standard_normal((nao, nemb))
    Be = dfmi.embed_cholesky(dev(B), nao, dev(M))
    torch.cuda.synchronize()
    assert rel(Be, OB.embed(B, nao, M)) <= TOL


def test_embed_identity_is_exact():
    """M = I: every product is by 1 or 0, so the embedded vectors are B bit for bit."""
    naux, nao = 70, 37
    B = dev(synth.cholesky_vectors(naux, nao, 10.0, seed=3))
    Be = dfmi.embed_cholesky(B, nao, dev(np.eye(nao)))
    torch.cuda.synchronize()
    assert torch.equal(Be, B)


def test_embed_in_chunks_sampled_rows():
    """N_ao 1200 into 400 embedding orbitals: P runs in chunks of 209 rows; rows on both sides of
    the chunk boundaries against the oracle on those rows."""
    naux, nao, nemb = 480, 1200, 400
    B = synth.device_cholesky_vectors(naux, nao, 40.0, seed=2)
    M = np.linalg.qr(np.random.default_rng(1).standard_normal((nao, nemb)))[0]
    Be = dfmi.embed_cholesky(B, nao, dev(M))
    torch.cuda.synchronize()
    rows = [0, 1, 208, 209, 210, 417, 418, 479]
    idx = torch.as_tensor(rows, device=B.device)
    assert rel(Be[idx], OB.embed(B[idx].cpu().numpy(), nao, M)) <= TOL


def test_build_paper_scale_sampled_pairs():
    """N_aux 4800, N_ao 1200 (B 27.7 GB), in place: L against the oracle's factor; sampled pair
    columns of B against the oracle's substitution on those columns (columns are independent)."""
    naux, nao = 4800, 1200
    metric = synth.coulomb_metric(naux, 1e6, seed=11)
    E = synth.device_cholesky_vectors(naux, nao, 40.0, seed=12)
    cols = torch.as_tensor([0, 1, 2, 777, 4096, 300000, 720598, 720599], device=E.device)
    Es = E[:, cols].cpu().numpy()
    L, B, _ = dfmi.build_cholesky(dev(metric), E, nao, in_place=True)
    Lr = OB.metric_cholesky(metric)
    assert rel(L, Lr) <= TOL
    assert rel(B[:, cols], OB.cholesky_vectors(metric, Es)) <= TOL
    del L, B, E
    torch.cuda.empty_cache()
