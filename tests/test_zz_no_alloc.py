"""df_jk_noalloc (the JK call on the library's static scratch, no allocation) against df_jk.

Two calls in a row, through the C ABI: a larger problem whose workspace does not fit the 128 MiB
scratch (so the auxiliary rows run in several blocks, the last one ragged), with signed weights
and all three outputs, then a smaller one (one block) that reuses the scratch the first left
behind.  Each is compared with df_jk on the same inputs at the 1e-10 bar (normwise and max
relative); J and K are summed in a different order (over the blocks), v is the same per row.
DF_ACCUMULATE adds onto what the outputs hold.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import df_oracle as O
from paper_2505_03755_amd import dfmi

pytestmark = pytest.mark.gpu
TOL = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def close(gpu, ref, what, tol=TOL):
    g = gpu.detach().cpu().numpy()
    r = ref.detach().cpu().numpy() if isinstance(ref, torch.Tensor) else np.asarray(ref)
    assert g.shape == r.shape, what
    assert np.all(np.isfinite(g)), what
    d = g - r
    assert np.linalg.norm(d) <= tol * np.linalg.norm(r), (what, np.linalg.norm(d) / np.linalg.norm(r))
    assert np.abs(d).max() <= tol * np.abs(r).max(), (what, np.abs(d).max() / np.abs(r).max())


def inputs(nao, naux, ndm, nocc, seed):
    rng = np.random.default_rng(seed)
    env = np.exp(-np.abs(np.subtract.outer(np.arange(nao), np.arange(nao))) / 20.0)[np.tril_indices(nao)]
    B = rng.standard_normal((naux, O.npair(nao))) * env
    C = np.stack([np.linalg.qr(rng.standard_normal((nao, nocc)))[0] for _ in range(ndm)])
    w = rng.uniform(-1.0, 2.0, (ndm, nocc))
    return B, C, w


def run_pair(nao, naux, ndm, nocc, seed):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"df_jk_noalloc: nao={nao} naux={naux} ndm={ndm} nocc={nocc}", flush=True)
    B, C, w = inputs(nao, naux, ndm, nocc, seed)
    gB, gC, gw = dev(B), dev(C), dev(w)
    J, K, v = dfmi.jk(gB, nao, gC, w=gw)
    out = {"J": torch.empty_like(J), "K": torch.empty_like(K), "v": torch.empty_like(v)}
    Jn, Kn, vn = dfmi.jk_noalloc(gB, nao, gC, w=gw, out=out)
    torch.cuda.synchronize()
    close(Jn, J, "J")
    close(Kn, K, "K")
    close(vn, v, "v")
    assert torch.equal(Kn, Kn.transpose(1, 2)) and torch.equal(Jn, Jn.transpose(1, 2))
    first = (Jn.clone(), Kn.clone(), vn.clone())
    # accumulate: the second call adds the same results again
    dfmi.jk_noalloc(gB, nao, gC, w=gw, out=out, accumulate=True)
    torch.cuda.synchronize()
    close(out["J"], 2.0 * J, "J accumulated")
    close(out["K"], 2.0 * K, "K accumulated")
    close(out["v"], 2.0 * v, "v accumulated")
    return (B, C, w) + first


def test_two_calls_larger_then_smaller():
    # 1) about 123 auxiliary rows fit the scratch per block here: 6 blocks, the last one ragged
    run_pair(400, 700, 3, 100, seed=1)
    # 2) a smaller problem, one block, on the scratch the first call left behind
    B, C, w, Jn, Kn, vn = run_pair(57, 33, 1, 9, seed=2)
    Jr, Kr, vr = O.jk(B, 57, C[0], w[0])
    close(Jn[0], Jr, "J vs oracle")
    close(Kn[0], Kr, "K vs oracle")
    close(vn[0], vr, "v vs oracle")


def test_rejects_what_does_not_fit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # one auxiliary row at nao 3000 needs 3000^2 doubles of K partials alone (72 MB) per density:
    # two densities do not fit
    nao = 3000
    B = torch.zeros((1, O.npair(nao)), dtype=torch.float64, device="cuda")
    C = torch.zeros((2, nao, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(dfmi.DFError, match="static scratch"):
        dfmi.jk_noalloc(B, nao, C, out={"K": torch.zeros((2, nao, nao), dtype=torch.float64, device="cuda")})
    with pytest.raises(dfmi.DFError, match="DF_ERR_UNSUPPORTED"):
        ctx = dfmi.context()
        ctx.check(ctx._lib.df_jk_noalloc(ctx.handle, dfmi._ptr(B), 1, nao, 1, dfmi._ptr(C), 1, None,
                                         None, None, None, dfmi.DF_PREC_SPLIT))
