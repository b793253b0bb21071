"""GPU parity: every C-ABI call against the FP64 CPU oracle on the same seeded inputs.

Bar (FP64 mode): ||Y_gpu - Y_ref||_F <= 1e-10 ||Y_ref||_F and
max|Y_gpu - Y_ref| <= 1e-10 max|Y_ref|  (normwise, since cancellation leaves
entries of J and (pu|vw) far below the matrix scale).  FP64 rounding over the
longest contraction here (N_aux * N_occ = 3.6e5 terms at the medium size) is
of order sqrt(n) * 2^-53 ~ 1e-13, so 1e-10 leaves a wide margin while any
indexing or packing slip shows up as an O(1) error.
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


def close(gpu, ref, tol=TOL, what=""):
    g = gpu.detach().cpu().numpy() if isinstance(gpu, torch.Tensor) else np.asarray(gpu)
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, (what, g.shape, r.shape)
    assert np.all(np.isfinite(g)), what
    d = g - r
    rn, rm = np.linalg.norm(r), np.abs(r).max(initial=0.0)
    if rm == 0.0:
        assert np.abs(d).max(initial=0.0) == 0.0, what
        return
    assert np.linalg.norm(d) <= tol * rn, (what, np.linalg.norm(d) / rn)
    assert np.abs(d).max() <= tol * rm, (what, np.abs(d).max() / rm)


def rand_inputs(nao, naux, nocc, nac, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((naux, O.npair(nao)))
    C = np.linalg.qr(rng.standard_normal((nao, nao)))[0]
    return B, C


def workload_inputs(name):
    wl = synth.WORKLOADS[name]
    B = synth.cholesky_vectors(wl.naux, wl.nao, wl.L, seed=wl.seed)
    C = synth.orbitals(wl.nao, seed=wl.seed)
    return wl, B, C


@pytest.fixture(scope="module", params=["tiny", "medium"])
def wl_case(request):
    wl, B, C = workload_inputs(request.param)
    Cocc = C[:, :wl.nocc]
    Cact = C[:, wl.nocc:wl.nocc + wl.nac]
    ref = {}
    ref["J"], ref["K"], ref["v"] = O.jk(B, wl.nao, Cocc)
    ref["eri"], ref["buv"] = O.active_eri(B, wl.nao, Cact)
    ref["papa"] = O.papa(B, wl.nao, C, Cact)
    gpu = {"B": dev(B), "C": dev(C), "Cocc": dev(Cocc), "Cact": dev(Cact)}
    return wl, B, C, ref, gpu


def test_step_matches_oracle(wl_case):
    wl, B, C, ref, g = wl_case
    out = dfmi.step(g["B"], wl.nao, g["Cocc"], g["Cact"], g["C"])
    torch.cuda.synchronize()
    for k in ("J", "K", "v", "eri", "papa"):
        close(out[k], ref[k], what=f"{wl.name}:{k}")


def test_separate_calls_match_oracle(wl_case):
    wl, B, C, ref, g = wl_case
    J, K, v = dfmi.jk(g["B"], wl.nao, g["Cocc"])
    eri, buv = dfmi.active_eri(g["B"], wl.nao, g["Cact"], return_buv=True)
    pa = dfmi.papa(g["B"], wl.nao, g["C"], g["Cact"])
    torch.cuda.synchronize()
    close(J, ref["J"], what="J")
    close(K, ref["K"], what="K")
    close(v, ref["v"], what="v")
    close(eri, ref["eri"], what="eri")
    close(buv, ref["buv"], what="buv")
    close(pa, ref["papa"], what="papa")


def test_half_transform_and_second_transform(wl_case):
    wl, B, C, ref, g = wl_case
    P = min(wl.naux, 96)          # a slab of rows keeps the host comparison cheap
    Bs = g["B"][:P].contiguous()
    Ch = g["C"][:, : wl.nocc + wl.nac].contiguous()
    X, Y = dfmi.half_transform(Bs, wl.nao, Ch, C2=g["C"])
    torch.cuda.synchronize()
    Xr = O.half_transform(B[:P], wl.nao, C[:, : wl.nocc + wl.nac])
    close(X, Xr, what="X")
    close(Y, O.second_transform(Xr, C), what="Y")


def test_step_is_deterministic(wl_case):
    wl, B, C, ref, g = wl_case
    a = dfmi.step(g["B"], wl.nao, g["Cocc"], g["Cact"], g["C"])
    b = dfmi.step(g["B"], wl.nao, g["Cocc"], g["Cact"], g["C"])
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_symmetry_is_exact(wl_case):
    wl, B, C, ref, g = wl_case
    J, K, _ = dfmi.jk(g["B"], wl.nao, g["Cocc"])
    torch.cuda.synchronize()
    assert torch.equal(J, J.T)
    assert torch.equal(K, K.T)


# shapes that straddle the 128-wide tiles and the 16-wide k slabs, plus degenerate ones
RAGGED = [(1, 1, 1, 1), (2, 3, 1, 1), (7, 5, 3, 2), (33, 17, 5, 3), (130, 9, 17, 5),
          (129, 40, 129, 7), (257, 31, 40, 9), (300, 3, 1, 16)]


@pytest.mark.parametrize("nao,naux,nocc,nac", RAGGED)
def test_ragged_shapes(nao, naux, nocc, nac):
    nocc = min(nocc, nao)
    nac = min(nac, nao)
    B, C = rand_inputs(nao, naux, nocc, nac, seed=nao * 1000 + naux)
    Cocc, Cact = C[:, :nocc], C[:, nao - nac:]
    gB, gC, gO, gA = dev(B), dev(C), dev(Cocc), dev(Cact)
    out = dfmi.step(gB, nao, gO, gA, gC)
    X = dfmi.half_transform(gB, nao, gO)
    torch.cuda.synchronize()
    J, K, v = O.jk(B, nao, Cocc)
    close(out["J"], J, what="J")
    close(out["K"], K, what="K")
    close(out["v"], v, what="v")
    close(out["eri"], O.active_eri(B, nao, Cact)[0], what="eri")
    close(out["papa"], O.papa(B, nao, C, Cact), what="papa")
    close(X, O.half_transform(B, nao, Cocc), what="X")


def test_weighted_and_multiple_densities():
    nao, naux, nocc, ndm = 150, 37, 11, 3
    rng = np.random.default_rng(5)
    B = rng.standard_normal((naux, O.npair(nao)))
    Cs = np.stack([np.linalg.qr(rng.standard_normal((nao, nocc)))[0] for _ in range(ndm)])
    w = rng.standard_normal((ndm, nocc))
    J, K, v = dfmi.jk(dev(B), nao, dev(Cs), w=dev(w))
    torch.cuda.synchronize()
    for z in range(ndm):
        Jr, Kr, vr = O.jk(B, nao, Cs[z], w[z])
        close(J[z], Jr, what=f"J{z}")
        close(K[z], Kr, what=f"K{z}")
        close(v[z], vr, what=f"v{z}")
    # a general (indefinite) symmetric density through its eigen-factorisation
    G = rng.standard_normal((nao, nao))
    G = (G + G.T) / 2
    n, U = np.linalg.eigh(G)
    Jg, Kg, vg = dfmi.jk(dev(B), nao, dev(U), w=dev(n))
    torch.cuda.synchronize()
    # the oracle on the same factorisation (U, n): the bar of every FP64 output
    Jr, Kr, vr = O.jk(B, nao, U, n)
    close(Kg, Kr, what="K general gamma")
    close(Jg, Jr, what="J general gamma")
    close(vg, vr, what="v general gamma")


def test_step_with_weights():
    nao, naux, nocc, nac = 70, 23, 9, 4
    B, C = rand_inputs(nao, naux, nocc, nac, seed=11)
    w = np.random.default_rng(2).standard_normal(nocc)
    Cocc, Cact = C[:, :nocc], C[:, nocc:nocc + nac]
    out = dfmi.step(dev(B), nao, dev(Cocc), dev(Cact), dev(C), w=dev(w))
    torch.cuda.synchronize()
    J, K, v = O.jk(B, nao, Cocc, w)
    close(out["J"], J, what="J")
    close(out["K"], K, what="K")
    close(out["v"], v, what="v")


def test_zero_occupied_and_zero_active():
    nao, naux = 40, 12
    B, C = rand_inputs(nao, naux, 0, 0, seed=3)
    gB = dev(B)
    J, K, v = dfmi.jk(gB, nao, dev(np.zeros((nao, 0))))
    torch.cuda.synchronize()
    assert torch.count_nonzero(J) == 0 and torch.count_nonzero(K) == 0 and torch.count_nonzero(v) == 0
    out = dfmi.step(gB, nao, dev(np.zeros((nao, 0))), dev(C[:, :3]), dev(C))
    torch.cuda.synchronize()
    assert torch.count_nonzero(out["J"]) == 0 and torch.count_nonzero(out["K"]) == 0
    close(out["eri"], O.active_eri(B, nao, C[:, :3])[0], what="eri")
    e = dfmi.active_eri(gB, nao, dev(np.zeros((nao, 0))))
    assert e.numel() == 0


def test_full_papa_block():
    nao, naux, nac, nq = 90, 29, 5, 33
    B, C = rand_inputs(nao, naux, 0, nac, seed=9)
    Cact, Cq = C[:, :nac], C[:, 40:40 + nq]
    out = dfmi.papa(dev(B), nao, dev(C), dev(Cact), Cq=dev(Cq))
    torch.cuda.synchronize()
    close(out, O.papa_full(B, nao, C, Cact, Cq), what="papa full")


def test_full_k_and_j_on_128_tiles():
    """N_ao 700 (> 640) takes the 128 x 128 SYRK tiles the paper-scale K uses, with a ragged last
    tile (700 = 5 * 128 + 60): full J, K and v against the oracle, K and J exactly symmetric."""
    nao, naux, nocc = 700, 40, 75
    B, C = rand_inputs(nao, naux, nocc, 0, seed=700)
    Cocc = C[:, :nocc]
    J, K, v = dfmi.jk(dev(B), nao, dev(Cocc))
    torch.cuda.synchronize()
    Jr, Kr, vr = O.jk(B, nao, Cocc)
    close(K, Kr, what="K, 128-wide tiles")
    close(J, Jr, what="J")
    close(v, vr, what="v")
    assert torch.equal(K, K.T) and torch.equal(J, J.T)
