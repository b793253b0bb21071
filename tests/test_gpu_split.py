"""GPU tests of the split-precision path (int8 slices on the matrix cores).

The reference is the FP64 oracle itself; the bar is the error bound of the method, derived from
its definition (include/dfmi.h, split precision): for rows a, b of length K with exponents
e_a, e_b (max|a| < 2^e_a), the slice product differs from the exact dot product by at most
    K (S + 4) 2^(e_a + e_b - 7 S)
(dropped slice pairs and the residuals of both splits), plus FP64 rounding of the final sums.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import df_grad as G
from oracle import df_oracle as O
from paper_2505_03755_amd import dfmi, synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def row_exp(A):
    m = np.abs(A).max(axis=1)
    return np.where(m > 0, np.frexp(m)[1], 0).astype(np.float64)


def bound(A, B, S):
    """Elementwise bound of |split(A B^T) - A B^T| (method + FP64 rounding of the sums)."""
    K = A.shape[1]
    meth = K * (S + 4) * np.exp2(row_exp(A)[:, None] + row_exp(B)[None, :] - 7 * S)
    fp = 4 * K * np.finfo(np.float64).eps * (np.abs(A) @ np.abs(B).T)
    return meth + fp


@pytest.mark.parametrize("S", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (65, 17, 63), (64, 64, 64), (130, 70, 65), (200, 129, 1000)])
def test_split_matmul_within_bound(S, M, N, K):
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    # rows with very different scales, and entries spread over many binades within a row
    A = rng.standard_normal((M, K)) * np.exp2(rng.integers(-20, 20, (M, 1))) * np.exp2(rng.uniform(-8, 0, (M, K)))
    B = rng.standard_normal((N, K)) * np.exp2(rng.integers(-20, 20, (N, 1)))
    C = dfmi.split_matmul(dev(A), dev(B), nslice=S).cpu().numpy()
    ref = A @ B.T
    err = np.abs(C - ref)
    assert np.all(err <= bound(A, B, S)), (np.max(err / bound(A, B, S)))


@pytest.mark.parametrize("S", [5, 7])
def test_split_matmul_split_over_k(S):
    """K = 40000: the product runs as several k splits (each at most 32768 k) and a fixed-order sum."""
    rng = np.random.default_rng(41)
    M, N, K = 70, 50, 40000
    A = rng.standard_normal((M, K)) * np.exp2(rng.integers(-10, 10, (M, 1)))
    B = rng.standard_normal((N, K))
    C = dfmi.split_matmul(dev(A), dev(B), nslice=S).cpu().numpy()
    err = np.abs(C - A @ B.T)
    assert np.all(err <= bound(A, B, S)), (np.max(err / bound(A, B, S)))


def test_split_matmul_not_fp64_at_few_slices():
    """With 4 slices the method error dominates FP64 rounding: the int8 path really is in use."""
    rng = np.random.default_rng(5)
    A, B = rng.standard_normal((128, 512)), rng.standard_normal((96, 512))
    ref = A @ B.T
    e4 = np.abs(dfmi.split_matmul(dev(A), dev(B), nslice=4).cpu().numpy() - ref).max()
    e8 = np.abs(dfmi.split_matmul(dev(A), dev(B), nslice=8).cpu().numpy() - ref).max()
    assert e4 > 1e3 * e8
    assert e8 <= 1e-12 * np.abs(ref).max()


def test_split_matmul_zero_rows():
    A = np.zeros((3, 20))
    A[1] = np.arange(20.0)
    B = np.ones((5, 20))
    C = dfmi.split_matmul(dev(A), dev(B), nslice=7).cpu().numpy()
    assert np.array_equal(C, A @ B.T)


@pytest.mark.parametrize("S", [5, 7])
@pytest.mark.parametrize("nao,naux", [(1, 2), (33, 17), (70, 9)])
def test_split_cholesky_reconstructs_rows(S, nao, naux):
    Bp = synth.cholesky_vectors(naux, nao, 8.0, seed=nao)
    Bs, Be = dfmi.split_cholesky(dev(Bp), nao, nslice=S)
    torch.cuda.synchronize()
    blocks = Bs.cpu().numpy().astype(np.float64)         # [S][row group][k block][1024]
    G, KB = blocks.shape[1], blocks.shape[2]
    assert blocks.shape == (S, (naux * nao + 31) // 32, (nao + 63) // 64 * 2, 1024)
    # slot rr + 32 c of block (s, g, b) holds k = 32 b + 16 c + [0, 16) of row 32 g + rr
    planes = blocks.reshape(S, G, KB, 2, 32, 16).transpose(0, 1, 4, 2, 3, 5).reshape(S, 32 * G, 32 * KB)
    ex = Be.cpu().numpy().astype(np.float64)
    assert np.abs(planes).max() <= 64
    full = O.unpack(Bp, nao).reshape(naux * nao, nao)     # rows (P, mu)
    assert np.array_equal(ex, row_exp(full))
    assert not planes[:, :, nao:].any() and not planes[:, naux * nao:, :].any()
    planes = planes[:, :naux * nao, :]
    rec = sum(planes[s, :, :nao] * np.exp2(-6 - 7 * s) for s in range(S)) * np.exp2(ex)[:, None]
    assert np.all(np.abs(rec - full) <= np.exp2(ex - 7 * S)[:, None])


def close(gpu, ref, tol):
    g = gpu.detach().cpu().numpy()
    r = np.asarray(ref)
    assert np.linalg.norm(g - r) <= tol * np.linalg.norm(r), np.linalg.norm(g - r) / np.linalg.norm(r)


def split_problem(nao, naux, nocc, nac, S, seed=0, L=10.0):
    Bp = synth.cholesky_vectors(naux, nao, L, seed=seed)
    C = synth.orbitals(nao, seed=seed)
    gB = dev(Bp)
    Bs, Be = dfmi.split_cholesky(gB, nao, nslice=S)
    return Bp, C, gB, Bs, Be


@pytest.mark.parametrize("nao,naux,nocc,nac", [(120, 480, 30, 8), (33, 17, 5, 3), (130, 9, 17, 5), (7, 70, 0, 3),
                                               (9, 20, 4, 0), (40, 1100, 16, 3)])
def test_step_split_matches_oracle(nao, naux, nocc, nac):
    Bp, C, gB, Bs, Be = split_problem(nao, naux, nocc, nac, 7, seed=nao + naux)
    Co, Ca = C[:, :nocc], C[:, nocc:nocc + nac]
    out = dfmi.step_split(gB, Bs, Be, nao, dev(Co), dev(Ca), dev(C))
    torch.cuda.synchronize()
    J, K, v = O.jk(Bp, nao, Co)
    eri, _ = O.active_eri(Bp, nao, Ca)
    pa = O.papa(Bp, nao, C, Ca)
    tol = 1e-11
    if nocc:
        close(out["J"], J, tol)
        close(out["K"], K, tol)
        close(out["v"], v, tol)
        assert torch.equal(out["K"], out["K"].T)
    else:
        assert not out["J"].any() and not out["K"].any() and not out["v"].any()
    if nac:
        close(out["eri"], eri, tol)
        close(out["papa"], pa, tol)


@pytest.mark.parametrize("S,bar", [(7, 1e-8), (8, 1e-8)])
def test_split_energy_error_medium(S, bar):
    """Delta E of the model energy against the FP64 oracle, medium workload (|E| ~ 8e5)."""
    wl = synth.WORKLOADS["medium"]
    Bp, C, gB, Bs, Be = split_problem(wl.nao, wl.naux, wl.nocc, wl.nac, S, seed=0, L=wl.L)
    h, Gam = synth.symmetric_matrix(wl.nao), synth.two_body_density(wl.nac)
    Co, Ca = C[:, :wl.nocc], C[:, wl.nocc:wl.nocc + wl.nac]
    out = dfmi.step_split(gB, Bs, Be, wl.nao, dev(Co), dev(Ca), dev(C))
    torch.cuda.synchronize()
    D = Co @ Co.T
    terms = [O.fsum_dot(D, h), 0.5 * O.fsum_dot(D, out["J"].cpu().numpy()),
             -0.25 * O.fsum_dot(D, out["K"].cpu().numpy()), 0.5 * O.fsum_dot(out["eri"].cpu().numpy(), Gam)]
    E = math.fsum(terms)
    E_ref = G.energy(Bp, wl.nao, C, wl.nocc, wl.nac, h, Gam)
    assert abs(E - E_ref) <= bar, (E - E_ref, E_ref)


def unblock(blocks):
    """[S][row group][k block][1024] -> [S][32 G][32 KB]: slot rr + 32 c of block (s, g, b) holds
    k = 32 b + 16 c + [0, 16) of row 32 g + rr."""
    S, G, KB = blocks.shape[:3]
    return blocks.reshape(S, G, KB, 2, 32, 16).transpose(0, 1, 4, 2, 3, 5).reshape(S, 32 * G, 32 * KB)


@pytest.mark.parametrize("nao,naux", [(1, 2), (33, 17), (70, 9)])
def test_split_cholesky_t_reconstructs_rows(nao, naux):
    """Rows mu of the DF tensor over k = (P, nu): b^P_{mu nu} within 2^(e - 7 S) of the slices."""
    S = 7
    Bp = synth.cholesky_vectors(naux, nao, 8.0, seed=nao + 1)
    Bt, Bte = dfmi.split_cholesky_t(dev(Bp), nao, nslice=S)
    torch.cuda.synchronize()
    planes = unblock(Bt.cpu().numpy().astype(np.float64))
    assert planes.shape == (S, (nao + 31) // 32 * 32, (naux * nao + 63) // 64 * 64)
    assert np.abs(planes).max() <= 64
    rows = O.unpack(Bp, nao).transpose(1, 0, 2).reshape(nao, naux * nao)   # [mu][(P, nu)]
    ex = Bte.cpu().numpy().astype(np.float64)
    assert np.array_equal(ex, row_exp(rows))
    assert not planes[:, nao:, :].any() and not planes[:, :, naux * nao:].any()
    planes = planes[:, :nao, :naux * nao]
    rec = sum(planes[s] * np.exp2(-6 - 7 * s) for s in range(S)) * np.exp2(ex)[:, None]
    assert np.all(np.abs(rec - rows) <= np.exp2(ex - 7 * S)[:, None])


ADJ_SHAPES = [(120, 480, 30, 8), (33, 17, 5, 3), (130, 9, 17, 5), (40, 1100, 16, 3), (9, 20, 4, 0), (7, 70, 0, 3)]


@pytest.mark.parametrize("nao,naux,nocc,nac", ADJ_SHAPES)
def test_step_backward_split_matches_oracle(nao, naux, nocc, nac):
    """Split forward (keeping X) then the split adjoint, against the oracle's VJP; and against the
    FP64 adjoint on the same saved factors.  (40, 1100, 16, 3) contracts over 44000 (P, nu): the
    last product runs as two k splits."""
    Bp, C, gB, Bs, Be = split_problem(nao, naux, nocc, nac, 7, seed=nao + 2 * naux)
    Bt, Bte = dfmi.split_cholesky_t(gB, nao, nslice=7)
    Co, Ca = C[:, :nocc].copy(), C[:, nocc:nocc + nac].copy()
    out = dfmi.step_split(gB, Bs, Be, nao, dev(Co), dev(Ca), dev(C), keep_x=True)
    torch.cuda.synchronize()
    if nocc:
        close(out["Xocc"], O.half_transform(Bp, nao, Co), 1e-11)
    if nac:
        close(out["Xact"], O.half_transform(Bp, nao, Ca).transpose(1, 0, 2), 1e-11)
    rng = np.random.default_rng(nao)
    gJ, gK = rng.standard_normal((nao, nao)), rng.standard_normal((nao, nao))
    ge = rng.standard_normal((nac,) * 4)
    ref_o, ref_a = G.step_vjp(Bp, nao, Co, Ca, gJ, gK, ge)
    args = (dev(Co), dev(Ca), dev(gJ), dev(gK), dev(ge), out["Xocc"], out["Xact"])
    dCo, dCa = dfmi.step_backward_split(gB, Bt, Bte, nao, *args)
    f_o, f_a = dfmi.step_backward(gB, nao, *args)
    torch.cuda.synchronize()
    if nocc:
        close(dCo, ref_o, 1e-11)
        close(dCo, f_o.cpu().numpy(), 1e-11)
    if nac:
        close(dCa, ref_a, 1e-11)
        close(dCa, f_a.cpu().numpy(), 1e-11)


def test_step_backward_split_exchange_medium():
    """Medium workload: with gK = D/2 the exchange part of the adjoint is K C_occ (oracle K)."""
    wl = synth.WORKLOADS["medium"]
    Bp, C, gB, Bs, Be = split_problem(wl.nao, wl.naux, wl.nocc, wl.nac, 7, seed=0, L=wl.L)
    Bt, Bte = dfmi.split_cholesky_t(gB, wl.nao, nslice=7)
    Co, Ca = C[:, :wl.nocc].copy(), C[:, wl.nocc:wl.nocc + wl.nac].copy()
    out = dfmi.step_split(gB, Bs, Be, wl.nao, dev(Co), dev(Ca), dev(C), keep_x=True)
    D = Co @ Co.T
    dCo, _ = dfmi.step_backward_split(gB, Bt, Bte, wl.nao, dev(Co), dev(Ca), None, dev(0.5 * D), None,
                                      out["Xocc"], out["Xact"])
    torch.cuda.synchronize()
    K = O.exchange(Bp, wl.nao, Co)
    close(dCo, K @ Co, 1e-11)


def test_split_results_do_not_depend_on_workspace_alignment():
    """The slice planes sit on 4 KB offsets of the workspace; a workspace 256 bytes past such a
    boundary (the least alignment the ABI takes) only moves them, so the split forward and the
    split adjoint give the same bits."""
    nao, naux, nocc, nac = 130, 90, 20, 5
    Bp, C, gB, Bs, Be = split_problem(nao, naux, nocc, nac, 7, seed=3)
    Bt, Bte = dfmi.split_cholesky_t(gB, nao, nslice=7)
    Co, Ca = dev(C[:, :nocc].copy()), dev(C[:, nocc:nocc + nac].copy())
    rng = np.random.default_rng(3)
    gJ, gK, ge = dev(rng.standard_normal((nao, nao))), dev(rng.standard_normal((nao, nao))), \
        dev(rng.standard_normal((nac,) * 4))
    ctx = dfmi.Context(torch.device("cuda", 0))

    def run():
        out = dfmi.step_split(gB, Bs, Be, nao, Co, Ca, dev(C), keep_x=True, ctx=ctx)
        dCo, dCa = dfmi.step_backward_split(gB, Bt, Bte, nao, Co, Ca, gJ, gK, ge, out["Xocc"], out["Xact"],
                                            ctx=ctx)
        torch.cuda.synchronize()
        return [out[k].clone() for k in ("J", "K", "eri", "papa", "Xocc", "Xact")] + [dCo.clone(), dCa.clone()]

    ref = run()
    need = ctx._ws.numel()
    big = torch.empty(need + 8192, dtype=torch.uint8, device="cuda")
    base = (-big.data_ptr()) % 4096 + 256                 # 256 bytes past a 4 KB boundary
    ctx._ws = big[base:base + need]
    assert ctx._ws.data_ptr() % 4096 == 256
    got = run()
    assert ctx._ws.data_ptr() % 4096 == 256               # the call kept the offset workspace
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
