"""Parity at the paper-scale workload (N_ao 1200, N_aux 4800, N_occ 300, N_ac 40) against the full
FP64 oracle, streamed over blocks of auxiliary rows (oracle/df_stream.py): every output the
benchmark times, in the launch configuration it times.

  * forward (df_step, p over all 1200 MOs): v and J in full, rows of K and K C_occ in full, (uv|wx)
    in full, sampled p rows of (pu|vw);
  * the differentiable step E(kappa), dE/dkappa through the library's adjoint (DFStep): at kappa = 0
    with the half transforms kept, recomputed in one piece, and recomputed in P chunks under a
    scratch limit (ragged last chunk); at kappa = 0.01 N(0,1) against the oracle's gradient at
    C0 exp(kappa - kappa^T) (SciPy's Frechet adjoint); central finite differences (h = 1e-5) of the
    GPU energy along 8 random unit directions, also with h = 1e-4.

Bars: 1e-10 normwise and max relative for every array (the FP64 bar); |E_gpu - E_oracle| <= 1e-8
Eh (|E| is 3.3e6 Eh here, so that is 3e-15 relative: the reordering floor of FP64 sums).
"""
import math

import numpy as np
import pytest
import scipy.linalg

torch = pytest.importorskip("torch")

from oracle import df_stream as S
from paper_2505_03755_amd import dfmi, synth

pytestmark = pytest.mark.gpu
TOL = 1e-10
E_BAR = 1e-8
P_ROWS = [0, 1, 299, 300, 320, 339, 340, 777, 1199]
K_ROWS = [0, 1, 150, 299, 600, 1000, 1198, 1199]


def close(gpu, ref, what, tol=TOL):
    g = gpu.detach().cpu().numpy() if isinstance(gpu, torch.Tensor) else np.asarray(gpu)
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, (what, g.shape, r.shape)
    assert np.all(np.isfinite(g)), what
    d = g - r
    en, em = np.linalg.norm(d) / np.linalg.norm(r), np.abs(d).max() / np.abs(r).max()
    print(f"{what}: normwise {en:.2e}, max {em:.2e}", flush=True)
    assert en <= tol and em <= tol, (what, en, em)


def dev_chunks(B, chunk=96):
    """Packed rows of the device B, copied to the host block by block, in P order."""
    for p0 in range(0, B.shape[0], chunk):
        yield p0, B[p0:p0 + chunk].cpu().numpy()


@pytest.fixture(scope="module")
def paper():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = synth.WORKLOADS["paper"]
    dev = torch.device("cuda", 0)
    B = synth.device_cholesky_vectors(wl.naux, wl.nao, wl.L, seed=wl.seed, device=dev)
    C0 = synth.orbitals(wl.nao, seed=wl.seed)
    h = synth.symmetric_matrix(wl.nao, seed=wl.seed)
    Gam = synth.two_body_density(wl.nac, seed=wl.seed)
    kap = synth.kappa(wl.nmo, seed=wl.seed)
    yield wl, B, C0, h, Gam, kap
    del B
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def oracle0(paper):
    """The oracle's pass at kappa = 0 (C = C0)."""
    wl, B, C0, h, Gam, kap = paper
    print("oracle pass at kappa = 0", flush=True)
    return S.step_pass(dev_chunks(B), wl.naux, wl.nao, C0, wl.nocc, wl.nac, h, Gam, p_rows=P_ROWS, k_rows=K_ROWS)


def gpu_energy(paper, kappa, keep_x=True, grad=True):
    wl, B, C0, h, Gam, kap = paper
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(B.device)
    k = d(kappa).requires_grad_(grad)
    E = dfmi.energy(B, wl.nao, d(C0), k, wl.nocc, wl.nac, d(h), d(Gam), keep_x=keep_x)
    if not grad:
        return E.item(), None
    E.backward()
    return E.item(), k.grad.detach()


def test_forward_against_oracle(paper, oracle0):
    wl, B, C0, h, Gam, kap = paper
    r = oracle0
    C = torch.from_numpy(C0).to(B.device)
    Cocc = C[:, :wl.nocc].contiguous()
    out = dfmi.step(B, wl.nao, Cocc, C[:, wl.nocc:wl.nocc + wl.nac].contiguous(), C)
    torch.cuda.synchronize()
    close(out["v"], r["v"], "v")
    close(out["J"], r["J"], "J")
    close(out["K"][K_ROWS], r["K_rows"], "K rows")
    close(out["K"] @ Cocc, r["KC"], "K C_occ")
    close(out["eri"], r["eri"], "(uv|wx)")
    close(out["papa"][P_ROWS], r["papa_rows"], "(pu|vw) rows")
    assert torch.equal(out["K"], out["K"].T) and torch.equal(out["J"], out["J"].T)


@pytest.mark.parametrize("keep_x, limit", [(True, 0), (False, 0), (False, 6 << 30)])
def test_energy_and_gradient_at_kappa0(paper, oracle0, keep_x, limit):
    """dE/dkappa = A - A^T with A = C0^T dE/dC at kappa = 0; keep_x=False recomputes the half
    transforms in the adjoint, in P chunks when the scratch limit is set (6 GiB: five chunks of 996 rows here, the last one ragged)."""
    wl = paper[0]
    ctx = dfmi.context(paper[1].device)
    ctx.set_scratch_limit(limit)
    try:
        if limit:
            rows = ctx.backward_chunk(naux=wl.naux, nao=wl.nao, nocc=wl.nocc, nac=wl.nac,
                                      flags=dfmi.DF_BWD_GJ | dfmi.DF_BWD_GK | dfmi.DF_BWD_GERI)
            assert 1 < -(-wl.naux // rows) and wl.naux % rows != 0, rows
        E, g = gpu_energy(paper, np.zeros((wl.nmo, wl.nmo)), keep_x=keep_x)
    finally:
        ctx.set_scratch_limit(0)
    print(f"E_gpu = {E!r}, E_oracle = {oracle0['E']!r}, dE = {E - oracle0['E']:.3e}", flush=True)
    assert abs(E - oracle0["E"]) <= E_BAR
    ref = S.orbital_gradient_from_G(paper[2], np.zeros((wl.nmo, wl.nmo)), oracle0["G"])
    close(g, ref, f"dE/dkappa at 0 (keep_x={keep_x}, limit={limit})")


def test_energy_and_gradient_at_kappa(paper):
    """kappa = 0.01 N(0,1): the oracle's own pass at C = C0 exp(kappa - kappa^T)."""
    wl, B, C0, h, Gam, kap = paper
    C = C0 @ scipy.linalg.expm(kap - kap.T)
    print("oracle pass at kappa = 0.01 N(0,1)", flush=True)
    r = S.step_pass(dev_chunks(B), wl.naux, wl.nao, C, wl.nocc, wl.nac, h, Gam)
    E, g = gpu_energy(paper, kap)
    print(f"E_gpu = {E!r}, E_oracle = {r['E']!r}, dE = {E - r['E']:.3e}", flush=True)
    assert abs(E - r["E"]) <= E_BAR
    close(g, S.orbital_gradient_from_G(C0, kap, r["G"]), "dE/dkappa at kappa")


def test_finite_differences_at_kappa(paper):
    """Central differences of the GPU energy along 8 unit directions against <dE/dkappa, d>, with
    h = 1e-5 and h = 1e-4.  Error budget: each energy carries a rounding error eps of a few units
    in the last place of |E| = 3.3e6 Eh (measured against the oracle: about 13 u |E|, 5e-9 Eh);
    the difference quotient turns it into eps / h (5e-4 at h = 1e-5), and the truncation term
    (h^2 / 6 times the third derivative) stays below 1e-6 relative at both steps.  Bound: 8 eps / h
    with eps = 16 u |E|, plus 1e-7 relative."""
    wl, B, C0, h, Gam, kap = paper
    E0, g = gpu_energy(paper, kap)
    g = g.cpu().numpy()
    eps = 16 * np.finfo(np.float64).eps / 2 * abs(E0)
    for i, d in enumerate(synth.directions(8, (wl.nmo, wl.nmo), seed=wl.seed)):
        an = math.fsum((g * d).ravel().tolist())
        for hstep in (1e-5, 1e-4):
            Ep, _ = gpu_energy(paper, kap + hstep * d, grad=False)
            Em, _ = gpu_energy(paper, kap - hstep * d, grad=False)
            fd = (Ep - Em) / (2 * hstep)
            bound = 8 * eps / hstep + 1e-7 * abs(an)
            print(f"direction {i}, h {hstep:.0e}: fd {fd:.10e}, analytic {an:.10e}, diff {fd - an:.2e} "
                  f"(bound {bound:.1e})", flush=True)
            assert abs(fd - an) <= bound, (i, hstep, fd, an)
