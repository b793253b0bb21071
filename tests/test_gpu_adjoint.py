"""GPU parity of the hand-written adjoint (df_step_backward) and of dE/dkappa through autograd.

Same bar as the forward: normwise 1e-10 relative against the FP64 oracle (oracle/df_grad.py),
whose derivatives are pinned by finite differences on the CPU.
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


def close(gpu, ref, tol=TOL, what=""):
    g = gpu.detach().cpu().numpy() if isinstance(gpu, torch.Tensor) else np.asarray(gpu)
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, (what, g.shape, r.shape)
    d = g - r
    rn, rm = np.linalg.norm(r), np.abs(r).max(initial=0.0)
    if rm == 0.0:
        assert np.abs(d).max(initial=0.0) == 0.0, what
        return
    assert np.linalg.norm(d) <= tol * rn, (what, np.linalg.norm(d) / rn)
    assert np.abs(d).max() <= tol * rm, (what, np.abs(d).max() / rm)


def problem(nao, naux, nocc, nac, seed, L=10.0):
    B = synth.cholesky_vectors(naux, nao, L, seed=seed)
    C = synth.orbitals(nao, seed=seed)
    return B, C[:, :nocc].copy(), C[:, nocc:nocc + nac].copy()


# (nao, naux, nocc, nac); the last two have no active / no occupied orbitals, so one of the
# saved half transforms is empty (and passed as NULL)
SHAPES = [(120, 480, 30, 8), (33, 17, 5, 3), (130, 9, 17, 5), (2, 3, 1, 1), (257, 23, 20, 9),
          (6, 4, 5, 0), (6, 4, 0, 3)]


def test_vjp_tall_tiles():
    """N_ao = 500 pads to 512 rows in both tile heights, so Y_P = S X_P and the second transforms
    take the 256 x 128 tiles (ragged in every dimension)."""
    nao, naux, nocc, nac = 500, 30, 21, 6
    B, Co, Ca = problem(nao, naux, nocc, nac, seed=5)
    rng = np.random.default_rng(11)
    gJ, gK = rng.standard_normal((nao, nao)), rng.standard_normal((nao, nao))
    ge = rng.standard_normal((nac,) * 4)
    ref_o, ref_a = G.step_vjp(B, nao, Co, Ca, gJ, gK, ge)
    gB, gCo, gCa = dev(B), dev(Co), dev(Ca)
    C = synth.orbitals(nao, seed=5)                       # all 500 orbitals as p: b_pu has 500 rows
    out = dfmi.step(gB, nao, gCo, gCa, dev(C), keep_x=True)
    dCo, dCa = dfmi.step_backward(gB, nao, gCo, gCa, dev(gJ), dev(gK), dev(ge), out["Xocc"], out["Xact"])
    torch.cuda.synchronize()
    close(dCo, ref_o, what="dCocc")
    close(dCa, ref_a, what="dCact")
    close(out["papa"], O.papa(B, nao, C, Ca), what="(pu|vw) with 500 orbitals p")


@pytest.mark.parametrize("nao,naux,nocc,nac", SHAPES)
@pytest.mark.parametrize("which", ["J", "K", "eri", "all"])
@pytest.mark.parametrize("keep_x", [False, True])
def test_vjp_matches_oracle(nao, naux, nocc, nac, which, keep_x):
    B, Co, Ca = problem(nao, naux, nocc, nac, seed=nao + naux)
    rng = np.random.default_rng(7)
    gJ = rng.standard_normal((nao, nao)) if which in ("J", "all") else None
    gK = rng.standard_normal((nao, nao)) if which in ("K", "all") else None
    ge = rng.standard_normal((nac,) * 4) if which in ("eri", "all") else None
    ref_o, ref_a = G.step_vjp(B, nao, Co, Ca, gJ, gK, ge)
    gB, gCo, gCa = dev(B), dev(Co), dev(Ca)
    Xo = Xa = None
    if keep_x:
        out = dfmi.step(gB, nao, gCo, gCa, gCa[:, :0].contiguous(), keep_x=True)
        Xo, Xa = out["Xocc"], out["Xact"]
        close(Xo, O.half_transform(B, nao, Co), what="saved Xocc")
        close(Xa, O.half_transform(B, nao, Ca).transpose(1, 0, 2), what="saved Xact (AO-major)")
    d = lambda a: None if a is None else dev(a)
    dCo, dCa = dfmi.step_backward(gB, nao, gCo, gCa, d(gJ), d(gK), d(ge), Xo, Xa)
    torch.cuda.synchronize()
    close(dCo, ref_o, what=f"dCocc {which}")
    close(dCa, ref_a, what=f"dCact {which}")


def test_vjp_medium_workload():
    wl = synth.WORKLOADS["medium"]
    B = synth.cholesky_vectors(wl.naux, wl.nao, wl.L)
    C = synth.orbitals(wl.nao)
    Co, Ca = C[:, :wl.nocc].copy(), C[:, wl.nocc:wl.nocc + wl.nac].copy()
    rng = np.random.default_rng(3)
    gJ = rng.standard_normal((wl.nao, wl.nao))
    ge = rng.standard_normal((wl.nac,) * 4)
    ref_o, ref_a = G.step_vjp(B, wl.nao, Co, Ca, gJ, None, ge)
    dCo, dCa = dfmi.step_backward(dev(B), wl.nao, dev(Co), dev(Ca), dev(gJ), None, dev(ge))
    torch.cuda.synchronize()
    close(dCo, ref_o, what="dCocc")
    close(dCa, ref_a, what="dCact")
    # the exchange part against D-shaped cotangents (low rank keeps the oracle cheap):
    # gK = D/2 gives sum_P b^P D b^P C_occ = K C_occ
    D = Co @ Co.T
    dCo_k, _ = dfmi.step_backward(dev(B), wl.nao, dev(Co), dev(Ca), None, dev(0.5 * D), None)
    torch.cuda.synchronize()
    K = O.exchange(B, wl.nao, Co)
    close(dCo_k, K @ Co, what="K C_occ from the adjoint")


@pytest.mark.parametrize("scale", [0.0, 0.01])
def test_orbital_gradient_through_autograd(scale):
    nao, naux, nocc, nac = 40, 70, 9, 5
    B, C0, h, Gam = (synth.cholesky_vectors(naux, nao, 8.0, seed=2), synth.orbitals(nao, seed=2),
                     synth.symmetric_matrix(nao, seed=2), synth.two_body_density(nac, seed=2))
    kappa = scale * np.random.default_rng(11).standard_normal((nao, nao))
    ref = G.orbital_gradient(B, nao, C0, kappa, nocc, nac, h, Gam)
    e_ref = G.energy(B, nao, G.rotate(C0, kappa), nocc, nac, h, Gam)
    gB, gC0, gh, gG = dev(B), dev(C0), dev(h), dev(Gam)
    for keep_x in (True, False):
        k = dev(kappa).requires_grad_(True)
        E = dfmi.energy(gB, nao, gC0, k, nocc, nac, gh, gG, keep_x=keep_x)
        E.backward()
        torch.cuda.synchronize()
        assert abs(E.item() - e_ref) <= 1e-12 * abs(e_ref)
        close(k.grad, ref, what=f"dE/dkappa keep_x={keep_x}")


def test_orbital_gradient_finite_differences_on_gpu():
    nao, naux, nocc, nac = 30, 40, 6, 4
    B, C0, h, Gam = (synth.cholesky_vectors(naux, nao, 6.0, seed=5), synth.orbitals(nao, seed=5),
                     synth.symmetric_matrix(nao, seed=5), synth.two_body_density(nac, seed=5))
    gB, gC0, gh, gG = dev(B), dev(C0), dev(h), dev(Gam)
    k = torch.zeros((nao, nao), dtype=torch.float64, device="cuda", requires_grad=True)
    E = dfmi.energy(gB, nao, gC0, k, nocc, nac, gh, gG)
    E.backward()
    g = k.grad.detach()
    step = 1e-5
    for d in synth.directions(8, (nao, nao), seed=1):
        dd = dev(d)
        with torch.no_grad():
            ep = dfmi.energy(gB, nao, gC0, step * dd, nocc, nac, gh, gG).item()
            em = dfmi.energy(gB, nao, gC0, -step * dd, nocc, nac, gh, gG).item()
        fd = (ep - em) / (2 * step)
        lin = (g * dd).sum().item()
        assert abs(fd - lin) <= 1e-7 * max(1.0, abs(fd)), (fd, lin)
