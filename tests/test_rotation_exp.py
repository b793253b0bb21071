"""The orbital rotation C = C0 exp(kappa - kappa^T) of the differentiable step: the adjoint of
the exponential's Frechet derivative (dfmi.rotation_exp's backward) against SciPy's expm_frechet
(Al-Mohy and Higham's algorithm), on the CPU, at the paper's N_mo = 1200 with kappa = 0.01 N(0,1)
and a cotangent of norm ~1e6 (the size of dE/dC there)."""
import numpy as np
import pytest
import scipy.linalg

torch = pytest.importorskip("torch")

from paper_2505_03755_amd import dfmi, synth


@pytest.mark.parametrize("n, scale", [(7, 1.0), (120, 1e3), (1200, 1e3)])
def test_rotation_exp_adjoint_against_scipy(n, scale):
    kap = synth.kappa(n, seed=3)
    R = kap - kap.T
    G = np.random.default_rng(n).standard_normal((n, n)) * scale
    Rt = torch.from_numpy(R).requires_grad_(True)
    U = dfmi.rotation_exp(Rt)
    (U * torch.from_numpy(G)).sum().backward()
    ref = scipy.linalg.expm_frechet(R.T, G, compute_expm=False)
    assert np.linalg.norm(Rt.grad.numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(U.detach().numpy() - scipy.linalg.expm(R)) <= 1e-13 * np.sqrt(n)
