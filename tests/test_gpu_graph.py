"""Graph capture and replay of library calls (df_batched_step, df_step, df_step_split, df_ppaa,
df_build_cholesky).

A call launches everything on the context's stream. Inside a call there is no allocation, no
memset and no host synchronisation, so a call can be captured into a HIP graph and replayed.
Each test captures once, after an eager warm-up, so the workspace is already large enough.
Then, three times, it writes new input values in place, runs the same call eagerly, replays the
graph, and requires the replay's outputs to equal the eager ones bit for bit. The kernels are
deterministic: fixed-order reductions and no atomics on floating-point values.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_03755_amd import dfmi, synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def capture(fn):
    """Warm fn up on a side stream, then capture it; returns (graph, outputs of the capture)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = fn()
    torch.cuda.synchronize()
    return g, out


def same(a, b):
    if isinstance(a, dict):
        assert a.keys() == b.keys()
        for k in a:
            same(a[k], b[k])
    elif isinstance(a, (list, tuple)):
        for x, y in zip(a, b):
            same(x, y)
    else:
        assert torch.equal(a, b)


def fragment_inputs(shapes, seed):
    out = []
    for i, (nemb, naux, nocc, nac, ndm) in enumerate(shapes):
        s = seed + i
        out.append({"B": synth.cholesky_vectors(naux, nemb, 10.0, seed=s),
                    "Cocc": synth.fragment_densities(nemb, nocc, ndm, s, seed=s),
                    "C": synth.orbitals(nemb, seed=s)})
    return out


def test_batched_step_graph_replay():
    shapes = [(33, 40, 7, 3, 3), (70, 90, 12, 4, 2), (17, 70, 4, 2, 4)]
    first = fragment_inputs(shapes, 1)
    dps = [{"B": dev(p["B"]), "nao": s[0], "Cocc": dev(p["Cocc"]), "Cact": dev(p["C"][:, s[2]:s[2] + s[3]]),
            "Cp": dev(p["C"])} for p, s in zip(first, shapes)]
    g, outs = capture(lambda: dfmi.batched_step(dps))
    for rep in range(3):
        for dp, p, s in zip(dps, fragment_inputs(shapes, 100 * (rep + 1)), shapes):
            dp["B"].copy_(dev(p["B"]))
            dp["Cocc"].copy_(dev(p["Cocc"]))
            dp["Cact"].copy_(dev(p["C"][:, s[2]:s[2] + s[3]]))
            dp["Cp"].copy_(dev(p["C"]))
        ref = dfmi.batched_step(dps)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same(outs, ref)


def step_inputs(nao, naux, nocc, nac, seed):
    B = synth.cholesky_vectors(naux, nao, 10.0, seed=seed)
    C = synth.orbitals(nao, seed=seed)
    return B, C[:, :nocc], C[:, nocc:nocc + nac], C


def test_step_graph_replay():
    nao, naux, nocc, nac = 90, 200, 20, 6
    t = [dev(a) for a in step_inputs(nao, naux, nocc, nac, 3)]
    g, out = capture(lambda: dfmi.step(t[0], nao, t[1], t[2], t[3]))
    for rep in range(3):
        for x, a in zip(t, step_inputs(nao, naux, nocc, nac, 10 + rep)):
            x.copy_(dev(a))
        ref = dfmi.step(t[0], nao, t[1], t[2], t[3])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same(out, ref)


def test_step_split_graph_replay():
    """The split-precision step (B split once per B, outside the graph)."""
    nao, naux, nocc, nac = 70, 150, 14, 5
    t = [dev(a) for a in step_inputs(nao, naux, nocc, nac, 5)]
    Bs, Be = dfmi.split_cholesky(t[0], nao, nslice=7)
    g, out = capture(lambda: dfmi.step_split(t[0], Bs, Be, nao, t[1], t[2], t[3]))
    for rep in range(3):
        for x, a in zip(t, step_inputs(nao, naux, nocc, nac, 20 + rep)):
            x.copy_(dev(a))
        Bs2, Be2 = dfmi.split_cholesky(t[0], nao, nslice=7)
        Bs.copy_(Bs2)
        Be.copy_(Be2)
        ref = dfmi.step_split(t[0], Bs, Be, nao, t[1], t[2], t[3])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same(out, ref)


def test_ppaa_graph_replay():
    nao, naux, nac = 60, 130, 5
    t = [dev(a) for a in step_inputs(nao, naux, 10, nac, 7)]
    g, out = capture(lambda: dfmi.ppaa(t[0], nao, t[3], t[2]))
    for rep in range(3):
        for x, a in zip(t, step_inputs(nao, naux, 10, nac, 30 + rep)):
            x.copy_(dev(a))
        ref = dfmi.ppaa(t[0], nao, t[3], t[2])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same(out, ref)


def build_inputs(naux, nao, seed):
    return dev(synth.coulomb_metric(naux, 1e4, seed=seed)), dev(synth.cholesky_vectors(naux, nao, 10.0, seed=seed))


def test_build_cholesky_graph_replay():
    """Forming B (out of place; the copies and the info write are part of the graph)."""
    naux, nao = 300, 20
    metric, E = build_inputs(naux, nao, 2)
    g, out = capture(lambda: dfmi.build_cholesky(metric, E, nao, check=False))
    for rep in range(3):
        m2, e2 = build_inputs(naux, nao, 40 + rep)
        metric.copy_(m2)
        E.copy_(e2)
        ref = dfmi.build_cholesky(metric, E, nao, check=False)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same(out, ref)
        assert int(out[2].item()) == 0
