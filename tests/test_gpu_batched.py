"""GPU parity of the batched fragment subproblems (df_batched_step).

Each problem's outputs are checked against the FP64 oracle (normwise 1e-10) and against the
unbatched library calls on the same inputs (df_jk, df_active_eri, df_papa with DF_PAPA_FULL),
which may tile differently: 1e-12.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import df_oracle as O
from paper_2505_03755_amd import dfmi, synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def rel(a, b):
    a = a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else np.asarray(a)
    b = b.detach().cpu().numpy() if isinstance(b, torch.Tensor) else np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def make(nemb, naux, nocc, nac, ndm, seed):
    B = synth.cholesky_vectors(naux, nemb, 10.0, seed=seed)
    Cd = synth.fragment_densities(nemb, nocc, ndm, seed, seed=seed) if nocc else np.zeros((ndm, nemb, 0))
    C = synth.orbitals(nemb, seed=seed)
    return {"B": B, "nao": nemb, "Cocc": Cd, "Cact": C[:, nocc:nocc + nac], "Cp": C}


def to_dev(p):
    return {"B": dev(p["B"]), "nao": p["nao"], "Cocc": dev(p["Cocc"]), "Cact": dev(p["Cact"]), "Cp": dev(p["Cp"])}


# (nemb, naux, nocc, nac, ndm): uneven sizes straddling the tiles, a problem without occupied
# columns and one without active orbitals
RAGGED = [(33, 40, 7, 3, 3), (130, 90, 20, 5, 2), (17, 70, 4, 2, 5), (64, 64, 0, 4, 2), (70, 30, 9, 0, 3)]


def packed_uv(ref):
    """oracle (pq|uv) [p][q][u][v] -> [pair(u, v)][p][q], u >= v"""
    u, v = np.tril_indices(ref.shape[2])
    return np.ascontiguousarray(ref[:, :, u, v].transpose(2, 0, 1))


def check_problem(p, out, tol_oracle=1e-10):
    B, nao = p["B"], p["nao"]
    ndm, nocc = p["Cocc"].shape[0], p["Cocc"].shape[2]
    nac = p["Cact"].shape[1]
    for z in range(ndm):
        if nocc:
            J, K, _ = O.jk(B, nao, p["Cocc"][z])
            assert rel(out["J"][z], J) <= tol_oracle
            assert rel(out["K"][z], K) <= tol_oracle
            assert torch.equal(out["K"][z], out["K"][z].T)
        else:
            assert not out["J"][z].any() and not out["K"][z].any()
    if nac:
        eri, _ = O.active_eri(B, nao, p["Cact"])
        assert rel(out["eri"], eri) <= tol_oracle
        pf = O.papa_full(B, nao, p["Cp"], p["Cact"], p["Cp"])
        assert rel(out["papa"], pf) <= tol_oracle
        if "ppaa" in out:
            assert rel(out["ppaa"], packed_uv(O.ppaa(B, nao, p["Cp"], p["Cp"], p["Cact"]))) <= 1e-10


def test_batched_ragged_against_oracle():
    probs = [make(*shape, seed=i + 1) for i, shape in enumerate(RAGGED)]
    outs = dfmi.batched_step([to_dev(p) for p in probs])
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        check_problem(p, o)


def test_batched_ppaa_against_oracle_and_single_call():
    """(pq|uv) requested in the batch: against the oracle, and bit for bit against df_ppaa (the
    same route on the same shapes)."""
    probs = [make(*shape, seed=i + 31) for i, shape in enumerate(RAGGED)]
    dps = [to_dev(p) for p in probs]
    outs = dfmi.batched_step(dps, ppaa=True)
    torch.cuda.synchronize()
    for p, dp, o in zip(probs, dps, outs):
        check_problem(p, o)
        assert torch.equal(o["ppaa"], dfmi.ppaa(dp["B"], dp["nao"], dp["Cp"], dp["Cact"]))


def test_batched_equals_unbatched_calls():
    probs = [make(*shape, seed=i + 11) for i, shape in enumerate(RAGGED)]
    dps = [to_dev(p) for p in probs]
    outs = dfmi.batched_step(dps)
    for dp, o in zip(dps, outs):
        ndm, nocc, nac = dp["Cocc"].shape[0], dp["Cocc"].shape[2], dp["Cact"].shape[1]
        if nocc:
            J, K, _ = dfmi.jk(dp["B"], dp["nao"], dp["Cocc"])
            assert rel(o["J"], J) <= 1e-12 and rel(o["K"], K) <= 1e-12
        if nac:
            eri = dfmi.active_eri(dp["B"], dp["nao"], dp["Cact"])
            eri = eri[0] if isinstance(eri, tuple) else eri
            assert rel(o["eri"], eri) <= 1e-12
            pf = dfmi.papa(dp["B"], dp["nao"], dp["Cp"], dp["Cact"], Cq=dp["Cp"])
            assert rel(o["papa"], pf) <= 1e-12
    torch.cuda.synchronize()


def test_batched_more_than_one_group():
    """Nine problems: two grouped launches per phase."""
    shapes = [(20 + 7 * i, 30 + 5 * i, 3 + i % 3, 2 + i % 2, 2) for i in range(9)]
    probs = [make(*s, seed=100 + i) for i, s in enumerate(shapes)]
    outs = dfmi.batched_step([to_dev(p) for p in probs])
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        check_problem(p, o)


def test_fragment_workload_reduced_densities():
    """The eight fragment shapes (N_emb 80..400, N_aux = 4 N_emb) with 4 densities each."""
    probs = []
    for f in synth.FRAGMENTS:
        B, Cd, C = synth.fragment_problem(f, ndm=4)
        probs.append({"B": B, "nao": f.nemb, "Cocc": Cd, "Cact": C[:, f.nocc:f.nocc + f.nac], "Cp": C})
    outs = dfmi.batched_step([to_dev(p) for p in probs])
    torch.cuda.synchronize()
    for p, o in zip(probs[:4], outs[:4]):          # the oracle on the four smaller ones
        check_problem(p, o)
    for p, o in zip(probs[4:], outs[4:]):          # sampled densities on the larger ones
        J, K, _ = O.jk(p["B"], p["nao"], p["Cocc"][3])
        assert rel(o["J"][3], J) <= 1e-10 and rel(o["K"][3], K) <= 1e-10


def oracle_outputs(p):
    B, nao = p["B"], p["nao"]
    ndm, nocc = p["Cocc"].shape[0], p["Cocc"].shape[2]
    nac = p["Cact"].shape[1]
    out = {}
    if nocc:
        jk = [O.jk(B, nao, p["Cocc"][z]) for z in range(ndm)]
        out["J"], out["K"] = [j[0] for j in jk], [j[1] for j in jk]
    if nac:
        out["eri"] = O.active_eri(B, nao, p["Cact"])[0]
        out["papa"] = O.papa_full(B, nao, p["Cp"], p["Cact"], p["Cp"])
    return out


def close_to_oracle(o, ref, tol=1e-10):
    for z in range(len(ref.get("J", []))):
        assert rel(o["J"][z], ref["J"][z]) <= tol and rel(o["K"][z], ref["K"][z]) <= tol
        assert torch.equal(o["K"][z], o["K"][z].T)
    if "eri" in ref:
        assert rel(o["eri"], ref["eri"]) <= tol and rel(o["papa"], ref["papa"]) <= tol


def test_batched_every_candidate_configuration():
    """Every configuration the autotuner can choose gives the oracle's results."""
    probs = [make(*shape, seed=i + 31) for i, shape in enumerate(RAGGED)]
    refs = [oracle_outputs(p) for p in probs]
    dps = [to_dev(p) for p in probs]
    ctx = dfmi.context(dps[0]["B"].device)
    try:
        for half_n in (176, 96, 48, 128):
            for k_tile in (64, 128):
                for k_rounds in (16, 4, 64):
                    dfmi.batched_set_tuning(dps, half_n, k_tile, k_rounds, ctx=ctx)
                    assert dfmi.batched_tuning(dps, ctx=ctx) == {"half_tile_n": half_n, "k_tile": k_tile,
                                                                 "k_rounds": k_rounds, "tuned": True}
                    outs = dfmi.batched_step(dps, ctx=ctx)
                    torch.cuda.synchronize()
                    for o, r in zip(outs, refs):
                        close_to_oracle(o, r)
    finally:
        dfmi.batched_set_tuning(dps, 176, 64, 16, ctx=ctx)


def test_batched_autotune_fragment_workload():
    """Autotuning on the eight fragment shapes (4 densities): the first call measures and stores a
    candidate configuration, and its outputs and those of the next call match the oracle."""
    probs = []
    for f in synth.FRAGMENTS:
        B, Cd, C = synth.fragment_problem(f, ndm=4)
        probs.append({"B": B, "nao": f.nemb, "Cocc": Cd, "Cact": C[:, f.nocc:f.nocc + f.nac], "Cp": C})
    dps = [to_dev(p) for p in probs]
    ctx = dfmi.context(dps[0]["B"].device)
    assert not dfmi.batched_tuning(dps, ctx=ctx)["tuned"]
    ctx.set_autotune(True)
    try:
        first = dfmi.batched_step(dps, ctx=ctx)
    finally:
        ctx.set_autotune(False)
    t = dfmi.batched_tuning(dps, ctx=ctx)
    assert t["tuned"] and t["half_tile_n"] in (176, 96, 48, 128) and t["k_tile"] in (64, 128)
    assert t["k_rounds"] in (16, 4, 64)
    second = dfmi.batched_step(dps, ctx=ctx)
    torch.cuda.synchronize()
    for a, b in zip(first, second):
        for k in a:
            assert torch.equal(a[k], b[k])
    for p, o in zip(probs[:3], first[:3]):
        close_to_oracle(o, oracle_outputs(p))
    J, K, _ = O.jk(probs[7]["B"], probs[7]["nao"], probs[7]["Cocc"][2])
    assert rel(first[7]["J"][2], J) <= 1e-10 and rel(first[7]["K"][2], K) <= 1e-10


def with_split(dps, S=7):
    for dp in dps:
        dp["Bs"], dp["Be"] = dfmi.split_cholesky(dp["B"], dp["nao"], nslice=S)
    return dps


@pytest.mark.parametrize("k_fp64", [False, True])
def test_batched_split_ragged_against_oracle(k_fp64):
    """Split precision (7 slices) against the oracle and against the FP64 batch; K from int8 slices
    or, with k_fp64, in FP64 from the split-precision X_occ."""
    probs = [make(*shape, seed=i + 51) for i, shape in enumerate(RAGGED)]
    dps = with_split([to_dev(p) for p in probs])
    outs = dfmi.batched_step_split(dps, k_fp64=k_fp64, ppaa=k_fp64)
    ref = dfmi.batched_step(dps, ppaa=k_fp64)
    torch.cuda.synchronize()
    for p, o, r in zip(probs, outs, ref):
        check_problem(p, o, tol_oracle=1e-11)
        for k in o:
            assert rel(o[k], r[k]) <= 1e-11, k


def test_batched_split_fragment_workload_reduced_densities():
    """The eight fragment shapes with 4 densities each: oracle on the smaller ones, a sampled
    density of the larger ones."""
    probs = []
    for f in synth.FRAGMENTS:
        B, Cd, C = synth.fragment_problem(f, ndm=4)
        probs.append({"B": B, "nao": f.nemb, "Cocc": Cd, "Cact": C[:, f.nocc:f.nocc + f.nac], "Cp": C})
    outs = dfmi.batched_step_split(with_split([to_dev(p) for p in probs]))
    torch.cuda.synchronize()
    for p, o in zip(probs[:3], outs[:3]):
        check_problem(p, o, tol_oracle=1e-11)
    for p, o in zip(probs[6:], outs[6:]):
        J, K, _ = O.jk(p["B"], p["nao"], p["Cocc"][1])
        assert rel(o["J"][1], J) <= 1e-11 and rel(o["K"][1], K) <= 1e-11


def test_fragment_shapes_with_ppaa():
    """The eight fragment shapes (one density each) with (pq|uv): the oracle on the three
    smallest, df_ppaa of the same problem on the rest (bitwise)."""
    probs = []
    for f in synth.FRAGMENTS:
        B, Cd, C = synth.fragment_problem(f, ndm=1)
        probs.append({"B": B, "nao": f.nemb, "Cocc": Cd, "Cact": C[:, f.nocc:f.nocc + f.nac], "Cp": C})
    dps = [to_dev(p) for p in probs]
    outs = dfmi.batched_step(dps, ppaa=True)
    torch.cuda.synchronize()
    for p, o in zip(probs[:3], outs[:3]):
        assert rel(o["ppaa"], packed_uv(O.ppaa(p["B"], p["nao"], p["Cp"], p["Cp"], p["Cact"]))) <= 1e-10
    for dp, o in zip(dps[3:], outs[3:]):
        assert torch.equal(o["ppaa"], dfmi.ppaa(dp["B"], dp["nao"], dp["Cp"], dp["Cact"]))


# The fragment workload as the benchmark times it: 64 densities per problem.  The oracle covers
# every density of the three smallest problems and densities 0, 31 and 63 of the others.
SAMPLED_Z = (0, 31, 63)


def fragment_probs(ndm):
    probs = []
    for f in synth.FRAGMENTS:
        B, Cd, C = synth.fragment_problem(f, ndm=ndm)
        probs.append({"B": B, "nao": f.nemb, "Cocc": Cd, "Cact": C[:, f.nocc:f.nocc + f.nac], "Cp": C})
    return probs


@pytest.fixture(scope="module")
def frag64():
    probs = fragment_probs(64)
    refs = []
    for i, p in enumerate(probs):
        zs = list(range(64)) if i < 3 else list(SAMPLED_Z)
        J, K, _ = O.jk_many(p["B"], p["nao"], [p["Cocc"][z] for z in zs])
        jk = {z: (J[k], K[k]) for k, z in enumerate(zs)}
        refs.append({"jk": jk, "eri": O.active_eri(p["B"], p["nao"], p["Cact"])[0],
                     "papa": O.papa_full(p["B"], p["nao"], p["Cp"], p["Cact"], p["Cp"])})
    return probs, [to_dev(p) for p in probs], refs


def check_frag64(outs, refs, tol):
    for i, (o, r) in enumerate(zip(outs, refs)):
        for z, (J, K) in r["jk"].items():
            assert rel(o["J"][z], J) <= tol, (i, z)
            assert rel(o["K"][z], K) <= tol, (i, z)
            assert torch.equal(o["K"][z], o["K"][z].T)
        assert rel(o["eri"], r["eri"]) <= tol, i
        assert rel(o["papa"], r["papa"]) <= tol, i


def test_fragment_workload_64_densities(frag64):
    """The benchmarked fragment batch (J of 64 densities through V B^T, K of each) in FP64."""
    probs, dps, refs = frag64
    outs = dfmi.batched_step(dps)
    torch.cuda.synchronize()
    check_frag64(outs, refs, 1e-10)


def test_fragment_workload_64_densities_2d_tiles(frag64):
    """The same batch with the half transforms on the 2-D tiling (tuning candidate 128: 128 x 128
    tiles, each fragment's rows past its last whole 128-row band on 64 x 176 tiles where that pads
    less), in a context of its own."""
    probs, dps, refs = frag64
    ctx = dfmi.Context(dps[0]["B"].device)
    dfmi.batched_set_tuning(dps, 128, 64, 16, ctx=ctx)
    outs = dfmi.batched_step(dps, ctx=ctx)
    torch.cuda.synchronize()
    check_frag64(outs, refs, 1e-10)


@pytest.mark.parametrize("k_fp64", [False, True])
def test_fragment_workload_64_densities_split(frag64, k_fp64):
    """The same batch in split precision (7 slices), K from int8 slices or in FP64."""
    probs, dps, refs = frag64
    outs = dfmi.batched_step_split(with_split(dps), k_fp64=k_fp64)
    torch.cuda.synchronize()
    check_frag64(outs, refs, 1e-11)


def test_autotune_choice_persists_through_the_cache_file(tmp_path, monkeypatch):
    """With DFMI_AUTOTUNE_CACHE set, a tuning call writes its choice (tagged with the device's gfx
    architecture) to the file, and a context created afterwards uses it without measuring."""
    import json
    path = tmp_path / "tune.json"
    monkeypatch.setenv("DFMI_AUTOTUNE_CACHE", str(path))
    # (batched_tuning reads a group's shape with every output requested: no empty ones here)
    probs = [make(*shape, seed=i + 71) for i, shape in enumerate(RAGGED[:3])]
    dps = [to_dev(p) for p in probs]
    a = dfmi.Context(0)
    a.set_autotune(True)
    outs = dfmi.batched_step(dps, ctx=a)
    torch.cuda.synchronize()
    t = dfmi.batched_tuning(dps, ctx=a)
    assert t["tuned"]
    doc = json.load(open(path))
    (e,) = doc["entries"]
    assert e["arch"].startswith("gfx") and e["op"] == "df_batched_step"
    assert (e["half_tile_n"], e["k_tile"], e["k_rounds"]) == (t["half_tile_n"], t["k_tile"], t["k_rounds"])
    b = dfmi.Context(0)                      # autotuning off: uses the file's choice
    assert dfmi.batched_tuning(dps, ctx=b) == t
    again = dfmi.batched_step(dps, ctx=b)
    torch.cuda.synchronize()
    for o1, o2 in zip(outs, again):
        for k in o1:
            assert torch.equal(o1[k], o2[k]), k
    for p, o in zip(probs, outs):
        check_problem(p, o)
    a.close()
    b.close()
