#!/usr/bin/env python3
"""Benchmark of the density-fitted contraction step on one MI355X.

One step = one pass of the whole hot path at paper scale (N_ao = 1200, N_aux = 4800,
N_occ = 300, N_ac = 40, N_mo = 1200, B = 27.7 GB packed FP64):
  forward  (df_step): the shared half transform X = b^P [C_occ | C_act], the J-vector and J,
           K, the second transform b^P_{pu}, (uv|wx) and (pu|vw), keeping X for the adjoint;
  adjoint  (df_step_backward): the vector-Jacobian product of (J, K, (uv|wx)) with respect to
           (C_occ, C_act) for the cotangents of the model energy
           E = tr(D h) + 1/2 tr(D J) - 1/4 tr(D K) + 1/2 sum (uv|wx) Gamma,
           i.e. gJ = D/2, gK = -D/4, g_eri = Gamma/2 (the contraction part of dE/dkappa).
Inputs are drawn on the GPU and are resident in HBM before the timed region starts.

Prints one JSON line with the step throughput (algorithmic TFLOP/s), the roofline figure
of the dominant kernel (live HIP-event timing on the library's stream) and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6     # MI355X dense FP64 matrix peak (published)
PEAK_HBM_GBS = 8000.0            # MI355X HBM3E (published)
METRIC = "DF J/K+papa step ms & TFLOP/s at N_ao=1200; split-prec vs FP64 @ΔE≤1e-8"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_flops(naux, nao, nocc, nac, nmo, adjoint=True):
    """Algorithmic FP64 FLOPs of one step: forward (half, J, K, b_pu, (pu|vw)) and the generic
    adjoint (J part 4 N_aux npair + 2 N_ao^2 N_occ, K part 4 N_aux N_ao^2 N_occ, eri part
    2 N_aux N_ac^4 + 2 N_aux N_ao N_ac^2)."""
    npair = nao * (nao + 1) // 2
    f = {
        "half_transform": 2 * naux * nao * nao * (nocc + nac),
        "j": 2 * naux * nao * nocc + 2 * naux * npair,
        "k_syrk": naux * nocc * nao * (nao + 1),
        "mo_transform": 2 * naux * nao * nmo * nac,
        "papa": 2 * naux * nmo * nac ** 3,
    }
    if adjoint:
        f["adjoint"] = (4 * naux * npair + 2 * nao * nao * nocc + 4 * naux * nao * nao * nocc
                        + 2 * naux * nac ** 4 + 2 * naux * nao * nac * nac)
    return f


def kernel_source_digest() -> str:
    """sha256 of the kernel sources: HBM byte counts are valid only for the kernels they came from."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2505_03755_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_per_launch(kernel: str):
    """Scaled HBM bytes (fetch + write) per launch of `kernel`, from the committed rocprofv3 counter
    summary, or None when there is none or it was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_paper_hbm_bytes.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel sources sha256") != kernel_source_digest():
        return None
    try:
        return float(fields["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def kernel_table(kt, naux, nao, nocc, nac, nmo, steps):
    """Per-kernel time per step and its roofline figure."""
    npair = nao * (nao + 1) // 2
    ncol = nocc + nac
    algo = {  # (kind of bound, algorithmic amount per step)
        "half_transform": ("mfma", 2 * naux * nao * nao * ncol),
        "k_syrk": ("mfma", naux * nocc * nao * (nao + 1)),
        "mo_transform": ("mfma", 2 * naux * nao * nmo * nac + 2 * naux * nao * nac * nac),
        "papa": ("mfma", 2 * naux * nmo * nac ** 3),
        "eri": ("mfma", 2 * naux * nac ** 4),
        "adjoint": ("mfma", 4 * naux * nao * nao * nocc + 2 * nao * nao * nocc + 2 * naux * nac ** 4
                    + 2 * naux * nao * nac * nac),
        # HBM-bound kernels: bytes read + written
        # the forward J-vector comes out of the half transform's epilogue; the adjoint's reads B
        # once; each Coulomb build streams B
        "jvec": ("hbm", 8 * (naux * npair + npair + naux)),
        "coulomb": ("hbm", 2 * 8 * (naux * npair + naux + 2 * nao * nao)),
        "k_reduce": ("hbm", None),
        "other": ("hbm", None),
    }
    out = {}
    for k, (ms, n) in kt.items():
        if n == 0:
            continue
        bound, amount = algo.get(k, ("hbm", None))
        row = {"ms_per_step": ms / steps, "launches_per_step": n / steps}
        if amount is not None and ms > 0:
            per_s = amount / (ms / steps * 1e-3)
            if bound == "mfma":
                row["tflops"] = per_s / 1e12
                row["frac_fp64_peak"] = per_s / 1e12 / PEAK_FP64_MFMA_TFLOPS
            else:
                row["gbs"] = per_s / 1e9
                row["frac_hbm_peak"] = per_s / 1e9 / PEAK_HBM_GBS
        out[k] = row
    return out


def cpu_baseline(wl, rows, seed, adjoint=True):
    """The FP64 oracle on `rows` auxiliary rows of the same workload (host cores): the forward
    outputs and, with `adjoint`, the vector-Jacobian product for the model-energy cotangents."""
    import numpy as np
    from oracle import df_grad as G
    from oracle import df_oracle as O
    from paper_2505_03755_amd import synth
    try:
        from threadpoolctl import threadpool_info
        blas = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        threads = max([i.get("num_threads", 1) for i in blas] or [1])
        vendor = ", ".join(f"{i.get('internal_api')} {i.get('version')} ({i.get('architecture')})" for i in blas)
    except Exception:
        threads, vendor = os.cpu_count() or 1, "unknown"
    B = synth.cholesky_vectors(rows, wl.nao, wl.L, seed=seed)
    C = synth.orbitals(wl.nao, seed=seed)
    Cocc, Cact = C[:, :wl.nocc], C[:, wl.nocc:wl.nocc + wl.nac]
    D = Cocc @ Cocc.T
    Gam = synth.two_body_density(wl.nac, seed=seed)
    t0 = time.perf_counter()
    J, K, v = O.jk(B, wl.nao, Cocc)
    eri, _ = O.active_eri(B, wl.nao, Cact)
    pa = O.papa(B, wl.nao, C, Cact)
    outs = [J, K, eri, pa]
    if adjoint:
        outs += list(G.step_vjp(B, wl.nao, Cocc, Cact, 0.5 * D, -0.25 * D, 0.5 * Gam))
    dt = time.perf_counter() - t0
    fl = sum(step_flops(rows, wl.nao, wl.nocc, wl.nac, wl.nmo, adjoint=adjoint).values())
    assert all(np.isfinite(o).all() for o in outs)
    what = "forward J, K, v, (uv|wx), (pu|vw)" + (" + adjoint" if adjoint else "")
    return {"value": fl / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle", "blas": vendor,
            "sample": f"{rows} of {wl.naux} auxiliary rows at N_ao={wl.nao}, N_occ={wl.nocc}, N_ac={wl.nac} "
                      f"({what}; rate in algorithmic FP64 FLOP/s of that sample); {dt:.2f} s"}


# rows of K and of (pu|vw) the oracle check compares entry by entry (K C_occ and the rest in full)
K_ROWS = (0, 1, 150, 299, 600, 1000, 1198, 1199)
P_ROWS = (0, 1, 299, 300, 320, 339, 340, 777, 1199)


def snapshot(o, Cocc, E):
    """Host copies of a forward step's outputs that the oracle check compares."""
    nao = Cocc.shape[0]
    kr = [r for r in K_ROWS if r < nao]
    pr = [r for r in P_ROWS if r < o["papa"].shape[0]]
    return {"J": o["J"].cpu().numpy(), "v": o["v"].cpu().numpy(), "eri": o["eri"].cpu().numpy(),
            "K_rows": o["K"][kr].cpu().numpy(), "KC": (o["K"] @ Cocc).cpu().numpy(),
            "papa_rows": o["papa"][pr].cpu().numpy(), "E": E}


def split_comparison(B, nao, Cocc, Cact, C, nslice, reps, ctx):
    """Forward step in FP64 (df_step) and in split precision (df_step_split, nslice int8 slices),
    timed alone with HIP events on the library's stream, and the model energy from both; then the
    adjoint for the model-energy cotangents in FP64 (df_step_backward) and in split precision
    (df_step_backward_split), timed the same way, with the difference of the gradients."""
    import math
    import torch
    from paper_2505_03755_amd import dfmi, synth
    dev = B.device
    nac = Cact.shape[1]
    Bs, Be = dfmi.split_cholesky(B, nao, nslice=nslice, ctx=ctx)     # once per B, not timed
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        out = fn(None)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for i in range(reps):
            fn(out)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))
        return out, ms[len(ms) // 2]

    ref, ms64 = timed(lambda o: dfmi.step(B, nao, Cocc, Cact, C, outputs=o, ctx=ctx))
    spl, mss = timed(lambda o: dfmi.step_split(B, Bs, Be, nao, Cocc, Cact, C, outputs=o, ctx=ctx))
    h = torch.from_numpy(synth.symmetric_matrix(nao)).to(dev)
    Gam = torch.from_numpy(synth.two_body_density(nac)).to(dev)
    D = Cocc @ Cocc.T

    def energy(o):
        return math.fsum([(D * h).sum().item(), 0.5 * (D * o["J"]).sum().item(),
                          -0.25 * (D * o["K"]).sum().item(), 0.5 * (o["eri"] * Gam).sum().item()])

    e64, es = energy(ref), energy(spl)
    rel = {k: ((spl[k] - ref[k]).norm() / ref[k].norm()).item() for k in ("J", "K", "v", "eri", "papa")}
    host = {name: snapshot(o, Cocc, E) for name, o, E in (("fp64", ref, e64), ("split", spl, es))}
    del ref, spl
    # the adjoint for the model-energy cotangents (gJ = D/2, gK = -D/4, geri = Gamma/2), each
    # path on the factors its own forward kept
    gJ, gK, ge = (0.5 * D).contiguous(), (-0.25 * D).contiguous(), (0.5 * Gam).contiguous()
    xs = dfmi.step_split(B, Bs, Be, nao, Cocc, Cact, C, keep_x=True, ctx=ctx)
    del Bs, Be
    Bt, Bte = dfmi.split_cholesky_t(B, nao, nslice=nslice, ctx=ctx)   # once per B, not timed
    x64 = dfmi.step(B, nao, Cocc, Cact, C, keep_x=True, ctx=ctx)
    g64, bms64 = timed(lambda o: dfmi.step_backward(B, nao, Cocc, Cact, gJ, gK, ge, x64["Xocc"], x64["Xact"],
                                                    ctx=ctx))
    gs, bmss = timed(lambda o: dfmi.step_backward_split(B, Bt, Bte, nao, Cocc, Cact, gJ, gK, ge, xs["Xocc"],
                                                        xs["Xact"], ctx=ctx))
    grel = {name: ((a - b).norm() / b.norm()).item() for name, a, b in (("dCocc", gs[0], g64[0]),
                                                                       ("dCact", gs[1], g64[1]))}
    for name, g in (("fp64", g64), ("split", gs)):
        host[name]["dCocc"], host[name]["dCact"] = g[0].cpu().numpy(), g[1].cpu().numpy()
    del xs, x64, Bt, Bte, g64, gs
    torch.cuda.empty_cache()
    return {"nslice": nslice, "forward_ms_fp64": ms64, "forward_ms_split": mss, "speedup": ms64 / mss,
            "E_fp64": e64, "dE_split_minus_fp64": es - e64, "dE_bar": 1e-8, "meets_bar": abs(es - e64) <= 1e-8,
            "rel_diff": rel, "adjoint_ms_fp64": bms64, "adjoint_ms_split": bmss,
            "adjoint_speedup": bms64 / bmss, "gradient_rel_diff": grel}, host


def oracle_check(B, wl, host, chunk=96):
    """Part of the CPU-baseline leg: the FP64 oracle's one pass over all of B at paper scale (the
    rows copied from the device block by block; oracle/df_stream.py), and the error of the FP64 and
    the split-precision GPU results against it: the model energy E and every output of the timed
    step (J, v, rows of K, K C_occ, (uv|wx), rows of (pu|vw), and the gradient dC)."""
    import math
    import numpy as np
    from oracle import df_stream as S
    from paper_2505_03755_amd import synth
    C = synth.orbitals(wl.nao, seed=wl.seed)
    h = synth.symmetric_matrix(wl.nao, seed=wl.seed)
    Gam = synth.two_body_density(wl.nac, seed=wl.seed)
    kr = [r for r in K_ROWS if r < wl.nao]
    pr = [r for r in P_ROWS if r < wl.nmo]

    def chunks():
        for p0 in range(0, B.shape[0], chunk):
            yield p0, B[p0:p0 + chunk].cpu().numpy()

    t0 = time.perf_counter()
    r = S.step_pass(chunks(), wl.naux, wl.nao, C, wl.nocc, wl.nac, h, Gam, p_rows=pr, k_rows=kr)
    dt = time.perf_counter() - t0
    Cocc = C[:, :wl.nocc]
    ref = {"J": r["J"], "v": r["v"], "K_rows": r["K_rows"], "KC": r["KC"], "eri": r["eri"],
           "papa_rows": r["papa_rows"],
           # the adjoint for the model-energy cotangents: (J - K/2) C_occ and dE/dC_act
           "dCocc": r["J"] @ Cocc - 0.5 * r["KC"], "dCact": r["G"][:, wl.nocc:wl.nocc + wl.nac]}

    def relerr(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {"E_oracle": r["E"], "oracle_pass_s": dt, "dE_bar": 1e-8,
           "outputs": "J and v in full, rows " + ",".join(map(str, kr)) + " of K, K C_occ, (uv|wx), rows "
                      + ",".join(map(str, pr)) + " of (pu|vw), dC_occ and dC_act (normwise relative errors)"}
    for name, g in host.items():
        dE = g["E"] - r["E"]
        out[name] = {"dE": dE, "dE_rel": abs(dE) / abs(r["E"]), "meets_bar": abs(dE) <= 1e-8,
                     "rel_err": {k: relerr(g[k], ref[k]) for k in ref}}
    return out


def recompute_block(B, nao, Cocc, Cact, C, gJ, gK, geri, reps, ctx, limits=(0, 8 << 30)):
    """The step with the half transforms recomputed in the adjoint instead of kept: df_step without
    X, then df_step_backward forming X again (in one piece, and in P chunks under a scratch limit),
    timed with HIP events on the library's stream."""
    import torch
    from paper_2505_03755_amd import dfmi
    naux = B.shape[0]
    nocc, nac, nmo = Cocc.shape[1], Cact.shape[1], C.shape[1]
    stream = torch.cuda.current_stream(B.device)
    out = dfmi.step(B, nao, Cocc, Cact, C, ctx=ctx)
    fl = sum(step_flops(naux, nao, nocc, nac, nmo).values()) + 2 * naux * nao * nao * (nocc + nac)
    res = {"flops_per_step": fl}
    for lim in limits:
        ctx.set_scratch_limit(lim)
        try:
            def run():
                dfmi.step(B, nao, Cocc, Cact, C, outputs=out, ctx=ctx)
                dfmi.step_backward(B, nao, Cocc, Cact, gJ, gK, geri, ctx=ctx)
            run()
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
            ev[0].record(stream)
            for i in range(reps):
                run()
                ev[i + 1].record(stream)
            torch.cuda.synchronize()
            ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))[reps // 2]
            rows = ctx.backward_chunk(naux=naux, nao=nao, nocc=nocc, nac=nac,
                                      flags=dfmi.DF_BWD_GJ | dfmi.DF_BWD_GK | dfmi.DF_BWD_GERI)
        finally:
            ctx.set_scratch_limit(0)
        key = "no_limit" if lim == 0 else f"limit_{lim >> 30}GiB"
        res[key] = {"ms": ms, "tflops": fl / ms / 1e9, "chunk_rows": rows, "chunks": -(-naux // rows)}
        torch.cuda.empty_cache()
    del out
    torch.cuda.empty_cache()
    return res


def ppaa_block(B, nao, Cact, C, reps, ctx):
    """(pq|uv) of Eq. (ppaa) with p, q over all MOs (df_ppaa, through the AO basis), timed alone
    with HIP events on the library's stream, then once more with per-kernel timing."""
    import torch
    from paper_2505_03755_amd import dfmi
    naux = B.shape[0]
    nac, nmo = Cact.shape[1], C.shape[1]
    npair, nuv = nao * (nao + 1) // 2, nac * (nac + 1) // 2
    stream = torch.cuda.current_stream(B.device)
    out = dfmi.ppaa(B, nao, C, Cact, ctx=ctx)
    del out
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        out = dfmi.ppaa(B, nao, C, Cact, ctx=ctx)
        del out
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))[reps // 2]
    ctx.set_timing(True)
    ctx.timing_read()
    out = dfmi.ppaa(B, nao, C, Cact, ctx=ctx)
    kt = ctx.timing_read()
    ctx.set_timing(False)
    del out
    torch.cuda.empty_cache()
    # the AO route's work: W_uv over the packed pairs, then C^T W_uv C
    fl_w = 2 * naux * npair * nuv
    fl_t = 2 * nuv * nao * nmo * (nao + nmo)
    fl_mo = 2 * naux * nao * nmo * (nao + nmo) + 2 * naux * nmo * nmo * nuv
    names = {"papa": "w_product", "half_transform": "half_transform", "mo_transform": "second_transform"}
    return {"shape": f"N_ao={nao}, N_aux={naux}, N_mo={nmo}, N_ac={nac}; out [{nuv}][{nmo}][{nmo}]",
            "ms": ms, "flops": fl_w + fl_t, "tflops": (fl_w + fl_t) / ms / 1e9,
            "flops_mo_route": fl_mo,
            "kernels_ms": {names.get(k, k): v[0] for k, v in kt.items() if v[1] > 0}}


def build_block(naux, nao, reps, ctx):
    """df_build_cholesky at N_aux x N_ao: the metric factored and B = L^-1 E formed (E drawn on the
    GPU, the metric on the host, neither timed), timed with HIP events on the library's stream."""
    import torch
    from paper_2505_03755_amd import dfmi, synth
    dev = torch.device("cuda", 0)
    metric = torch.from_numpy(synth.coulomb_metric(naux, 1e6, seed=11)).to(dev)
    E = synth.device_cholesky_vectors(naux, nao, 40.0, seed=12, device=dev)
    stream = torch.cuda.current_stream(dev)
    L, B, info = dfmi.build_cholesky(metric, E, nao, ctx=ctx)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        dfmi.build_cholesky(metric, E, nao, check=False, ctx=ctx)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))[reps // 2]
    ctx.set_timing(True)
    ctx.timing_read()
    dfmi.build_cholesky(metric, E, nao, check=False, ctx=ctx)
    kt = ctx.timing_read()
    ctx.set_timing(False)
    ok = int(info.item()) == 0
    del L, B, E, metric, info
    torch.cuda.empty_cache()
    npair = nao * (nao + 1) // 2
    fl = naux ** 3 / 3 + naux * naux * npair
    return {"shape": f"N_aux={naux}, N_ao={nao}; metric condition 1e6", "ms": ms, "flops": fl,
            "tflops": fl / ms / 1e9, "info_ok": ok,
            "kernels_ms": {k: v[0] for k, v in kt.items() if v[1] > 0}}


def fragment_flops(f, ndm):
    """Algorithmic FLOPs of one fragment subproblem: half transform, J, K, b_pu and the full
    (pu|qv), and (uv|wx)."""
    n, naux, nocc, nac = f.nemb, f.naux, f.nocc, f.nac
    npair = n * (n + 1) // 2
    return (2 * naux * n * n * (ndm * nocc + nac) + ndm * (2 * naux * n * nocc + 2 * naux * npair)
            + ndm * naux * nocc * n * (n + 1) + 2 * naux * n * n * nac + 2 * naux * (n * nac) ** 2
            + 2 * naux * n * nac * nac + 2 * naux * nac ** 4)


def batched_fragments(ndm, reps, ctx, nslice=7):
    """The eight fragment subproblems with ndm densities each: df_batched_step (grouped launches)
    with its default tiles, autotuned, and the tuned call replayed from a HIP graph, against the
    same work issued problem by problem (df_jk, df_active_eri, df_papa FULL); then the batch in
    split precision (df_batched_step_split, nslice slices; K from slices, and K kept in FP64) with
    its largest difference to FP64."""
    import numpy as np
    import torch
    from paper_2505_03755_amd import dfmi, synth
    dev = torch.device("cuda", 0)
    probs = []
    for f in synth.FRAGMENTS:
        B, Cd, C = synth.fragment_problem(f, ndm=ndm)
        probs.append({"B": torch.from_numpy(B).to(dev), "nao": f.nemb, "Cocc": torch.from_numpy(Cd).to(dev),
                      "Cact": torch.from_numpy(np.ascontiguousarray(C[:, f.nocc:f.nocc + f.nac])).to(dev),
                      "Cp": torch.from_numpy(C).to(dev)})
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for i in range(reps):
            fn()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))
        return ms[len(ms) // 2]

    def unbatched():
        for p in probs:
            dfmi.jk(p["B"], p["nao"], p["Cocc"], want_v=False, ctx=ctx)
            dfmi.active_eri(p["B"], p["nao"], p["Cact"], ctx=ctx)
            dfmi.papa(p["B"], p["nao"], p["Cp"], p["Cact"], Cq=p["Cp"], ctx=ctx)

    ms_default = timed(lambda: dfmi.batched_step(probs, ctx=ctx))
    # the autotuner measures its candidates on the first call of this group shape
    ctx.set_autotune(True)
    t0 = time.perf_counter()
    dfmi.batched_step(probs, ctx=ctx)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    ctx.set_autotune(False)
    tuning = dfmi.batched_tuning(probs, ctx=ctx)
    ms_b = timed(lambda: dfmi.batched_step(probs, ctx=ctx))
    # the tuned call captured once into a HIP graph and replayed
    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        dfmi.batched_step(probs, ctx=ctx)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        dfmi.batched_step(probs, ctx=ctx)
    ms_g = timed(graph.replay)
    del graph
    ms_u = timed(unbatched)
    # the same batch with (pq|uv) of every fragment added (p, q over all its MOs)
    ms_pp = timed(lambda: dfmi.batched_step(probs, ppaa=True, ctx=ctx))
    # split precision: each fragment's B split once (not timed), then df_batched_step_split
    ref = dfmi.batched_step(probs, ctx=ctx)
    for p in probs:
        p["Bs"], p["Be"] = dfmi.split_cholesky(p["B"], p["nao"], nslice=nslice, ctx=ctx)
    split = {"nslice": nslice}
    for name, kf in (("", False), ("k_fp64_", True)):
        ms_s = timed(lambda: dfmi.batched_step_split(probs, nslice=nslice, k_fp64=kf, ctx=ctx))
        spl = dfmi.batched_step_split(probs, nslice=nslice, k_fp64=kf, ctx=ctx)
        torch.cuda.synchronize()
        split[name + "ms_batched"] = ms_s
        split[name + "speedup_vs_fp64"] = ms_b / ms_s
        split[name + "max_rel_diff_vs_fp64"] = {
            k: max(((o[k] - r[k]).norm() / r[k].norm()).item() for o, r in zip(spl, ref)) for k in ("J", "K", "eri", "papa")}
        del spl
    del ref
    fl = sum(fragment_flops(f, ndm) for f in synth.FRAGMENTS)
    del probs
    torch.cuda.empty_cache()
    return {"workload": "8 fragment subproblems, N_emb 80..400, N_aux = 4 N_emb, N_occ = N_emb/4, "
                        f"N_ac 4..8, {ndm} densities each; J, K, (uv|wx), full (pu|qv)",
            "flops": fl, "ms_batched": ms_b, "tflops_batched": fl / ms_b / 1e9,
            "tuning": {k: tuning[k] for k in ("half_tile_n", "k_tile", "k_rounds")}, "tuning_call_s": tune_s,
            "ms_batched_default_tiles": ms_default, "ms_graph_replay": ms_g,
            "ms_unbatched": ms_u, "tflops_unbatched": fl / ms_u / 1e9,
            "ms_batched_with_ppaa": ms_pp,
            "split": split}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="paper", choices=["tiny", "medium", "paper"])
    ap.add_argument("--cpu-rows", type=int, default=24, help="auxiliary rows in the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forward-only", action="store_true", help="time df_step alone (no adjoint)")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched fragment workload")
    ap.add_argument("--no-ppaa", action="store_true", help="skip the (pq|uv) block")
    ap.add_argument("--no-build", action="store_true", help="skip forming B from the metric")
    ap.add_argument("--no-recompute", action="store_true", help="skip the step with X recomputed in the adjoint")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the oracle's full pass over B (errors of the GPU results against it)")
    ap.add_argument("--fragment-densities", type=int, default=64)
    ap.add_argument("--split-slices", type=int, default=7)
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="copy this many MiB device-to-device once before the steps (a known-size "
                         "reference for the HBM byte counters of a profiling run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path would shard "
              "over the auxiliary index, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2505_03755_amd import dfmi, synth

    wl = synth.WORKLOADS[args.workload]
    naux, nao, nocc, nac, nmo = wl.naux, wl.nao, wl.nocc, wl.nac, wl.nmo
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"[bench] generating inputs on the GPU: {wl}")
    t0 = time.perf_counter()
    B = synth.device_cholesky_vectors(naux, nao, wl.L, seed=wl.seed, device=dev)
    C = torch.from_numpy(synth.orbitals(nao, seed=wl.seed)).to(dev)
    Cocc = C[:, :nocc].contiguous()
    Cact = C[:, nocc:nocc + nac].contiguous()
    # cotangents of the model energy: gJ = D/2, gK = -D/4, g_eri = Gamma/2
    D = Cocc @ Cocc.T
    gJ = (0.5 * D).contiguous()
    gK = (-0.25 * D).contiguous()
    geri = (0.5 * torch.from_numpy(synth.two_body_density(nac, seed=wl.seed)).to(dev)).contiguous()
    del D
    torch.cuda.synchronize()
    log(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s (B {B.numel() * 8 / 1e9:.2f} GB)")

    ctx = dfmi.context(dev)
    out = {
        "J": torch.empty((nao, nao), dtype=torch.float64, device=dev),
        "K": torch.empty((nao, nao), dtype=torch.float64, device=dev),
        "v": torch.empty((naux,), dtype=torch.float64, device=dev),
        "eri": torch.empty((nac,) * 4, dtype=torch.float64, device=dev),
        "papa": torch.empty((nmo, nac, nac, nac), dtype=torch.float64, device=dev),
    }
    if not args.forward_only:
        out["Xocc"] = torch.empty((naux, nao, nocc), dtype=torch.float64, device=dev)
        out["Xact"] = torch.empty((nao, naux, nac), dtype=torch.float64, device=dev)
    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] calibration copy of {args.calibration_copy_mib} MiB done")
    def run():
        dfmi.step(B, nao, Cocc, Cact, C, outputs=out, ctx=ctx)
        if not args.forward_only:
            dfmi.step_backward(B, nao, Cocc, Cact, gJ, gK, geri, out["Xocc"], out["Xact"], ctx=ctx)
    for i in range(args.warmup):
        run()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")

    ctx.set_timing(True)
    ctx.timing_read()
    stream = torch.cuda.current_stream(dev)    # the stream the library launches on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        run()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
    kt = ctx.timing_read()
    ctx.set_timing(False)
    log(f"[bench] {args.steps} timed steps in {dt:.3f} s")

    fl = step_flops(naux, nao, nocc, nac, nmo, adjoint=not args.forward_only)
    w_alg = sum(fl.values())
    ms = dt / args.steps * 1e3
    value = w_alg / (dt / args.steps) / 1e12
    kernels = kernel_table(kt, naux, nao, nocc, nac, nmo, args.steps)
    half = kernels["half_transform"]
    roof = {
        "kernel": "half_transform",
        "bound": "mfma",
        "achieved": half["tflops"],
        "peak": PEAK_FP64_MFMA_TFLOPS,
        "unit": "TFLOP/s",
        "frac": half["tflops"] / PEAK_FP64_MFMA_TFLOPS,
        "traffic": traffic_per_launch("half_transform"),
        "algorithmic_per_launch": f"2*N_aux*N_ao^2*(N_occ+N_ac) = {fl['half_transform']:.4e} FLOP",
        "avg_launch_ms": kt["half_transform"][0] / kt["half_transform"][1],
    }
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "step_ms_median": step_ms[len(step_ms) // 2],
        "step_ms_min": step_ms[0],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"DF step ({wl.name}): N_ao={nao}, N_aux={naux}, N_occ={nocc}, N_ac={nac}, "
                        f"N_mo={nmo}; forward J, K, v, (uv|wx), (pu|vw)"
                        + ("" if args.forward_only else " + adjoint of (J, K, (uv|wx)) for the model-energy "
                           "cotangents"),
            "precision": "fp64",
            "nao": nao, "naux": naux, "nocc": nocc, "nac": nac, "nmo": nmo,
            "flops_per_step": w_alg,
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "kernels": kernels,
    }
    for k in ("Xocc", "Xact"):
        out.pop(k, None)
    torch.cuda.empty_cache()
    if not args.forward_only and not args.no_recompute:
        log("[bench] adjoint with the half transforms recomputed")
        res["recompute_x"] = recompute_block(B, nao, Cocc, Cact, C, gJ, gK, geri, 3, ctx)
    host = None
    if not args.no_split:
        log(f"[bench] split precision ({args.split_slices} slices) against FP64, forward and adjoint")
        res["split_precision"], host = split_comparison(B, nao, Cocc, Cact, C, args.split_slices, 5, ctx)
    if host is not None and not args.no_cpu_baseline and not args.no_oracle_check:
        log("[bench] CPU-baseline leg: the FP64 oracle's pass over all of B, against both GPU paths")
        res["oracle_check"] = oracle_check(B, wl, host)
    if not args.no_ppaa:
        log("[bench] (pq|uv) over all MOs")
        for k in ("Xocc", "Xact"):
            out.pop(k, None)
        torch.cuda.empty_cache()
        res["ppaa"] = ppaa_block(B, nao, Cact, C, 3, ctx)
    del B
    out.clear()
    torch.cuda.empty_cache()
    if not args.no_build:
        log("[bench] B from the metric and the three-centre integrals")
        res["build_cholesky"] = build_block(naux, nao, 3, ctx)
    if not args.no_batched:
        log(f"[bench] batched fragment subproblems, {args.fragment_densities} densities each")
        res["batched_fragments"] = batched_fragments(args.fragment_densities, 3, ctx, args.split_slices)
    if not args.no_cpu_baseline:
        log(f"[bench] timing the CPU oracle on {args.cpu_rows} auxiliary rows")
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_rows, wl.seed, adjoint=not args.forward_only)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
