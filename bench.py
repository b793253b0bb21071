#!/usr/bin/env python3
"""Benchmark of the density-fitted contraction step on one MI355X.

One step = one forward pass of the whole hot path through df_step at paper scale
(N_ao = 1200, N_aux = 4800, N_occ = 300, N_ac = 40, N_mo = 1200, B = 27.7 GB packed FP64):
the shared half transform X = b^P [C_occ | C_act], the J-vector and J, K, the second
transform b^P_{pu}, (uv|wx) and (pu|vw).  Inputs are drawn on the GPU and are resident
in HBM before the timed region starts.

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


def step_flops(naux, nao, nocc, nac, nmo):
    """Algorithmic FP64 FLOPs of one forward step (half, J, K, b_pu, (pu|vw))."""
    npair = nao * (nao + 1) // 2
    f = {
        "half_transform": 2 * naux * nao * nao * (nocc + nac),
        "j": 2 * naux * nao * nocc + 2 * naux * npair,
        "k_syrk": naux * nocc * nao * (nao + 1),
        "mo_transform": 2 * naux * nao * nmo * nac,
        "papa": 2 * naux * nmo * nac ** 3,
    }
    return f


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
        # HBM-bound kernels: bytes read + written
        "jvec": ("hbm", 8 * (naux * nao * nocc + nao * nocc + naux)),
        "coulomb": ("hbm", 8 * (naux * npair + naux + 2 * nao * nao)),
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


def cpu_baseline(wl, rows, seed):
    """The FP64 oracle on `rows` auxiliary rows of the same workload (host cores)."""
    import numpy as np
    from oracle import df_oracle as O
    from paper_2505_03755_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    B = synth.cholesky_vectors(rows, wl.nao, wl.L, seed=seed)
    C = synth.orbitals(wl.nao, seed=seed)
    Cocc, Cact = C[:, :wl.nocc], C[:, wl.nocc:wl.nocc + wl.nac]
    t0 = time.perf_counter()
    J, K, v = O.jk(B, wl.nao, Cocc)
    eri, _ = O.active_eri(B, wl.nao, Cact)
    pa = O.papa(B, wl.nao, C, Cact)
    dt = time.perf_counter() - t0
    fl = sum(step_flops(rows, wl.nao, wl.nocc, wl.nac, wl.nmo).values())
    assert np.isfinite(J).all() and np.isfinite(K).all() and np.isfinite(pa).all() and np.isfinite(eri).all()
    return {"value": fl / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{rows} of {wl.naux} auxiliary rows at N_ao={wl.nao}, N_occ={wl.nocc}, N_ac={wl.nac} "
                      f"(forward J, K, v, (uv|wx), (pu|vw)); {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="paper", choices=["tiny", "medium", "paper"])
    ap.add_argument("--cpu-rows", type=int, default=240, help="auxiliary rows in the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] calibration copy of {args.calibration_copy_mib} MiB done")
    run = lambda: dfmi.step(B, nao, Cocc, Cact, C, outputs=out, ctx=ctx)
    for i in range(args.warmup):
        run()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")

    ctx.set_timing(True)
    ctx.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = ctx.timing_read()
    ctx.set_timing(False)
    log(f"[bench] {args.steps} timed steps in {dt:.3f} s")

    fl = step_flops(naux, nao, nocc, nac, nmo)
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
        "traffic": None,
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
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"DF forward step ({wl.name}): N_ao={nao}, N_aux={naux}, N_occ={nocc}, N_ac={nac}, "
                        f"N_mo={nmo}; outputs J, K, v, (uv|wx), (pu|vw)",
            "nao": nao, "naux": naux, "nocc": nocc, "nac": nac, "nmo": nmo,
            "flops_per_step": w_alg,
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "kernels": kernels,
    }
    del B
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log(f"[bench] timing the CPU oracle on {args.cpu_rows} auxiliary rows")
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_rows, wl.seed)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
