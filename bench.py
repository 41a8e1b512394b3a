#!/usr/bin/env python
"""Benchmark of the twisted-mass Wilson Dslash / CG hot path on one MI355X.

One step = one FP64 conjugate-gradient solve of Mhat^dag Mhat x = b on the even
sites of a 24^3 x 48 lattice (links exp(i eps H), eps = 0.5, kappa = 0.16,
mu = 0.005, periodic space, antiperiodic time, Gaussian source) to a true
relative residual of 1e-10.  Each step runs the hop stencil with its fused
twisted-diagonal / Schur / CG epilogues, the BLAS-1 and FP64 reductions.

`value` = Dslash GB/s delivered inside the timed solves: the algorithmic bytes
of every hop launch (8 links + 1 neighbour spinor + 1 output spinor per output
site, 1536 B in FP64) divided by the wall time of the timed steps.  Beside it:
the hop kernel's own bandwidth against the HBM peak (HIP events), a precision
and link-compression sweep, FP64 vs mixed-precision CG time to the same 1e-10
FP64 residual on 32^3 x 64, the oracle's check of the solution, and the oracle
timed on the host.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0          # MI355X published HBM3E bandwidth
BYTES_PER_SITE = {(0, 0): 1536, (0, 1): 1152, (1, 0): 768, (1, 1): 576, (2, 0): 392, (2, 1): 296}
FLOPS_PER_SITE = 1320           # Wilson hop, per output site
WORKLOAD = dict(dims=(24, 24, 24, 48), eps=0.5, kappa=0.16, mu=0.005, seed=24, src_seed=26)
MIXED = dict(dims=(32, 32, 32, 64), eps=0.5, kappa=0.162, mu=0.003, seed=32, src_seed=34)
HOP_SOURCES = ("hop.hip", "device.h", "layout.h")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def hop_source_hash() -> str:
    h = hashlib.sha256()
    for f in HOP_SOURCES:
        with open(os.path.join(ROOT, "paper_1209_5942_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(vh: int):
    """HBM bytes per hop launch measured with rocprofv3 counters, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hop_f64_24x24x24x48_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != hop_source_hash() or rec.get("vh") != vh:
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle residual check and CPU baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 32^3 x 64 FP64-vs-mixed comparison")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X and this build has no "
              "multi-GPU path (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1209_5942_amd import synth
    from paper_1209_5942_amd import tmqcd as T

    T.lib()                                      # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # ------------------------------------------------------------ inputs ---
    w = WORKLOAD
    dims = w["dims"]
    prob = T.Problem(dims, w["kappa"], w["mu"], (1, 1, 1, -1))
    vh = prob.volume // 2
    log(f"drawing links {dims}")
    U = synth.random_links(dims, w["eps"], w["seed"])
    b = synth.gaussian_spinor(vh, w["src_seed"])
    U_dev = torch.from_numpy(U).to(dev)
    gauges = {(p, r): T.pack_gauge(prob, U_dev, p, r) for p in (T.F64, T.F32, T.F16) for r in (0, 1)}
    del U_dev
    b_dev = T.pack_spinor(prob, torch.from_numpy(b).to(dev), T.F64, T.EVEN)
    x_dev = torch.empty(T.spinor_bytes(prob, T.F64, T.EVEN), dtype=torch.uint8, device=dev)
    ws = T.workspace(prob, T.MHATDAGMHAT)
    torch.cuda.synchronize()

    def step():
        _, st, _ = T.cg(prob, {T.F64: gauges[(0, 0)]}, b_dev, x_dev, x_is_zero=True, tol=1e-10, max_iter=5000,
                        op=T.MHATDAGMHAT, ws=ws, check_every=16)
        return st

    # ------------------------------------------------------- timed steps ---
    log(f"warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    hop_launches = sum(s["hop_launches"] for s in stats)
    value = hop_launches * vh * BYTES_PER_SITE[(0, 0)] / elapsed / 1e9
    st0 = stats[-1]
    log(f"FP64 CG: {st0['iters']} iters, {1e3 * elapsed / args.steps:.2f} ms/solve, {value:.0f} GB/s")

    # ------------------------------------------- hop kernel: HIP events ---
    def time_hop(prec, recon, launches=100):
        src = T.pack_spinor(prob, torch.from_numpy(b).to(dev), prec, T.EVEN)
        out = torch.empty(T.spinor_bytes(prob, prec, T.ODD), dtype=torch.uint8, device=dev)
        g = gauges[(prec, recon)]
        for _ in range(5):
            T.dslash(prob, g, src, T.DSLASH_OE, prec, recon, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(launches):
            T.dslash(prob, g, src, T.DSLASH_OE, prec, recon, out=out)
        e1.record(stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / launches
        return t, vh * BYTES_PER_SITE[(prec, recon)] / t / 1e9, vh * FLOPS_PER_SITE / t / 1e9

    t_hop, gbs_hop, gflops_hop = time_hop(T.F64, T.RECON18, 200)
    sweep = {}
    for p, pn in ((T.F64, "f64"), (T.F32, "f32"), (T.F16, "f16")):
        for r, rn in ((0, "rec18"), (1, "rec12")):
            t, gbs, gf = time_hop(p, r)
            sweep[f"{pn}_{rn}"] = {"us": round(t * 1e6, 2), "GB_s": round(gbs, 1), "GFLOPS": round(gf, 1),
                                   "bytes_per_site": BYTES_PER_SITE[(p, r)]}
    log(f"hop f64: {t_hop * 1e6:.1f} us, {gbs_hop:.0f} GB/s, {gflops_hop:.0f} GFLOPS")

    # HBM copy probe (torch copy of a 4 GiB buffer) for the measured peak
    a = torch.empty(1 << 32, dtype=torch.uint8, device=dev)
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        c.copy_(a)
    e1.record(stream)
    e1.synchronize()
    copy_gbs = 2 * a.numel() * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, c

    result = {
        "metric": "Dslash GB/s (% HBM peak); CG time to 1e-10 residual, FP64 vs mixed",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 CG on Mhat^dag Mhat to 1e-10, 24^3x48 even-odd twisted-mass Wilson",
                   "dims": list(dims), "kappa": w["kappa"], "mu": w["mu"], "link_eps": w["eps"],
                   "bc": "periodic space, antiperiodic time", "recon": 18, "parallelism": "1 GPU"},
        "cg_fp64_24x24x24x48": {"iters": st0["iters"], "ms": round(1e3 * elapsed / args.steps, 3),
                                "true_rel_residual": st0["true_rel_residual"],
                                "hop_launches_per_solve": st0["hop_launches"]},
        "roofline": {"bound": "hbm", "achieved": round(gbs_hop, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(gbs_hop / PEAK_HBM_GBPS, 4), "traffic": traffic_from_profile(vh),
                     "kernel": "hop_kernel<F64,RECON18,dag=0,own=0,store> (DSLASH_OE / first Schur hop)",
                     "bytes_per_launch": vh * BYTES_PER_SITE[(0, 0)], "us_per_launch": round(t_hop * 1e6, 2),
                     "gflops": round(gflops_hop, 1), "measured_copy_peak_GB_s": round(copy_gbs, 1),
                     "frac_of_measured_copy": round(gbs_hop / copy_gbs, 4)},
        "dslash_sweep_24x24x24x48": sweep,
        "context": {"paper_hd5870_dslash_dp_gflops": 60, "paper_hmc_speedup_vs_server_cpu": 4},
    }

    # ---------------------------------------------- FP64 vs mixed CG -------
    if not args.no_mixed:
        m = MIXED
        pm = T.Problem(m["dims"], m["kappa"], m["mu"], (1, 1, 1, -1))
        log(f"drawing links {m['dims']}")
        Um = torch.from_numpy(synth.random_links(m["dims"], m["eps"], m["seed"])).to(dev)
        gm = {p: T.pack_gauge(pm, Um, p, 0) for p in (T.F64, T.F32, T.F16)}
        del Um
        bm = T.pack_spinor(pm, torch.from_numpy(synth.gaussian_spinor(pm.volume // 2, m["src_seed"])).to(dev),
                           T.F64, T.EVEN)
        xm = torch.empty(T.spinor_bytes(pm, T.F64, T.EVEN), dtype=torch.uint8, device=dev)
        wsm = T.workspace(pm, T.MHATDAGMHAT)
        mixed = {}
        for p, name in ((T.F64, "fp64"), (T.F32, "mixed_f32"), (T.F16, "mixed_f16")):
            best = None
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st, _ = T.cg(pm, gm, bm, xm, x_is_zero=True, tol=1e-10, max_iter=20000, op=T.MHATDAGMHAT,
                                inner_prec=p, ws=wsm, check_every=16)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if best is None or dt < best[0]:
                    best = (dt, st)
            dt, st = best
            mixed[name] = {"ms": round(1e3 * dt, 2), "iters": st["iters"], "reliable_updates": st["reliable_updates"],
                           "true_rel_residual": st["true_rel_residual"], "converged": st["converged"]}
            log(f"32^3x64 {name}: {1e3 * dt:.1f} ms, {st['iters']} iters, res {st['true_rel_residual']:.2e}")
        for k in ("mixed_f32", "mixed_f16"):
            mixed[k]["speedup_vs_fp64"] = round(mixed["fp64"]["ms"] / mixed[k]["ms"], 3)
        mixed["workload"] = "Mhat^dag Mhat, 32^3x64, kappa 0.162, mu 0.003, eps 0.5, tol 1e-10 (FP64 true residual)"
        result["cg_32x32x32x64"] = mixed
        del gm, bm, xm, wsm

    # ------------------------------------- oracle check and CPU baseline ---
    if not args.no_oracle:
        from threadpoolctl import threadpool_limits

        from oracle import dirac as D
        log("oracle check of the 24^3x48 solution")
        x = T.unpack_spinor(prob, x_dev, T.F64, T.EVEN).cpu().numpy()
        A = lambda v: D.apply_MhatdagMhat(U, v, dims, w["kappa"], w["mu"], (1, 1, 1, -1))
        result["cg_fp64_24x24x24x48"]["oracle_rel_residual"] = D.true_rel_residual(A, b, x)
        log("CPU baseline: oracle hop")
        psi = synth.gaussian_spinor(prob.volume, 27)
        with threadpool_limits(1):
            reps = 2
            t0 = time.perf_counter()
            for _ in range(reps):
                D.hop(U, psi, dims, (1, 1, 1, -1))
            dt = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": round(reps * prob.volume * BYTES_PER_SITE[(0, 0)] / dt / 1e9, 4), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{reps} whole-lattice hops H psi of the FP64 NumPy oracle at 24^3x48 "
                      f"({reps * prob.volume} output sites x 1536 B), {dt:.1f} s, one thread"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
