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
# per output site of a hop: 8 links + one input spinor + one output spinor (perfect neighbour reuse);
# links by (precision, encoding) 144/96/80/64 B in FP64 (REC18/12/10/8), half and a quarter of that in
# FP32 and FP16; spinors 192 / 96 / 52 B (FP16 with its FP32 scale)
_LINK = {0: (144, 96, 80, 64), 1: (72, 48, 40, 32), 2: (36, 24, 20, 16)}
_SPINOR = {0: 192, 1: 96, 2: 52}
BYTES_PER_SITE = {(p, r): 8 * _LINK[p][r] + 2 * _SPINOR[p] for p in range(3) for r in range(4)}
FLOPS_PER_SITE = 1320           # Wilson hop, per output site
# one FP64 iteration of CG on Mhat^dag Mhat per even site (algorithmic, REC18 links): the operator's four
# hops -- two plain stores (1536 B each), the one that adds A p and sums |Mhat p|^2 (also reads p: 1728 B),
# the one that adds A^dag t, updates r and sums |r|^2 (reads t, reads and writes r: 1920 B) -- and
# x += alpha p, p = r + beta p (reads p, r, x; writes p, x: 960 B)
CG_ITER_BYTES_PER_SITE = 1536 + 1728 + 1536 + 1920 + 960
WORKLOAD = dict(dims=(24, 24, 24, 48), eps=0.5, kappa=0.16, mu=0.005, seed=24, src_seed=26)
MIXED = dict(dims=(32, 32, 32, 64), eps=0.5, kappa=0.162, mu=0.003, seed=32, src_seed=34)
HOP_SOURCES = ("hop.hip", "stencil.h", "device.h", "layout.h")
_HOST = {}   # host fields drawn by one leg and reused by a later one (the 32^3 x 64 links, source, x* stats)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def oracle_error(op, U, b, x, x_star, dims, kappa, mu, bc=(1, 1, 1, -1), U_solve=None):
    """The C++ oracle's check of a GPU solution x of op x = b: the true relative residual
    ||b - op x|| / ||b|| on the links the solver used (U_solve, e.g. the oracle's own
    reconstruction of compressed links; default U) and the relative error ||x - x*|| / ||x*||
    against the oracle's solution x* (a CG on the same system to 1e-12)."""
    import numpy as np

    from oracle import cref
    res = cref.true_rel_residual(op, U if U_solve is None else U_solve, b, x, dims, kappa, mu, bc)
    out = {"oracle_rel_residual": res}
    if x_star is not None:
        out["rel_error_vs_oracle_solution"] = float(np.linalg.norm(x - x_star) / np.linalg.norm(x_star))
    return out


def oracle_solution(op, U, b, dims, kappa, mu, bc=(1, 1, 1, -1), tol=1e-12):
    """x* = op^{-1} b by the C++ oracle's CG (all host threads), and its statistics (the iterate at
    which the recursive residual first reached 1e-10 is timed separately)."""
    from oracle import cref
    x, st, rc = cref.cg(op, U, b, dims, kappa, mu, bc, tol=tol, report_tol=1e-10)
    assert rc == 0 and st["true_rel_residual"] <= 2 * tol, st
    return x, st


def hop_source_hash() -> str:
    h = hashlib.sha256()
    for f in HOP_SOURCES:
        with open(os.path.join(ROOT, "paper_1209_5942_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(vh: int, block: int, order: int):
    """HBM bytes per hop launch in the given launch shape, measured with rocprofv3 counters, if taken on
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hop_f64_24x24x24x48_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != hop_source_hash() or rec.get("vh") != vh:
        return None
    return rec.get("shapes", {}).get(f"{block}/{order}", {}).get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle residual check and CPU baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 32^3 x 64 FP64-vs-mixed comparison")
    ap.add_argument("--no-extras", action="store_true", help="skip the multi-RHS, batch and HMC measurements")
    ap.add_argument("--normal-exit", action="store_true",
                    help="end through the interpreter's normal shutdown instead of leaving at once after the JSON "
                         "line (needed under rocprofv3, which writes its results at exit)")
    ap.add_argument("--kernel-only", nargs="?", const="hop",
                    choices=("hop", "mrhs", "force24", "force32", "heatbath24", "tlsym16"),
                    help="only a 1 GiB copy (counter calibration) and 10 launches of one kernel, for rocprofv3 --pmc: "
                         "the tuned FP64 hop (default) or the tuned 12-RHS hop in FP64 and FP32 at 24^3x48, the "
                         "FP64 fermion force at 24^3x48 or 32^3x64, 10 FP64 heatbath sweeps at 24^3x48 (8 launches "
                         "each), or 10 tree-level Symanzik gauge forces at 16^3x32 (2 launches each)")
    ap.add_argument("--traffic-from", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "KERNEL_ONLY_LOG"),
                    help="write the hop's measured HBM traffic from two --pmc runs of --kernel-only, then exit")
    ap.add_argument("--mrhs-shapes-from", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "KERNEL_ONLY_LOG"),
                    help="print the FP64 12-RHS hop's counters in each pinned shape of --kernel-only mrhs, then exit")
    ap.add_argument("--durations-from", nargs=3, metavar=("KERNEL_TRACE_CSV", "NAME_SUBSTRING", "LAST_N"),
                    help="mean/min/max duration of the last N dispatches of a kernel in a rocprofv3 kernel trace")
    ap.add_argument("--counters-from", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "NAME_SUBSTRING", "LAST_N"),
                    help="HBM bytes of the last N dispatches of a kernel from two --pmc runs, scaled by the "
                         "first copy kernel of each run (1 GiB)")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from_counters(*args.traffic_from)
        return
    if args.durations_from:
        durations_from_trace(*args.durations_from)
        return
    if args.mrhs_shapes_from:
        mrhs_shapes_from_counters(*args.mrhs_shapes_from)
        return
    if args.counters_from:
        counters_from(*args.counters_from)
        return
    if args.kernel_only in ("force24", "force32", "heatbath24", "tlsym16") and args.gpus == 1:
        kernel_only_force(args.kernel_only)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X and the library has no "
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
    gauges = {(p, r): T.pack_gauge(prob, U_dev, p, r) for p in (T.F64, T.F32, T.F16) for r in (0, 1, 2, 3)}
    del U_dev
    b_dev = T.pack_spinor(prob, torch.from_numpy(b).to(dev), T.F64, T.EVEN)
    x_dev = torch.empty(T.spinor_bytes(prob, T.F64, T.EVEN), dtype=torch.uint8, device=dev)
    ws = T.workspace(prob, T.MHATDAGMHAT)
    torch.cuda.synchronize()

    if args.kernel_only == "hop":
        kernel_only(T, prob, gauges, b, dev)
        return
    if args.kernel_only == "mrhs":
        kernel_only_mrhs(T, prob, gauges, dev)
        return

    # launch shapes of the hop kernels chosen by the autotuner on this problem
    tuning = {f"class{r['kernel_class']}": {"block": r["block"], "order": r["order"], "us": round(r["us"], 2),
                                          "default_us": round(r["default_us"], 2)}
              for r in T.tune(prob, gauges[(0, 0)], T.F64, T.RECON18)}
    log(f"tuned: {tuning}")

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
    for p in (T.F64, T.F32, T.F16):            # the sweep in tuned shapes too
        for r in (0, 1, 2, 3):
            if (p, r) != (T.F64, T.RECON18):
                T.tune(prob, gauges[(p, r)], p, r)
    sweep = {}
    for p, pn in ((T.F64, "f64"), (T.F32, "f32"), (T.F16, "f16")):
        for r, rn in ((0, "rec18"), (1, "rec12"), (2, "rec10"), (3, "rec8")):
            t, gbs, gf = time_hop(p, r)
            sweep[f"{pn}_{rn}"] = {"us": round(t * 1e6, 2), "GB_s": round(gbs, 1), "GFLOPS": round(gf, 1),
                                   "bytes_per_site": BYTES_PER_SITE[(p, r)]}
    log(f"hop f64: {t_hop * 1e6:.1f} us, {gbs_hop:.0f} GB/s, {gflops_hop:.0f} GFLOPS")

    # measured ceilings on a 4 GiB buffer (far beyond the 256 MB of MALL): the library's streaming
    # probe (16-byte reads; copy) at two grid sizes, and torch's copy
    a = torch.ones(1 << 32, dtype=torch.uint8, device=dev)
    c = torch.empty_like(a)
    word = torch.zeros(1, dtype=torch.int32, device=dev)
    read_gbs = max(a.numel() / _events_time(lambda: T.hbm_probe(a, xor_out=word, grid=g), 5) / 1e9
                   for g in (1024, 2048))
    probe_copy_gbs = max(2 * a.numel() / _events_time(lambda: T.hbm_probe(a, c, grid=g), 5) / 1e9
                         for g in (1024, 2048))
    copy_gbs = 2 * a.numel() / _events_time(lambda: c.copy_(a), 5) / 1e9
    del a, c

    traffic = traffic_from_profile(vh, tuning["class0"]["block"], tuning["class0"]["order"])
    cg_gbs = st0["iters"] * vh * CG_ITER_BYTES_PER_SITE / (elapsed / args.steps) / 1e9
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
                                "hop_launches_per_solve": st0["hop_launches"],
                                "algorithmic_bytes_per_iteration": vh * CG_ITER_BYTES_PER_SITE,
                                # the iterations' bytes over the whole solve's time (set-up and the final
                                # true residual included)
                                "iteration_GB_s": round(cg_gbs, 1),
                                "iteration_frac_of_measured_read": round(cg_gbs / read_gbs, 4)},
        "roofline": {"bound": "hbm", "achieved": round(gbs_hop, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(gbs_hop / PEAK_HBM_GBPS, 4), "traffic": traffic,
                     "kernel": f"hop_kernel<F64,RECON18,dag=0,own=0,store> block {tuning['class0']['block']} "
                               f"order {tuning['class0']['order']} (DSLASH_OE / first Schur hop)",
                     "bytes_per_launch": vh * BYTES_PER_SITE[(0, 0)], "us_per_launch": round(t_hop * 1e6, 2),
                     "gflops": round(gflops_hop, 1), "measured_read_peak_GB_s": round(read_gbs, 1),
                     "measured_copy_peak_GB_s": round(max(copy_gbs, probe_copy_gbs), 1),
                     "hbm_traffic_GB_s": round(traffic / (t_hop) / 1e9, 1) if traffic else None,
                     "frac_of_measured_read": round(gbs_hop / read_gbs, 4)},
        "dslash_sweep_24x24x24x48": sweep,
        "tuning_f64_rec18": tuning,
        "context": {"paper_hd5870_dslash_dp_gflops": 60, "paper_hmc_speedup_vs_server_cpu": 4},
    }

    # ------------------------------- BiCGStab on Mhat vs CG on the normal equations ---
    # the same system Mhat x = b: BiCGStab on Mhat itself, CG on Mhat^dag Mhat x = Mhat^dag b
    log("BiCGStab vs CGNE on Mhat x = b")
    ws_bi = T._bytes(T.bicgstab_workspace_bytes(prob, T.MHAT), dev)
    xb_dev = torch.empty_like(x_dev)
    bd_dev = T.dslash(prob, gauges[(0, 0)], b_dev, T.MHATDAG, ws=ws)
    xc_dev = torch.empty_like(x_dev)

    def best_of(fn, n=3):
        best = None
        for _ in range(n):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, st)
        return best
    t_bi, st_bi = best_of(lambda: T.bicgstab(prob, gauges[(0, 0)], b_dev, xb_dev, x_is_zero=True, tol=1e-10,
                                             op=T.MHAT, ws=ws_bi, check_every=8)[1])
    t_cgne, st_cgne = best_of(lambda: T.cg(prob, {T.F64: gauges[(0, 0)]}, bd_dev, xc_dev, x_is_zero=True, tol=1e-10,
                                           max_iter=5000, op=T.MHATDAGMHAT, ws=ws, check_every=16)[1])
    result["bicgstab_24x24x24x48"] = {
        "workload": "Mhat x = b, 24^3x48 (the step's lattice and source), tol 1e-10 on the solver's own system",
        "bicgstab_ms": round(1e3 * t_bi, 3), "bicgstab_iters": st_bi["iters"],
        "bicgstab_hop_launches": st_bi["hop_launches"], "bicgstab_true_rel_residual": st_bi["true_rel_residual"],
        "cgne_ms": round(1e3 * t_cgne, 3), "cgne_iters": st_cgne["iters"], "cgne_hop_launches": st_cgne["hop_launches"],
        "speedup_bicgstab_vs_cgne": round(t_cgne / t_bi, 3)}
    log(f"BiCGStab {1e3 * t_bi:.1f} ms ({st_bi['iters']} it), CGNE {1e3 * t_cgne:.1f} ms ({st_cgne['iters']} it)")

    # ---------------------------------------------- FP64 vs mixed CG -------
    if not args.no_mixed:
        result["cg_32x32x32x64"] = bench_mixed(T, synth, dev, not args.no_oracle)

    if not args.no_extras:
        result["small_4x4x4x4"] = bench_small(T, synth, dev, not args.no_oracle)
        result["dslash_sizes_f64_rec18"] = bench_sizes(T, dev)
        result["multi_rhs_24x24x24x48"] = bench_multi_rhs(T, prob, U, dev)
        result["cg_multi_rhs_24x24x24x48"] = bench_cg_mrhs(T, synth, U, dev, not args.no_oracle)
        result["batch_cg"] = bench_batch(T, synth, dev, not args.no_oracle)
        result["batch_cg_thermal"] = bench_batch(T, synth, dev, not args.no_oracle, BATCH_THERMAL)
        result["hmc_16x16x16x32"] = bench_hmc(T, synth, dev)
        result["force_f64_large"] = bench_force_large(T, dev, read_gbs)
        result["heatbath"] = bench_heatbath(T, synth, dev)

    # ------------------------------------- oracle check and CPU baseline ---
    if not args.no_oracle:
        from oracle import cref
        U64 = U.reshape(-1, 4, 3, 3)
        kap, mu_ = w["kappa"], w["mu"]
        log("oracle solution x* on 24^3x48 and CPU baseline (C++ oracle)")
        x_star, ost = oracle_solution("MHATDAGMHAT", U64, b, dims, kap, mu_)
        x = T.unpack_spinor(prob, x_dev, T.F64, T.EVEN).cpu().numpy()
        result["cg_fp64_24x24x24x48"].update(oracle_error("MHATDAGMHAT", U64, b, x, x_star, dims, kap, mu_))
        # BiCGStab and CGNE solve Mhat x = b: x* = (Mhat^dag Mhat)^{-1} Mhat^dag b, all by the oracle
        bh = cref.apply("MHATDAG", U64, b, dims, kap, mu_, (1, 1, 1, -1))
        xh_star, _ = oracle_solution("MHATDAGMHAT", U64, bh, dims, kap, mu_)
        for name, xd in (("bicgstab", xb_dev), ("cgne", xc_dev)):
            xh = T.unpack_spinor(prob, xd, T.F64, T.EVEN).cpu().numpy()
            e = oracle_error("MHAT", U64, b, xh, xh_star, dims, kap, mu_)
            result["bicgstab_24x24x24x48"][f"{name}_oracle_rel_residual_of_Mhat_x_eq_b"] = e["oracle_rel_residual"]
            result["bicgstab_24x24x24x48"][f"{name}_rel_error_vs_oracle_solution"] = e["rel_error_vs_oracle_solution"]
        result["cpu_baseline"] = cpu_baseline(T, synth, U64, b, ost, cg_seconds=elapsed / args.steps)
    print(json.dumps(result), flush=True)
    if args.normal_exit:
        return
    # leave at once: nothing below needs the interpreter's teardown (GPU buffers, thread pools)
    sys.stdout.flush()
    sys.stderr.flush()
    os._exit(0)


def cpu_baseline(T, synth, U64, b, ost, cg_seconds):
    """The C++ FP64 oracle on the host cores: `value` is its Dslash GB/s inside its CG on Mhat^dag Mhat
    at 24^3 x 48 (the bench step's solve, in the same unit as `value`: 1536 B per hop output site, four
    hops per iteration), timed up to the iterate that first reached 1e-10 (the iterations of the x*
    solve above).  Beside it: the hop, Mhat and Mhat^dag Mhat at 4^4, 24^3 x 48 and 32^3 x 64 with all
    threads and with one, CG time to 1e-10 at 4^4 (all threads and one) and 32^3 x 64 (all threads,
    the x* solve of the mixed-precision leg), and two hops of the NumPy oracle (one thread)."""
    import platform

    import numpy as np

    from oracle import cref
    from oracle import dirac as D
    threads = cref.threads()
    cpu_model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            names = [l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")]
        cpu_model = names[0] if names else cpu_model
    except OSError:
        pass
    bc = (1, 1, 1, -1)

    def timed(fn, reps):
        if reps > 1:
            fn()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        return (time.perf_counter() - t0) / reps

    vh1 = U64.shape[0] // 2
    cg_gbs = ost["report_iters"] * 4 * vh1 * BYTES_PER_SITE[(0, 0)] / ost["report_seconds"] / 1e9
    out = {"value": round(cg_gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": (f"the C++ FP64 oracle's CG on Mhat^dag Mhat at 24^3x48 (kappa 0.16, mu 0.005, the bench "
                      f"step's links and source) up to 1e-10: {ost['report_iters']} iterations in "
                      f"{ost['report_seconds']:.1f} s on {threads} threads (4 hops of 1536 B per even site each); "
                      f"the GPU step takes {1e3 * cg_seconds:.1f} ms"),
           "host": {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "threads_used": threads,
                    "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "cpu_model": cpu_model},
           "cg_to_1e-10_24x24x24x48": {"threads": threads, "iters": ost["report_iters"],
                                       "seconds": round(ost["report_seconds"], 3),
                                       "true_rel_residual": ost["report_true_rel_residual"]}}
    cfgs = [("4x4x4x4", (4, 4, 4, 4), 0.3, 0.15, 0.01, 1, 2), ("24x24x24x48", (24, 24, 24, 48), None, 0.16, 0.005, 0, 0),
            ("32x32x32x64", MIXED["dims"], MIXED["eps"], MIXED["kappa"], MIXED["mu"], MIXED["seed"], MIXED["src_seed"])]
    for name, dims, eps, kappa, mu, seed, src_seed in cfgs:
        ost_n = None
        if eps is None:
            U, src = U64, b
        elif name == "32x32x32x64" and "mixed" in _HOST:
            U, src, ost_n = _HOST["mixed"]
        else:
            log(f"CPU baseline {name}: drawing links")
            U = synth.random_links(dims, eps, seed).reshape(-1, 4, 3, 3)
            src = synth.gaussian_spinor(U.shape[0] // 2, src_seed)
        vh = U.shape[0] // 2
        reps = 200 if vh < 1000 else 1
        rec = {}
        for nt in sorted({threads, 1}, reverse=True):
            cref.set_threads(nt)
            t_hop = timed(lambda: cref.apply("HOP_OE", U, src, dims, kappa, mu, bc), reps)
            t_mhat = timed(lambda: cref.apply("MHAT", U, src, dims, kappa, mu, bc), reps)
            t_nrm = timed(lambda: cref.apply("MHATDAGMHAT", U, src, dims, kappa, mu, bc), reps)
            rec[f"threads_{nt}"] = {"hop_ms": round(1e3 * t_hop, 4), "hop_GB_s": round(vh * 1536 / t_hop / 1e9, 3),
                                    "mhat_ms": round(1e3 * t_mhat, 4), "mhatdagmhat_ms": round(1e3 * t_nrm, 4)}
            if vh < 1000:
                _, st = oracle_solution("MHATDAGMHAT", U, src, dims, kappa, mu, bc, tol=1e-10)
                rec[f"threads_{nt}"]["cg_to_1e-10"] = {"iters": st["iters"], "seconds": round(st["seconds"], 4),
                                                       "true_rel_residual": st["true_rel_residual"]}
            elif ost_n is not None and nt == threads:   # the x* solve of the mixed-precision leg, up to 1e-10
                rec[f"threads_{nt}"]["cg_to_1e-10"] = {"iters": ost_n["report_iters"],
                                                       "seconds": round(ost_n["report_seconds"], 3),
                                                       "true_rel_residual": ost_n["report_true_rel_residual"]}
        cref.set_threads(threads)
        out[name] = rec
    # the NumPy definitional oracle, for information: two whole-lattice hops at 24^3 x 48, one thread
    from threadpoolctl import threadpool_limits
    psi = synth.gaussian_spinor(U64.shape[0], 27)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for _ in range(2):
            D.hop(U64, psi, (24, 24, 24, 48), bc)
        dt = (time.perf_counter() - t0) / 2
    out["numpy_oracle_hop_24x24x24x48"] = {"threads": 1, "seconds": round(dt, 2),
                                           "GB_s": round(U64.shape[0] * 1536 / dt / 1e9, 4)}
    return out



def bench_mixed(T, synth, dev, check):
    """32^3 x 64 (kappa 0.162, mu 0.003, eps 0.5): CG on Mhat^dag Mhat to a true FP64 residual of 1e-10
    with FP64, FP32-inner and FP16-inner hops, for each link encoding (REC18/12/10/8).  Each solve is the
    best of three; its solution is checked by the C++ oracle: the true residual on the links the solver
    used (for REC10/REC8 the oracle's own reconstruction from its encoding of the same links) and the
    relative error against the oracle's solution x* (CG to 1e-12 on the uncompressed links)."""
    import numpy as np
    import torch
    m = MIXED
    dims, kappa, mu = m["dims"], m["kappa"], m["mu"]
    pm = T.Problem(dims, kappa, mu, (1, 1, 1, -1))
    log(f"drawing links {dims}")
    Um_host = synth.random_links(dims, m["eps"], m["seed"]).reshape(-1, 4, 3, 3)
    bm_host = synth.gaussian_spinor(pm.volume // 2, m["src_seed"])
    bm = T.pack_spinor(pm, torch.from_numpy(bm_host).to(dev), T.F64, T.EVEN)
    xm = torch.empty(T.spinor_bytes(pm, T.F64, T.EVEN), dtype=torch.uint8, device=dev)
    wsm = T.workspace(pm, T.MHATDAGMHAT)
    x_star, ost = None, None
    if check:
        log("oracle solution x* on 32^3x64 (C++ oracle, CG to 1e-12)")
        x_star, ost = oracle_solution("MHATDAGMHAT", Um_host, bm_host, dims, kappa, mu)
    _HOST["mixed"] = (Um_host, bm_host, ost)
    out = {"workload": "Mhat^dag Mhat, 32^3x64, kappa 0.162, mu 0.003, eps 0.5, tol 1e-10 (FP64 true residual)"}
    if ost is not None:
        out["oracle_solution"] = {"iters": ost["iters"], "true_rel_residual": ost["true_rel_residual"],
                                  "seconds": round(ost["seconds"], 2)}
    fp64_ms = None
    for rec, rname in ((0, "rec18"), (1, "rec12"), (2, "rec10"), (3, "rec8")):
        Um = torch.from_numpy(Um_host).to(dev)
        gr = {p: T.pack_gauge(pm, Um, p, rec) for p in (T.F64, T.F32, T.F16)}
        del Um
        for p in (T.F64, T.F32, T.F16):      # every precision in its tuned launch shapes
            T.tune(pm, gr[p], p, rec)
        U_solve = None
        if check and rec != 0:               # the links the solver sees, rebuilt by the oracle
            from oracle import compress as OC
            U_solve = {1: lambda u: OC.rec12_decode(u[..., :2, :]), 2: lambda u: OC.rec10_decode(OC.rec10_encode(u)),
                       3: lambda u: OC.rec8_decode(OC.rec8_encode(u))}[rec](Um_host)
        res = {}
        for p, name in ((T.F64, "fp64"), (T.F32, "mixed_f32"), (T.F16, "mixed_f16")):
            best = None
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st, _ = T.cg(pm, gr, bm, xm, x_is_zero=True, tol=1e-10, max_iter=20000, op=T.MHATDAGMHAT,
                                inner_prec=p, recon=rec, ws=wsm, check_every=16)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if best is None or dt < best[0]:
                    best = (dt, st)
            dt, st = best
            if fp64_ms is None:
                fp64_ms = 1e3 * dt
            r = {"ms": round(1e3 * dt, 2), "iters": st["iters"], "reliable_updates": st["reliable_updates"],
                 "true_rel_residual": st["true_rel_residual"], "converged": st["converged"],
                 "speedup_vs_fp64_rec18": round(fp64_ms / (1e3 * dt), 3)}
            if check:
                xs = T.unpack_spinor(pm, xm, T.F64, T.EVEN).cpu().numpy()
                r.update(oracle_error("MHATDAGMHAT", Um_host, bm_host, xs, x_star, dims, kappa, mu, U_solve=U_solve))
                if U_solve is not None:
                    r["oracle_rel_residual_uncompressed_links"] = oracle_error(
                        "MHATDAGMHAT", Um_host, bm_host, xs, None, dims, kappa, mu)["oracle_rel_residual"]
            res[name] = r
            log(f"32^3x64 {rname} {name}: {1e3 * dt:.1f} ms, {st['iters']} iters, "
                f"oracle res {r.get('oracle_rel_residual', float('nan')):.2e}, "
                f"err {r.get('rel_error_vs_oracle_solution', float('nan')):.2e}")
        for k in ("mixed_f32", "mixed_f16"):
            res[k]["speedup_vs_fp64"] = round(res["fp64"]["ms"] / res[k]["ms"], 3)
        if rec == 0:
            out.update(res)                   # REC18 at the top level, as before
        else:
            out[rname] = res
        del gr, U_solve
    return out


def kernel_only(T, prob, gauges, b, dev):
    """Calibration copy of known size, then the tuner and 10 FP64 hops in each of the 12 launch shapes
    (block size x block order, pinned one after the other); for counter runs."""
    import torch
    a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
    c = torch.empty_like(a)
    c.copy_(a)                     # the first copy kernel of the run: the calibration
    torch.cuda.synchronize()
    tuned = T.tune(prob, gauges[(0, 0)], T.F64, T.RECON18)[0]
    src = T.pack_spinor(prob, torch.from_numpy(b).to(dev), T.F64, T.EVEN)
    out = torch.empty(T.spinor_bytes(prob, T.F64, T.ODD), dtype=torch.uint8, device=dev)
    shapes = [(block, order) for block in (128, 256) for order in range(6)]
    for block, order in shapes:
        T.tune_set(prob, T.F64, T.RECON18, 0, block, order)
        for _ in range(10):
            T.dslash(prob, gauges[(0, 0)], src, T.DSLASH_OE, out=out)
    torch.cuda.synchronize()
    T.tune_clear()
    print(json.dumps({"copy_bytes": a.numel(), "hop_launches": 10, "shapes": shapes, "hop_block": tuned["block"],
                      "hop_order": tuned["order"], "hop_algorithmic_bytes": prob.volume // 2 * 1536,
                      "hop_source_sha": hop_source_hash()}), flush=True)


def kernel_only_mrhs(T, prob, gauges, dev):
    """Calibration copy, then 10 tuned 12-RHS hops (point sources) in FP64 and in FP32, RECON18."""
    import torch

    from paper_1209_5942_amd import synth
    a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    del a, c
    src = torch.from_numpy(synth.point_sources(prob.volume // 2, 0)).to(dev)
    info = {"copy_bytes": 1 << 30, "launches": 10}
    for p, name in ((T.F64, "f64"), (T.F32, "f32")):
        g = gauges[(p, 0)]
        s = T.pack_spinor(prob, src, p, T.EVEN, nrhs=12)
        o = torch.empty(T.spinor_bytes(prob, p, T.ODD, 12), dtype=torch.uint8, device=dev)
        tuned = T.tune_mrhs(prob, g, 12, p, 0)
        for _ in range(10):
            T.dslash(prob, g, s, T.DSLASH_OE, p, 0, nrhs=12, out=o)
        torch.cuda.synchronize()
        info[name] = {"order": tuned["order"], "group": tuned["group"]}
        if p == T.F64:
            # then 3 launches in each pinned shape: block order x right-hand sides per sweep
            shapes = [(order, group) for order in range(6) for group in (0, 6, 4)]
            for order, group in shapes:
                T.tune_set(prob, p, 0, 3, 256, order, nrhs=12, group=group)
                for _ in range(3):
                    T.dslash(prob, g, s, T.DSLASH_OE, p, 0, nrhs=12, out=o)
            torch.cuda.synchronize()
            T.tune_clear()
            info["f64_shapes"] = shapes
            info["f64_shape_launches"] = 3
            info["vh"] = prob.volume // 2
    print(json.dumps(info), flush=True)


def kernel_only_force(which):
    """Calibration copy (1 GiB), then 10 FP64 fermion-force launches (RECON18) at 24^3x48 or 32^3x64 on
    random fields (values do not change the kernel's memory traffic); or 10 FP64 heatbath sweeps at 24^3x48
    (SU(3) links, beta 5.7); or 10 tree-level Symanzik forces (c1 = -1/12) at 16^3x32."""
    import torch

    from paper_1209_5942_amd import synth
    from paper_1209_5942_amd import tmqcd as T
    dev = torch.device("cuda:0")
    a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    del a, c
    if which in ("heatbath24", "tlsym16"):
        dims = (24, 24, 24, 48) if which == "heatbath24" else (16, 16, 16, 32)
        prob = T.Problem(dims, 0.15, 0.0, (1, 1, 1, -1))
        g = T.pack_gauge(prob, torch.from_numpy(synth.random_links(dims, 0.4, 91)).to(dev))
        if which == "heatbath24":
            for k in range(10):
                T.heatbath(prob, g, 5.7, 92, k)
            info = {"sweeps": 10, "launches_per_sweep": 8, "sweep_algorithmic_bytes": 5184 * prob.volume}
        else:
            ws = T._bytes(T.gauge_force_tlsym_workspace_bytes(prob), dev)
            G = torch.empty((prob.volume, 4, 8), dtype=torch.float64, device=dev)
            for _ in range(10):
                T.gauge_force_tlsym(prob, g, 3.9, -1.0 / 12.0, out=G, ws=ws)
            info = {"forces": 10, "staple_field_bytes": 3456 * prob.volume}
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "dims": list(dims), **info}), flush=True)
        return
    dims = (24, 24, 24, 48) if which == "force24" else (32, 32, 32, 64)
    prob = T.Problem(dims, 0.155, 0.01, (1, 1, 1, -1))
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    g = T.pack_gauge(prob, torch.randn((prob.volume, 4, 3, 3), dtype=torch.complex128, device=dev, generator=gen))
    X = T.pack_spinor(prob, torch.randn((prob.volume, 4, 3), dtype=torch.complex128, device=dev, generator=gen))
    Y = T.pack_spinor(prob, torch.randn((prob.volume, 4, 3), dtype=torch.complex128, device=dev, generator=gen))
    G = torch.empty((prob.volume, 4, 8), dtype=torch.float64, device=dev)
    for _ in range(10):
        T.force(prob, g, X, Y, out=G)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 1 << 30, "launches": 10, "dims": list(dims),
                      "force_algorithmic_bytes": prob.volume * 1216}), flush=True)


def traffic_from_counters(fetch_csv, write_csv, kernel_log):
    """Write the per-launch HBM traffic of the FP64 hop in each launch shape from two rocprofv3 --pmc runs
    of --kernel-only.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same counters read for the
    calibration copy of known size in the same run; the last 12 x 10 hop dispatches are the 12 pinned
    shapes in the order the run printed.
    """
    import csv
    with open(kernel_log) as fh:
        info = [json.loads(l) for l in fh if l.startswith("{")][-1]

    def rows(path, counter):
        out = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.append(r)
        return sorted(out, key=lambda r: int(r["Dispatch_Id"]))

    n, shapes = info["hop_launches"], [tuple(x) for x in info["shapes"]]
    per_shape = {f"{b}/{o}": {} for b, o in shapes}
    factors = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rs = rows(path, counter)
        copy = [float(r["Counter_Value"]) for r in rs if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer")][:1]
        hop = [r for r in rs if "hop_kernel<0, 0, false, false, 0, 0," in r["Kernel_Name"]][-n * len(shapes):]
        assert len(copy) == 1 and len(hop) == n * len(shapes), (counter, len(copy), len(hop))
        factor = info["copy_bytes"] / 1024.0 / copy[0]
        factors[counter] = {"copy_kib": copy[0], "factor": round(factor, 4)}
        for i, (block, order) in enumerate(shapes):
            grp = hop[i * n:(i + 1) * n]
            assert all(int(r["Workgroup_Size"]) == block for r in grp), (counter, block, order)
            kib = sum(float(r["Counter_Value"]) for r in grp) / n
            per_shape[f"{block}/{order}"][counter] = round(kib * 1024.0 * factor)
    alg = info["hop_algorithmic_bytes"]
    for v in per_shape.values():
        v["bytes_per_launch"] = v["FETCH_SIZE"] + v["WRITE_SIZE"]
        v["ratio_to_algorithmic"] = round(v["bytes_per_launch"] / alg, 4)
    rec = {"source_sha": info["hop_source_sha"], "vh": alg // 1536, "algorithmic_bytes_per_launch": alg,
           "launches_per_shape": n, "calibration": factors, "shapes": per_shape}
    path = os.path.join(ROOT, "profiles", "hop_f64_24x24x24x48_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))


def bench_heatbath(T, synth, dev):
    """Pure-gauge sweeps (Wilson action, beta 5.7) on 24^3x48 and 32^3x64: time per heatbath and per
    overrelaxation sweep from HIP events, link updates per second, the FP64 flop rate in the paper's
    count (3912 / 3846 flops per link update, its Table 2), and the HBM roofline of a sweep: each of its
    8 launches (one direction and parity) reads the whole link field (the staples of the updated links
    touch every direction of both parities) and writes the links it updates, 8 x 576 + 8 x 72 = 5184
    algorithmic bytes per site and sweep."""
    import numpy as np
    import torch
    log("heatbath / overrelaxation sweeps")
    out = {}
    for dims in ((24, 24, 24, 48), (32, 32, 32, 64)):
        prob = T.Problem(dims, 0.15, 0.0, (1, 1, 1, -1))
        g = T.pack_gauge(prob, torch.from_numpy(synth.random_links(dims, 0.4, 91)).to(dev))
        for i in range(3):      # away from the start
            T.heatbath(prob, g, 5.7, 92, 1000 + i)
        counter = iter(range(10 ** 6))
        t_hb = _events_time(lambda: T.heatbath(prob, g, 5.7, 92, next(counter)), 10)
        t_or = _events_time(lambda: T.overrelax(prob, g), 10)
        links = 4 * prob.volume
        sweep_bytes = 5184 * prob.volume
        plaq = float(T.plaquette(prob, g)[0]) / (18 * prob.volume)
        # the same sweeps on FP32 links with FP32 arithmetic (the precision of the paper's measurement):
        # 2592 algorithmic bytes per site and sweep
        g32 = T.pack_gauge(prob, T.unpack_gauge(prob, g), T.F32)
        counter32 = iter(range(10 ** 6))
        t_hb32 = _events_time(lambda: T.heatbath(prob, g32, 5.7, 93, next(counter32), prec=T.F32), 10)
        t_or32 = _events_time(lambda: T.overrelax(prob, g32, prec=T.F32), 10)
        del g32
        fp32 = {"heatbath_ms": round(t_hb32 * 1e3, 3), "overrelax_ms": round(t_or32 * 1e3, 3),
                "heatbath_Glinks_s": round(links / t_hb32 / 1e9, 3), "overrelax_Glinks_s": round(links / t_or32 / 1e9, 3),
                "heatbath_TFLOP_s_paper_count": round(links * 3912 / t_hb32 / 1e12, 2),
                "overrelax_TFLOP_s_paper_count": round(links * 3846 / t_or32 / 1e12, 2),
                "roofline_heatbath": {"bound": "hbm", "achieved": round(2592 * prob.volume / t_hb32 / 1e9, 1),
                                      "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                                      "frac": round(2592 * prob.volume / t_hb32 / 1e9 / PEAK_HBM_GBPS, 4)}}
        out["x".join(map(str, dims))] = {
            "fp32": fp32,
            "heatbath_ms": round(t_hb * 1e3, 3), "overrelax_ms": round(t_or * 1e3, 3),
            "heatbath_Glinks_s": round(links / t_hb / 1e9, 3), "overrelax_Glinks_s": round(links / t_or / 1e9, 3),
            "heatbath_TFLOP_s_paper_count": round(links * 3912 / t_hb / 1e12, 2),
            "overrelax_TFLOP_s_paper_count": round(links * 3846 / t_or / 1e12, 2),
            "roofline_heatbath": {"bound": "hbm", "achieved": round(sweep_bytes / t_hb / 1e9, 1), "peak": PEAK_HBM_GBPS,
                                  "unit": "GB/s", "frac": round(sweep_bytes / t_hb / 1e9 / PEAK_HBM_GBPS, 4)},
            "roofline_overrelax": {"bound": "hbm", "achieved": round(sweep_bytes / t_or / 1e9, 1),
                                   "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                                   "frac": round(sweep_bytes / t_or / 1e9 / PEAK_HBM_GBPS, 4)},
            "plaquette_after": round(plaq, 5)}
        del g
    out["setup"] = ("FP64 RECON18 links (and FP32 links with FP32 arithmetic under fp32), Wilson action beta 5.7 "
                    "from the eps 0.4 start; 3 sweeps before timing")
    return out


def creutz_4x4x4x4(T, synth, dev, eo=False):
    """<exp(-dH)> over a 4^4 Markov chain (beta 5.5, kappa 0.15, mu 0.01, tau 0.5) after burn-in: the
    full-lattice action with 10 leapfrog steps, or (eo) the even-odd action with 4 outer 2MN steps of 2
    inner steps each."""
    import math

    import numpy as np
    import torch

    from paper_1209_5942_amd.hmc import HMC
    log(f"Creutz equality on 4^4 ({'even-odd, 2MN' if eo else 'leapfrog'})")
    dims = (4, 4, 4, 4)
    prob = T.Problem(dims, 0.15, 0.01, (1, 1, 1, -1))
    h = HMC(prob, torch.from_numpy(synth.random_links(dims, 0.3, 601).reshape(-1, 4, 3, 3)).to(dev), beta=5.5,
            tol=1e-12, md_tol=1e-10, eo=eo)
    rng = np.random.default_rng(602)
    dh, acc = [], 0
    for k in range(200):
        p = torch.from_numpy(synth.gaussian_momenta(prob.volume, 10000 + k)).to(dev)
        eta = torch.from_numpy(synth.gaussian_spinor(prob.volume // 2 if eo else prob.volume, 20000 + k)).to(dev)
        if eo:
            out = h.trajectory(p, eta, float(rng.random()), 4, 0.125, integrator="2mn", n_inner=2)
        else:
            out = h.trajectory(p, eta, float(rng.random()), 10, 0.05)
        if k >= 40:
            dh.append(out["dH"])
            acc += int(out["accepted"])
    e = np.exp(-np.array(dh))
    return {"exp_minus_dH_mean": round(float(e.mean()), 4),
            "exp_minus_dH_stderr": round(float(e.std(ddof=1) / math.sqrt(len(e))), 4),
            "acceptance": round(acc / len(dh), 3), "trajectories": len(dh), "burn_in": 40}


def counters_from(fetch_csv, write_csv, name, last_n):
    """Mean FETCH_SIZE and WRITE_SIZE bytes of the last N dispatches of a kernel, calibrated by the 1 GiB copy."""
    import csv
    out = {"kernel": name}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        with open(path) as fh:
            rows = sorted((r for r in csv.DictReader(fh) if r["Counter_Name"] == counter),
                          key=lambda r: int(r["Dispatch_Id"]))
        copy = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer")][0]
        factor = (1 << 30) / 1024.0 / copy
        v = [float(r["Counter_Value"]) for r in rows if name in r["Kernel_Name"]][-int(last_n):]
        out[counter] = {"factor": round(factor, 4), "dispatches": len(v),
                        "bytes_mean": round(sum(v) / len(v) * 1024.0 * factor)}
    print(json.dumps(out))


def mrhs_shapes_from_counters(fetch_csv, write_csv, kernel_log):
    """FETCH_SIZE / WRITE_SIZE bytes of the FP64 12-RHS hop in each pinned shape of --kernel-only mrhs
    (the calibration copy's factor applied), with the links' and spinors' share of the fetch; then the
    same for the launches in the shape the tuner chose (the ones before the pinned shapes)."""
    import csv
    with open(kernel_log) as fh:
        info = [json.loads(l) for l in fh if l.startswith("{")][-1]
    shapes, n = [tuple(x) for x in info["f64_shapes"]], info["f64_shape_launches"]
    pinned, tuned = n * len(shapes), info["launches"]
    links, spinors = info["vh"] * 1152, 12 * info["vh"] * 192   # FP64 RECON18 links (8 per output site), 12 half spinors
    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        with open(path) as fh:
            rs = sorted((r for r in csv.DictReader(fh) if r["Counter_Name"] == counter),
                        key=lambda r: int(r["Dispatch_Id"]))
        copy = [float(r["Counter_Value"]) for r in rs if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer")][0]
        factor = (1 << 30) / 1024.0 / copy
        v = [float(r["Counter_Value"]) * 1024.0 * factor for r in rs
             if "hop_mrhs_kernel<0, 0, false, false, 0>" in r["Kernel_Name"]][-(pinned + tuned):]
        assert len(v) == pinned + tuned, (counter, len(v))
        out.setdefault("tuned", {})[counter] = round(sum(v[:tuned]) / tuned)
        v = v[tuned:]
        for i, (order, group) in enumerate(shapes):
            out.setdefault(f"{order}/{group}", {})[counter] = round(sum(v[i * n:(i + 1) * n]) / n)
    tuned_shape = f'{info["f64"]["order"]}/{info["f64"]["group"]}'
    for key in [f"{o}/{g}" for o, g in shapes] + ["tuned"]:
        r = out[key]
        shape = tuned_shape if key == "tuned" else key
        sweeps = 1 if shape.endswith("/0") else 12 // int(shape.split("/")[1])
        r["spinor_fetch_ratio"] = round((r["FETCH_SIZE"] - sweeps * links) / spinors, 2)
        print(json.dumps({"shape": key if key != "tuned" else "tuned " + tuned_shape, **r}))


def durations_from_trace(path, name, last_n):
    """Duration statistics of the last N dispatches whose kernel name contains `name`."""
    import csv
    with open(path) as fh:
        rows = [r for r in csv.DictReader(fh) if name in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows[-int(last_n):]]
    last = rows[-1]
    print(json.dumps({"kernel": name, "dispatches": len(d), "mean_us": round(sum(d) / len(d), 2),
                      "min_us": round(min(d), 2), "max_us": round(max(d), 2),
                      "workgroup_size": last.get("Workgroup_Size", last.get("Workgroup_Size_X")),
                      "grid_size": last.get("Grid_Size", last.get("Grid_Size_X"))}))


def _events_time(fn, reps, warm=3):
    import torch
    for _ in range(warm):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def bench_multi_rhs(T, prob, U, dev):
    """12 spin-colour point sources through the odd<-even hop: one 12-RHS launch vs 12 launches."""
    import torch

    from paper_1209_5942_amd import synth
    log("multi-RHS hop, 12 point sources")
    vh = prob.volume // 2
    src = torch.from_numpy(synth.point_sources(vh, 0)).to(dev)
    U_dev = torch.from_numpy(U).to(dev)
    out = {}
    for p, r, pn in ((T.F64, 0, "f64_rec18"), (T.F64, 1, "f64_rec12"), (T.F32, 0, "f32_rec18"), (T.F32, 1, "f32_rec12")):
        g = T.pack_gauge(prob, U_dev, p, r)
        s = T.pack_spinor(prob, src, p, T.EVEN, nrhs=12)
        o = torch.empty(T.spinor_bytes(prob, p, T.ODD, 12), dtype=torch.uint8, device=dev)
        fi, fo = T.spinor_bytes(prob, p, T.EVEN), T.spinor_bytes(prob, p, T.ODD)
        # both sides in their tuned launch shapes
        tuned = T.tune_mrhs(prob, g, 12, p, r)
        T.tune(prob, g, p, r)
        t_multi = _events_time(lambda: T.dslash(prob, g, s, T.DSLASH_OE, p, r, nrhs=12, out=o), 20)

        def singles():
            for k in range(12):
                T.dslash(prob, g, s[k * fi:(k + 1) * fi], T.DSLASH_OE, p, r, out=o[k * fo:(k + 1) * fo])
        t_single = _events_time(singles, 10)
        link = BYTES_PER_SITE[(p, r)] - 2 * (192 if p == T.F64 else 96)
        spin = 2 * (192 if p == T.F64 else 96)
        out[pn] = {"multi_us": round(t_multi * 1e6, 1), "multi_order": tuned["order"], "multi_group": tuned["group"],
                   "multi_default_order_us": round(tuned["default_us"], 1),
                   "twelve_single_us": round(t_single * 1e6, 1),
                   "speedup": round(t_single / t_multi, 3),
                   "bytes_per_site_rhs": round(link / 12 + spin, 1),
                   "multi_GB_s": round(vh * (link + 12 * spin) / t_multi / 1e9, 1)}
    return out


def bench_cg_mrhs(T, synth, U, dev, check):
    """The 12 spin-colour point sources at the origin on 24^3 x 48 (the step's links, kappa 0.155, mu 0.01):
    one 12-RHS FP64 CG on Mhat^dag Mhat to 1e-10 (every operator application one multi-RHS launch) against
    12 single-RHS solves, both in their tuned launch shapes; each column's true residual recomputed by the
    C++ oracle, and column 0 against the oracle's own solution."""
    import numpy as np
    import torch
    log("12-RHS CG, point sources")
    dims, kappa, mu = WORKLOAD["dims"], 0.155, 0.01
    prob = T.Problem(dims, kappa, mu, (1, 1, 1, -1))
    vh = prob.volume // 2
    b = synth.point_sources(vh, 0)
    g = T.pack_gauge(prob, torch.from_numpy(U).to(dev))
    T.tune(prob, g, T.F64, T.RECON18)
    T.tune_mrhs(prob, g, 12, T.F64, T.RECON18)
    bp = T.pack_spinor(prob, torch.from_numpy(b).to(dev), T.F64, T.EVEN, nrhs=12)
    fe = T.spinor_bytes(prob, T.F64, T.EVEN)
    x = torch.empty(12 * fe, dtype=torch.uint8, device=dev)
    ws12 = T.workspace(prob, T.MHATDAGMHAT, 1, 12)
    ws1 = T.workspace(prob, T.MHATDAGMHAT, 1)

    def multi():
        return T.cg(prob, {T.F64: g}, bp, x, x_is_zero=True, tol=1e-10, op=T.MHATDAGMHAT, nrhs=12, ws=ws12,
                    check_every=16)[1]

    def singles():
        return [T.cg(prob, {T.F64: g}, bp[k * fe:(k + 1) * fe], x[k * fe:(k + 1) * fe], x_is_zero=True, tol=1e-10,
                     op=T.MHATDAGMHAT, ws=ws1, check_every=16)[1] for k in range(12)]

    res = {}
    for name, fn in (("twelve_single_solves", singles), ("multi_rhs_solve", multi)):
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = (dt, st) if best is None or dt < best[0] else best
        res[name + "_ms"] = round(1e3 * best[0], 2)
        res[name + "_iters"] = [s["iters"] for s in best[1]]
        res[name + "_hop_launches"] = best[1][0]["hop_launches"] if name == "multi_rhs_solve" else \
            sum(s["hop_launches"] for s in best[1])
    res["speedup"] = round(res["twelve_single_solves_ms"] / res["multi_rhs_solve_ms"], 3)
    log(f"12-RHS CG {res['multi_rhs_solve_ms']} ms vs 12 solves {res['twelve_single_solves_ms']} ms")
    if check:    # x holds the multi-RHS solution (its solve ran last)
        from oracle import cref
        xs = T.unpack_spinor(prob, x, T.F64, T.EVEN, 12).cpu().numpy()
        U64 = U.reshape(-1, 4, 3, 3)
        res["oracle_rel_residual"] = [cref.true_rel_residual("MHATDAGMHAT", U64, b[k], xs[k], dims, kappa, mu,
                                                             (1, 1, 1, -1)) for k in range(12)]
        x0, _ = oracle_solution("MHATDAGMHAT", U64, b[0], dims, kappa, mu)
        res["rel_error_vs_oracle_solution_column0"] = float(np.linalg.norm(xs[0] - x0) / np.linalg.norm(x0))
    res["workload"] = ("Mhat^dag Mhat x_k = b_k for the 12 spin-colour point sources at the origin, 24^3x48, "
                       "eps 0.5 links, kappa 0.155, mu 0.01, FP64, tol 1e-10")
    return res


def bench_small(T, synth, dev, check):
    """4^4 (eps 0.3, kappa 0.15, mu 0 and 0.01): every operator once (latency-bound: microseconds per call)
    and FP64 CG on M^dag M and Mhat^dag Mhat to 1e-10, each solution checked by the oracle: its true
    residual and its error against the dense LU solution."""
    import numpy as np
    import torch
    log("4^4 operators and solves")
    dims, kappa, bc = (4, 4, 4, 4), 0.15, (1, 1, 1, -1)
    U = synth.random_links(dims, 0.3, 1)
    out = {}
    for mu in (0.0, 0.01):
        prob = T.Problem(dims, kappa, mu, bc)
        g = T.pack_gauge(prob, torch.from_numpy(U).to(dev))
        rec = {"op_us": {}}
        for name, op in T.OPS.items():
            sub_in, _ = T.OP_SUBSETS[op]
            n = prob.volume // (1 if sub_in == T.FULL else 2)
            src = T.pack_spinor(prob, torch.from_numpy(synth.gaussian_spinor(n, 3)).to(dev), T.F64, sub_in)
            ws = T.workspace(prob, op, 1)
            rec["op_us"][name] = round(_events_time(lambda: T.dslash(prob, g, src, op, ws=ws), 50) * 1e6, 2)
        for op, name in ((T.MDAGM, "cg_MdagM"), (T.MHATDAGMHAT, "cg_MhatdagMhat")):
            n = prob.volume if op == T.MDAGM else prob.volume // 2
            b = synth.gaussian_spinor(n, 4)
            bp = T.pack_spinor(prob, torch.from_numpy(b).to(dev), T.F64, T.FULL if op == T.MDAGM else T.EVEN)
            T.cg(prob, {T.F64: g}, bp, tol=1e-10, op=op)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st, _ = T.cg(prob, {T.F64: g}, bp, tol=1e-10, op=op)
            torch.cuda.synchronize()
            r = {"us": round((time.perf_counter() - t0) * 1e6, 1), "iters": st["iters"],
                 "true_rel_residual": st["true_rel_residual"]}
            if check:
                from oracle import dirac as D
                xs = T.unpack_spinor(prob, x, T.F64, T.FULL if op == T.MDAGM else T.EVEN).cpu().numpy()
                A = (lambda v: D.apply_MdagM(U, v, dims, kappa, mu, bc)) if op == T.MDAGM else \
                    (lambda v: D.apply_MhatdagMhat(U, v, dims, kappa, mu, bc))
                r["oracle_rel_residual"] = D.true_rel_residual(A, b, xs)
                dense = D.dense_matrix(A, n)
                x_lu = np.linalg.solve(dense, b.reshape(-1)).reshape(b.shape)
                r["rel_error_vs_dense_lu"] = float(np.linalg.norm(xs - x_lu) / np.linalg.norm(x_lu))
            rec[name] = r
        out[f"mu_{mu:g}"] = rec
    return out


def bench_sizes(T, dev):
    """FP64 R18 odd<-even hop over the paper's grid of lattice sizes (N_s in 16..48, N_t in 4..16) and
    32^3x64, each in its tuned shape.  Timing only: links are random complex matrices drawn on the device."""
    import torch
    log("hop over lattice sizes")
    out = {}
    sizes = [(n, n, n, t) for n in (16, 24, 32, 48) for t in (4, 8, 12, 16)] + [(32, 32, 32, 64)]
    for dims in sizes:
        prob = T.Problem(dims, 0.16, 0.005, (1, 1, 1, -1))
        vh = prob.volume // 2
        g = torch.Generator(device=dev)
        g.manual_seed(5)
        gp = T.pack_gauge(prob, torch.randn((prob.volume, 4, 3, 3), dtype=torch.complex128, device=dev,
                                            generator=g))
        src = T.pack_spinor(prob, torch.randn((vh, 4, 3), dtype=torch.complex128, device=dev, generator=g),
                            T.F64, T.EVEN)
        o = torch.empty(T.spinor_bytes(prob, T.F64, T.ODD), dtype=torch.uint8, device=dev)
        best = T.tune(prob, gp, T.F64, T.RECON18)[0]
        t = _events_time(lambda: T.dslash(prob, gp, src, T.DSLASH_OE, out=o), 50)
        out["x".join(map(str, dims))] = {"us": round(t * 1e6, 2), "GB_s": round(vh * 1536 / t / 1e9, 1),
                                         "GFLOPS": round(vh * FLOPS_PER_SITE / t / 1e9, 1),
                                         "block": best["block"], "order": best["order"]}
        del gp, src, o
    return out


# Lattices of one batched solve.  Mixed volumes: the 16^3x32 member alone fills the chip's wave
# slots at the hop's one wave per SIMD (1024 waves of 64 half sites), so the batch needs a second
# round of waves.  Thermal lattices (short time extent, paper section 2.1): four together still fit
# one round, where each alone occupies a fraction of the chip.
BATCH_MIXED = [(8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32)]
BATCH_THERMAL = [(16, 16, 16, 4), (16, 16, 16, 6), (16, 16, 16, 8), (20, 20, 20, 4)]


def bench_batch(T, synth, dev, check=True, dims_list=BATCH_MIXED):
    """One batched solve over the lattices of dims_list (kappa 0.155, mu 0.01) with and without the
    hipGraph, against the same solves one after the other; the batched solutions checked by the C++
    oracle (true residual, error against its own solution)."""
    import torch
    log("batched CG over %d lattices" % len(dims_list))
    probs = [T.Problem(d, 0.155, 0.01, (1, 1, 1, -1)) for d in dims_list]
    n = len(probs)
    gauges, bs, hostf = [], [], []
    for k, (pr, d) in enumerate(zip(probs, dims_list)):
        Uh = synth.random_links(d, 0.4, 60 + k)
        bh = synth.gaussian_spinor(pr.volume // 2, 70 + k)
        hostf.append((Uh.reshape(-1, 4, 3, 3), bh))
        gauges.append(T.pack_gauge(pr, torch.from_numpy(Uh).to(dev)))
        bs.append(T.pack_spinor(pr, torch.from_numpy(bh).to(dev), T.F64, T.EVEN))
    side = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(side):
        xs = [torch.empty(T.spinor_bytes(pr, T.F64, T.EVEN), dtype=torch.uint8, device=dev) for pr in probs]
        cp = (T.CProblem * n)(*[pr.c() for pr in probs])
        ws = torch.empty(T.lib().tmqcd_cg_batch_workspace_bytes(n, cp), dtype=torch.uint8, device=dev)
        wss = [T.workspace(pr, T.MHATDAGMHAT, 1) for pr in probs]
        for name, fn in (
                ("graph_batch", lambda: T.cg_batch(probs, gauges, bs, xs, use_graph=True, ws=ws, stream=side)),
                ("eager_batch", lambda: T.cg_batch(probs, gauges, bs, xs, use_graph=False, ws=ws, stream=side)),
                ("separate_solves", lambda: [T.cg(pr, {T.F64: g}, b, x, x_is_zero=True, ws=w, stream=side)
                                             for pr, g, b, x, w in zip(probs, gauges, bs, xs, wss)])):
            best = None
            for _ in range(4):
                side.synchronize()
                t0 = time.perf_counter()
                r = fn()
                side.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            res[name + "_ms"] = round(best * 1e3, 3)
            if name == "graph_batch":
                res["iters"] = [st["iters"] for st in r[1]]
                res["true_rel_residual"] = [st["true_rel_residual"] for st in r[1]]
                sols = [T.unpack_spinor(pr, x, T.F64, T.EVEN, stream=side).cpu().numpy() for pr, x in zip(probs, xs)]
    if check:
        errs = []
        for pr, (Uh, bh), xh in zip(probs, hostf, sols):
            xst, _ = oracle_solution("MHATDAGMHAT", Uh, bh, pr.dims, pr.kappa, pr.mu)
            errs.append(oracle_error("MHATDAGMHAT", Uh, bh, xh, xst, pr.dims, pr.kappa, pr.mu))
        res["oracle_rel_residual"] = [e["oracle_rel_residual"] for e in errs]
        res["rel_error_vs_oracle_solution"] = [e["rel_error_vs_oracle_solution"] for e in errs]
    res["lattices"] = ["x".join(map(str, d)) for d in dims_list]
    res["sites"] = sum(pr.volume for pr in probs)
    res["speedup_graph_vs_separate"] = round(res["separate_solves_ms"] / res["graph_batch_ms"], 3)
    res["speedup_eager_vs_separate"] = round(res["separate_solves_ms"] / res["eager_batch_ms"], 3)
    return res


def bench_force_large(T, dev, read_gbs):
    """The fermion force kernel (FP64 RECON18) at 24^3x48 and 32^3x64 on random links and spinors (the
    values do not change the memory traffic): time per launch from HIP events, the compulsory bytes per
    site (4 links, X and Y once each, the 4 x 8 outputs: 1216 B) over it, against the 8 TB/s peak and the
    read rate measured in the same run."""
    import torch
    log("force kernel at 24^3x48 and 32^3x64")
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    out = {}
    for dims in ((24, 24, 24, 48), (32, 32, 32, 64)):
        prob = T.Problem(dims, 0.155, 0.01, (1, 1, 1, -1))
        v = prob.volume
        g = T.pack_gauge(prob, torch.randn((v, 4, 3, 3), dtype=torch.complex128, device=dev, generator=gen))
        X = T.pack_spinor(prob, torch.randn((v, 4, 3), dtype=torch.complex128, device=dev, generator=gen))
        Y = T.pack_spinor(prob, torch.randn((v, 4, 3), dtype=torch.complex128, device=dev, generator=gen))
        G = torch.empty((v, 4, 8), dtype=torch.float64, device=dev)
        t = _events_time(lambda: T.force(prob, g, X, Y, out=G), 20)
        gbs = v * (4 * 144 + 2 * 192 + 256) / t / 1e9
        out["x".join(map(str, dims))] = {"us": round(t * 1e6, 1), "GB_s": round(gbs, 1),
                                         "frac_of_8TB_s": round(gbs / PEAK_HBM_GBPS, 4),
                                         "frac_of_measured_read": round(gbs / read_gbs, 4)}
        del g, X, Y, G
    out["bytes_per_site"] = 1216
    return out


def bench_hmc(T, synth, dev):
    """16^3x32, eps 0.4, kappa 0.155, mu 0.01: force kernel times, 10 leapfrog trajectories (tau 1, 20 steps)
    of the full-lattice action and 10 two-level 2MN trajectories (tau 1, 10 outer steps) of the even-odd one."""
    import math

    import numpy as np
    import torch

    from paper_1209_5942_amd.hmc import HMC
    log("HMC 16^3x32")
    dims = (16, 16, 16, 32)
    prob = T.Problem(dims, 0.155, 0.01, (1, 1, 1, -1))
    U = torch.from_numpy(synth.random_links(dims, 0.4, 80)).to(dev)
    h = HMC(prob, U, beta=0.0, tol=1e-12, md_tol=1e-10)
    # the hop kernels in their tuned launch shapes on this lattice (FP64, and FP32 for the FP32-inner solves)
    T.tune(prob, h.U, T.F64, T.RECON18)
    T.tune(prob, T.pack_gauge(prob, U, T.F32), T.F32, T.RECON18)
    X = T.pack_spinor(prob, torch.from_numpy(synth.gaussian_spinor(prob.volume, 81)).to(dev))
    Y = T.pack_spinor(prob, torch.from_numpy(synth.gaussian_spinor(prob.volume, 82)).to(dev))
    G = torch.empty((prob.volume, 4, 8), dtype=torch.float64, device=dev)
    t_force = _events_time(lambda: T.force(prob, h.U, X, Y, out=G), 20)
    # compulsory bytes per site: 4 links, X and Y once each, the 4 x 8 outputs
    force_bytes = prob.volume * (4 * 144 + 2 * 192 + 256)
    # the even-odd force: three hops (X_o, Y_e = Mhat X_e, Y_o) and the force kernel
    Xe = T.pack_spinor(prob, torch.from_numpy(synth.gaussian_spinor(prob.volume // 2, 83)).to(dev), T.F64, T.EVEN)
    ws_eo = T._bytes(T.force_eo_workspace_bytes(prob), dev)
    t_force_eo = _events_time(lambda: T.force_eo(prob, h.U, Xe, out=G, ws=ws_eo), 20)
    # gauge forces: Wilson plaquettes and the tree-level Symanzik action (c1 = -1/12).  Two flop counts:
    # the paper's Table 2 per site and direction (plaquette force 2717, rectangle force 14813), and the
    # products these kernels execute at 198 flops per 3x3 complex product: Wilson 13 per link (6
    # staples of 2 products, U V); Symanzik 2 per stored staple (24 per site) plus, per link, 12
    # plaquette-staple additions, 18 rectangle staples of 2 products and U V (37 products)
    t_gauge_w = _events_time(lambda: T.gauge_force(prob, h.U, 3.9, out=G), 20)
    ws_sym = T._bytes(T.gauge_force_tlsym_workspace_bytes(prob), dev)
    t_gauge_s = _events_time(lambda: T.gauge_force_tlsym(prob, h.U, 3.9, -1.0 / 12.0, out=G, ws=ws_sym), 20)
    del ws_sym
    paper_w = 4 * prob.volume * 2717
    paper_s = 4 * prob.volume * (2717 + 14813)
    exec_w = 4 * prob.volume * 198 * 13
    exec_s = prob.volume * 198 * (24 * 2 + 4 * 37)

    def run(hmc, n_steps, integrator="leapfrog", n_inner=1):
        dh, acc = [], 0
        n_eta = prob.volume // 2 if hmc.eo else prob.volume
        t0 = time.perf_counter()
        for k in range(10):
            p = torch.from_numpy(synth.gaussian_momenta(prob.volume, 1000 + k)).to(dev)
            eta = torch.from_numpy(synth.gaussian_spinor(n_eta, 2000 + k)).to(dev)
            u = float(np.random.default_rng(3000 + k).random())
            hmc.U.copy_(U_start)   # every trajectory from the same start: dH of one field, two step sizes
            out = hmc.trajectory(p, eta, u, n_steps, 1.0 / n_steps, integrator=integrator, n_inner=n_inner)
            dh.append(out["dH"])
            acc += int(out["accepted"])
        torch.cuda.synchronize()
        return dh, acc / 10, (time.perf_counter() - t0) / 10

    U_start = h.U.clone()
    dh20, acc20, t_traj = run(h, 20)
    dh40, acc40, _ = run(h, 40)
    # the same 20-step trajectories with FP32-inner solves (same FP64 tolerances)
    h32 = HMC(prob, U, beta=0.0, tol=1e-12, md_tol=1e-10, inner_prec=T.F32)
    dh32, _, t_traj32 = run(h32, 20)
    # and with every solve started from the previous solution
    h32g = HMC(prob, U, beta=0.0, tol=1e-12, md_tol=1e-10, inner_prec=T.F32, guess=True)
    dh32g, _, t_traj32g = run(h32g, 20)
    # the even-odd action with the two-level 2MN integrator: 10 outer steps take 21 fermion forces, as
    # 20 leapfrog steps do; 20 outer steps for the dt^2 scaling; and with FP32-inner solves from the
    # previous solution
    heo = HMC(prob, U, beta=0.0, tol=1e-12, md_tol=1e-10, eo=True)
    dh_eo, acc_eo, t_eo = run(heo, 10, "2mn")
    it_eo = heo.cg_iters / max(1, heo.solves)
    dh_eo20, _, _ = run(heo, 20, "2mn")
    heo32g = HMC(prob, U, beta=0.0, tol=1e-12, md_tol=1e-10, eo=True, inner_prec=T.F32, guess=True)
    dh_eo32g, acc_eo32g, t_eo32g = run(heo32g, 10, "2mn")
    # the paper's production setting: even-odd action, tree-level Symanzik gauge action (beta 3.9,
    # c1 = -1/12) on the inner scale with 2 inner steps, FP32-inner solves from the previous solution
    hprod = HMC(prob, U, beta=3.9, tol=1e-12, md_tol=1e-10, eo=True, inner_prec=T.F32, guess=True, c1=-1.0 / 12.0)
    dh_prod, acc_prod, t_prod = run(hprod, 10, "2mn", n_inner=2)
    creutz = creutz_4x4x4x4(T, synth, dev)
    chain = thermalised_chain(T, synth, dev, prob, U)
    e = np.exp(-np.clip(np.array(dh20), -700, 700))
    ratio = float(np.mean(np.abs(dh20)) / np.mean(np.abs(dh40)))
    return {"force_us": round(t_force * 1e6, 1), "force_GB_s": round(force_bytes / t_force / 1e9, 1),
            "trajectory_s": round(t_traj, 3), "trajectory_s_fp32_inner": round(t_traj32, 3),
            "dH_fp32_inner_max_abs_diff": float(np.max(np.abs(np.array(dh32) - np.array(dh20)))),
            "trajectory_s_fp32_inner_guess": round(t_traj32g, 3),
            "dH_fp32_inner_guess_max_abs_diff": float(np.max(np.abs(np.array(dh32g) - np.array(dh20)))),
            "cg_iters_per_solve_fp32_inner": round(h32.cg_iters / max(1, h32.solves), 1),
            "cg_iters_per_solve_fp32_inner_guess": round(h32g.cg_iters / max(1, h32g.solves), 1),
            "dH": [round(x, 6) for x in dh20], "acceptance": acc20,
            "exp_minus_dH_mean": round(float(e.mean()), 4),
            "exp_minus_dH_stderr": round(float(e.std(ddof=1) / math.sqrt(len(e))), 4),
            "dH_40_steps": [round(x, 6) for x in dh40], "acceptance_40_steps": acc40,
            "mean_abs_dH_ratio_20_to_40_steps": round(ratio, 3),
            "cg_iters_per_solve": round(h.cg_iters / max(1, h.solves), 1),
            "creutz_4x4x4x4": creutz,
            "force_eo_us": round(t_force_eo * 1e6, 1),
            "gauge_force_wilson_us": round(t_gauge_w * 1e6, 1),
            "gauge_force_wilson_TFLOP_s_paper_count": round(paper_w / t_gauge_w / 1e12, 2),
            "gauge_force_wilson_TFLOP_s_executed": round(exec_w / t_gauge_w / 1e12, 2),
            "gauge_force_tlsym_us": round(t_gauge_s * 1e6, 1),
            "gauge_force_tlsym_TFLOP_s_paper_count": round(paper_s / t_gauge_s / 1e12, 2),
            "gauge_force_tlsym_TFLOP_s_executed": round(exec_s / t_gauge_s / 1e12, 2),
            "gauge_force_tlsym_executed_frac_of_fp64_peak": round(exec_s / t_gauge_s / 78.6e12, 4),
            "gauge_force_flop_counts": "paper: Table 2 per site and direction (2717 plaquette, 14813 rectangles); "
                                       "executed: 198 flops per 3x3 complex product the kernels perform",
            "eo_2mn_tlsym_beta3.9": {"trajectory_s": round(t_prod, 3), "acceptance": acc_prod,
                                     "mean_abs_dH": round(float(np.mean(np.abs(dh_prod))), 4),
                                     "cg_iters_per_solve": round(hprod.cg_iters / max(1, hprod.solves), 1),
                                     "setup": "even-odd action, tree-level Symanzik gauge action beta 3.9, "
                                              "c1 = -1/12, 10 outer 2MN steps of 2 inner steps, FP32-inner "
                                              "solves from the previous solution, tau 1"},
            "eo_2mn": {"trajectory_s": round(t_eo, 3), "dH": [round(x, 6) for x in dh_eo], "acceptance": acc_eo,
                       "mean_abs_dH": round(float(np.mean(np.abs(dh_eo))), 6),
                       "mean_abs_dH_ratio_10_to_20_outer_steps":
                           round(float(np.mean(np.abs(dh_eo)) / np.mean(np.abs(dh_eo20))), 3),
                       "cg_iters_per_solve": round(it_eo, 1),
                       "trajectory_s_fp32_inner_guess": round(t_eo32g, 3),
                       "acceptance_fp32_inner_guess": acc_eo32g,
                       "dH_fp32_inner_guess_max_abs_diff": float(np.max(np.abs(np.array(dh_eo32g) - np.array(dh_eo)))),
                       "cg_iters_per_solve_fp32_inner_guess": round(heo32g.cg_iters / max(1, heo32g.solves), 1),
                       "creutz_4x4x4x4": creutz_4x4x4x4(T, synth, dev, eo=True)},
            "thermalised_chain_eo_2mn_tlsym_beta3.9": chain,
            "leapfrog_mean_abs_dH": round(float(np.mean(np.abs(dh20))), 6),
            "setup": "two-flavour twisted-mass pseudofermion action (beta = 0), tau = 1 leapfrog with 20 steps "
                     "(and 40: second-order integrator, mean |dH| ratio near 4) from the eps 0.4 start, force solves "
                     "1e-10, acceptance solves 1e-12; eo_2mn: the even-odd action and the two-level 2MN "
                     "integrator with 10 outer steps (and 20), the same solver tolerances"}


def thermalised_chain(T, synth, dev, prob, U, n_traj=48, burn_in=16):
    """A Markov chain at 16^3x32 from a thermalised start: 40 heatbath + overrelaxation sweeps of the Wilson
    action at beta 5.9 from the eps 0.4 links, then the production setting (even-odd action, tree-level
    Symanzik gauge action beta 3.9, c1 = -1/12; 20 outer 2MN steps of 2 inner steps, tau 1; FP32-inner
    solves from the previous solution).  <exp(-dH)> over the trajectories after the burn-in (a 96-trajectory
    chain gave 0.91 over its first 16 trajectories, while the plaquette relaxed, and 0.98-1.04 over each
    later block of 16)."""
    import math

    import numpy as np
    import torch

    from paper_1209_5942_amd.hmc import HMC
    g = T.pack_gauge(prob, U)
    for sw in range(40):
        T.heatbath(prob, g, 5.9, 7, sw)
        T.overrelax(prob, g)
    per_plaq = 6 * prob.volume * 3.0
    plaq0 = float(T.plaquette(prob, g)[0]) / per_plaq
    Uth = T.unpack_gauge(prob, g).contiguous()
    del g
    h = HMC(prob, Uth, beta=3.9, tol=1e-12, md_tol=1e-10, eo=True, inner_prec=T.F32, guess=True, c1=-1.0 / 12.0)
    dh, acc = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_traj):
        p = torch.from_numpy(synth.gaussian_momenta(prob.volume, 5000 + k)).to(dev)
        eta = torch.from_numpy(synth.gaussian_spinor(prob.volume // 2, 6000 + k)).to(dev)
        u = float(np.random.default_rng(7000 + k).random())
        out = h.trajectory(p, eta, u, 20, 1.0 / 20, integrator="2mn", n_inner=2)
        dh.append(out["dH"])
        acc += int(out["accepted"])
    torch.cuda.synchronize()
    t_traj = (time.perf_counter() - t0) / n_traj
    e = np.exp(-np.array(dh[burn_in:]))
    return {"trajectory_s": round(t_traj, 3), "trajectories": n_traj, "burn_in": burn_in,
            "acceptance": round(acc / n_traj, 3), "dH": [round(x, 5) for x in dh],
            "exp_minus_dH_mean": round(float(e.mean()), 4),
            "exp_minus_dH_stderr": round(float(e.std(ddof=1) / math.sqrt(len(e))), 4),
            "plaquette_start": round(plaq0, 5),
            "plaquette_end": round(float(T.plaquette(prob, h.U)[0]) / per_plaq, 5),
            "cg_iters_per_solve": round(h.cg_iters / max(1, h.solves), 1),
            "setup": "40 heatbath + overrelaxation sweeps (Wilson beta 5.9) from the eps 0.4 links, then a chain "
                     "of even-odd 2MN trajectories (tree-level Symanzik beta 3.9, c1 = -1/12, kappa 0.155, "
                     "mu 0.01, 20 outer x 2 inner steps, tau 1, FP32-inner solves from the previous solution)"}


if __name__ == "__main__":
    main()
