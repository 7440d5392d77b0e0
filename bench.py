#!/usr/bin/env python
"""Benchmark of the chi0 / E_c(q) path on one MI355X.

Workload: the O2-in-box configuration - 12 x 12 x 13 bohr cell, 48^3 grid, one
k-point (Gamma), 16 occupied + 800 unoccupied plane-wave states (about 11,900
coefficients each), 2 PAW atoms x 13 projectors, 1500-1503 G-vectors, 16
imaginary frequencies, three q-points (q -> 0 with the optical head, 0.1 and
0.2 x 2 pi / 12 along x). Inputs are seeded synthetic data of that shape and
are resident on the device before timing starts.

One step = E_c(q) for all three q-points through the C ABI: orbitals, pair
densities, PAW correction, optical row, weights, grouped rank-k update of
chi0 and the FP64 Cholesky log-determinant with the frequency sum.

value = useful chi0 flops (4 NG^2 P nw per q, the Hermitian complex count)
        per second of the whole step, split precision (FP32 FFT, BF16x3 MFMA).
The FP64 path is timed on the same inputs for the split-vs-FP64 comparison.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chi0 build TFLOP/s + ms/q-point for E_c at 1e-6 Ha, split-precision vs FP64"
PEAK_TFLOPS = {"split_bf16": 2500.0, "split_fp16": 2500.0, "fp64": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(rpa, wl, device):
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    ks = [rpa.States.from_synth(s, wl.paw, device) for s in wl.kpoints]
    import synth
    qspecs = []
    for qp in wl.qpoints:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
        qspecs.append(rpa.QSpec(qp.q, gm, Q, optical=qp.optical, qhat=qp.qhat, Dpaw=synth.paw_d_table(wl.paw),
                                weight=qp.weight, device=device))
    return ks, qspecs, fr


def run_steps(torch, ctx, ks, qspecs, fr, prec, steps, profile=False, use_graph=False):
    """`steps` passes of E_c(q) over all q-points (one batched call per step)."""
    if steps <= 0:
        return 0.0, None, None
    out = None
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.ec_batched(ks, ks, qspecs, fr, prec, use_graph=use_graph, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check()
    prof = ctx.profile_get() if profile else None
    if profile:
        ctx.profile(False)
    ecs = [float(x) for x in out[0].cpu().numpy()[: len(qspecs)]]
    return (t1 - t0), ecs, prof


HERK_KERNELS = {1: ("k_herk_split", "k_herk_split.hip"), 4: ("k_herk_split4", "k_herk_split2.hip"),
                5: ("k_herk_split5", "k_herk_split2.hip")}


def measured_traffic(kernel, src):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, if that summary was
    taken on the current source of the kernel (sha256 recorded in it); None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_o2box_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1307_8052_amd", "csrc", src), "rb").read()).hexdigest()
    if fields.get("source_sha256") != sha or "bytes_per_launch" not in fields:
        return None
    return float(fields["bytes_per_launch"])


def cpu_baseline(wl, iq=1, n_sample_occ=8):
    """The FP64 oracle on a bounded sample of the same workload: the chi0 build of
    q-point iq (orbitals, pair densities, PAW, weights, grouped update) for the
    pairs of the first n_sample_occ occupied states with every unoccupied state."""
    import oracle
    import synth
    try:
        import threadpoolctl
        blas = max((d.get("num_threads", 1) for d in threadpoolctl.threadpool_info()), default=1)
    except Exception:
        blas = 1
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    qp = wl.qpoints[iq]
    s = wl.kpoints[0]
    t0 = time.perf_counter()
    gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    phi = oracle.orbitals(s.C, s.miller, wl.grid)
    n_all, m_all = oracle.pair_list(s.f, s.f)
    sel = n_all < n_sample_occ
    pairs = (n_all[sel], m_all[sel])
    rho = oracle.pseudo_pair_density(phi, phi, pairs, gm, wl.grid)
    rho += oracle.paw_correction(s.P, s.P, pairs, Q, wl.paw.offsets)
    a = oracle.transition_weights(s.eps, s.eps, s.f, s.f, pairs, s.weight, wl.volume, wl.omega)
    chi = oracle.chi0_grouped(rho, a)
    t1 = time.perf_counter()
    P = pairs[0].size
    flops = 4.0 * len(gm) ** 2 * P * wl.omega.size
    return {"value": flops / (t1 - t0) / 1e12, "unit": "TFLOP/s", "cores": int(max(ncpu, blas)),
            "kind": "oracle",
            "sample": f"chi0 build of q-point {iq} (NG={len(gm)}) for {P} pairs (first {n_sample_occ} occupied "
                      f"states x all unoccupied), orbitals included; {t1 - t0:.1f} s",
            "seconds": t1 - t0, "chi0_norm": float(np.abs(chi).max())}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="split_bf16", choices=["split_bf16", "split_fp16"])
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 steps (default: steps)")
    ap.add_argument("--n-unocc", type=int, default=800)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--variant", type=int, default=0,
                    help="force the split rank-k kernel variant (1, 4, 5); 0 keeps the library's choice")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the per-q loop and adjoint timings")
    ap.add_argument("--cpu-sample-occ", type=int, default=8,
                    help="occupied states in the oracle's sample (all unoccupied states paired with each)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); the path "
              f"shards over pair chunks or q-points with one reduce-scatter of chi0, which this build does not "
              f"launch.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1307_8052_amd as rpa

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = "cuda:0"
    t = time.perf_counter()
    wl = synth.config1(n_unocc=args.n_unocc)
    log(f"workload generated in {time.perf_counter() - t:.1f} s")
    ks, qspecs, fr = make_inputs(rpa, wl, dev)
    P = int(np.sum(ks[0].f[:, None] - ks[0].f[None, :] > 1e-8))
    NGs = [qs.NG for qs in qspecs]
    nw = fr.nw
    flops_step = sum(4.0 * ng * ng * P * nw for ng in NGs)
    herk_flops_step = flops_step

    ctx = rpa.Context(wl.A, wl.grid, device=0)
    if args.variant:
        for ng in NGs:
            ctx.tune_set(ng, args.variant, args.precision)
    ctx_variant = ctx.tune_get(NGs[0], args.precision)
    # split path
    run_steps(torch, ctx, ks, qspecs, fr, args.precision, args.warmup)
    dt, ec_split, prof = run_steps(torch, ctx, ks, qspecs, fr, args.precision, args.steps, profile=True)
    ms_step = dt / args.steps * 1e3
    value = flops_step * args.steps / dt / 1e12
    log(f"split: {ms_step:.2f} ms/step, {value:.2f} TFLOP/s, E_c = {ec_split}")
    log("stage ms (timed region): " + ", ".join(f"{k}={v[0]:.2f}/{v[1]}" for k, v in prof.items()))
    # the same step replayed from a captured graph (launch overhead removed)
    ms_step_graph, ec_graph = None, None
    if not args.no_graph:
        run_steps(torch, ctx, ks, qspecs, fr, args.precision, 1, use_graph=True)
        dtg, ec_graph, _ = run_steps(torch, ctx, ks, qspecs, fr, args.precision, args.steps, use_graph=True)
        ms_step_graph = dtg / args.steps * 1e3
        log(f"split (graph replay): {ms_step_graph:.2f} ms/step")

    # the same q-points as a loop of single-q calls, and the adjoint of one q-point
    extras = {}
    if not args.no_extras:
        def loop_step():
            for qs in qspecs:
                ctx.ec(ks, ks, qs, fr, args.precision)
        loop_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            loop_step()
        torch.cuda.synchronize()
        extras["per_q_loop_ms_per_step"] = (time.perf_counter() - t0) / args.steps * 1e3
        log(f"per-q loop: {extras['per_q_loop_ms_per_step']:.2f} ms/step")
        ctx.ec_backward(ks[0], ks[0], qspecs[1], fr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ecb, _ = ctx.ec_backward(ks[0], ks[0], qspecs[1], fr)
        torch.cuda.synchronize()
        extras["adjoint_fp64_ms_q1"] = (time.perf_counter() - t0) * 1e3
        ctx.check()
        log(f"adjoint (FP64, q-point 1, E_c and dE_c/d(eps, C, P)): {extras['adjoint_fp64_ms_q1']:.1f} ms")

    # FP64 path on the same inputs
    k64 = args.fp64_steps if args.fp64_steps is not None else args.steps
    if k64 > 0:
        run_steps(torch, ctx, ks, qspecs, fr, "fp64", 1)
        dt64, ec64, prof64 = run_steps(torch, ctx, ks, qspecs, fr, "fp64", k64, profile=True)
        ms_step64 = dt64 / k64 * 1e3
        value64 = flops_step * k64 / dt64 / 1e12
        log(f"fp64: {ms_step64:.2f} ms/step, {value64:.2f} TFLOP/s, E_c = {ec64}")

    # roofline of the dominant kernel of the split step
    stage_ms = {k: v[0] / args.steps for k, v in prof.items()}
    dominant = max(stage_ms, key=stage_ms.get)
    herk_ms, herk_n = prof["herk"]
    # MFMA flops the split kernel issues: its lower-triangle tiles incl. the diagonal, K padded to 32,
    # 12 real 16-bit products per complex multiply-add (4 real products x 3 split terms)
    executed = 0.0
    for ng in NGs:
        if ctx_variant >= 4:
            nr = (ng + 63) // 64
            elems = sum(i // 2 + 1 for i in range(nr)) * 64 * 128
        else:
            tm = 64 if ctx_variant == 1 else 128
            nT = (ng + tm - 1) // tm
            elems = nT * (nT + 1) / 2 * tm * tm
        executed += elems * nw * ((P + 31) // 32 * 32) * 12 * 2
    executed *= args.steps
    herk_avg_ms = herk_ms / max(herk_n, 1)
    achieved = herk_flops_step * args.steps / (herk_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    variant = ctx_variant
    kname, ksrc = HERK_KERNELS[variant]
    roofline = {"kernel": f"{kname} (grouped complex rank-k update of chi0, variant {variant})", "bound": "mfma",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(kname, ksrc), "avg_launch_ms": herk_avg_ms, "launches": herk_n,
                "algorithmic_flops_per_launch": herk_flops_step / len(NGs),
                "executed_mfma_tflops": executed / (herk_ms * 1e-3) / 1e12,
                "executed_mfma_frac": executed / (herk_ms * 1e-3) / 1e12 / peak,
                "dominant_stage": dominant}
    fp64 = None
    if k64 > 0:
        herk64_ms, herk64_n = prof64["herk"]
        fp64 = {"value": value64, "unit": "TFLOP/s", "ms_per_step": ms_step64, "ms_per_q": ms_step64 / len(NGs),
                "steps": k64, "ec": ec64,
                "herk_tflops": herk_flops_step * k64 / (herk64_ms * 1e-3) / 1e12,
                "herk_frac_of_fp64_peak": herk_flops_step * k64 / (herk64_ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
                "stage_ms": {k: v[0] / k64 for k, v in prof64.items()}}

    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3 MFMA / f32 FFT / f64 log-det" if args.precision == "split_bf16"
        else "fp16x3 MFMA / f32 FFT / f64 log-det",
        "data": "synthetic",
        "config": {"workload": "O2-in-box: 12x12x13 bohr, 48^3 grid, Gamma, 16+%d states, 2x13 PAW projectors, "
                               "3 q-points (optical, 0.1, 0.2 x 2pi/12), 16 imaginary frequencies" % args.n_unocc,
                   "precision": args.precision, "NG": NGs, "pairs_per_q": P, "nw": nw},
        "ms_per_q": ms_step / len(NGs),
        "ec_split": ec_split, "ec_fp64": fp64 and fp64["ec"],
        "ec_split_minus_fp64_ha": fp64 and [a - b for a, b in zip(ec_split, fp64["ec"])],
        "ec_split_minus_fp64_rel": fp64 and [(a - b) / abs(b) for a, b in zip(ec_split, fp64["ec"])],
        "ms_per_step_graph": ms_step_graph,
        "ec_graph_equals_eager": None if ec_graph is None else ec_graph == ec_split,
        "speedup_vs_fp64": fp64 and fp64["ms_per_step"] / ms_step,
        **extras,
        "stage_ms": stage_ms,
        "fp64": fp64,
        "roofline": roofline,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl, n_sample_occ=args.cpu_sample_occ)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
