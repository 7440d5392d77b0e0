#!/usr/bin/env python
"""Benchmark of the chi0 / E_c(q) path on one MI355X.

Default workload: the metal slab in its precision form - 9 x 9 x 36 bohr cell,
40 x 40 x 160 grid, 8 k-points (2 x 2 x 2, Gamma-centred, w_k = 1/8), 120 + 3000
plane-wave states per k (about 32,000 coefficients each) with Fermi-smeared
occupations (T = 0.01 Ha, every pair with f_n - f_m > 1e-8: about 0.9 million
transitions per k), 20 PAW atoms x 18 projectors, NG = 4011 G-vectors at
q = 0.1 x 2 pi/9 along x, 16 imaginary frequencies. Inputs are seeded synthetic
data of that shape, resident on the device before timing starts.

One step = the complete chi0 contribution of one k-point (Eq. chi0's k sum,
Table 1 steps 3-11): orbitals, pair densities (FP32 FFTs), PAW correction,
weights and the grouped rank-k update on BF16 (or FP16) hi/lo MFMA, added into
the q-point's chi0 (rpa_chi0 for the first k of a pass over the 8 k-points,
rpa_chi0_add for the others). ms/q-point = 8 steps + the E_c stage (FP64
Cholesky log-determinant and frequency sum, Eq. rpa), which is timed apart on
the chi0 of one complete pass.

value = useful chi0 flops (4 NG^2 P nw per k, the Hermitian complex count) per
second of the timed steps. The FP64 path is timed on the first --fp64-kpoints
k-points (default: all 8), and E_c(q) of split and FP64 is compared on the chi0
of those same k-points (the whole q-point by default).

--workload o2box runs the O2-in-box line instead (12 x 12 x 13 bohr, 48^3 grid,
16 + 800 states, NG ~ 1500, three q-points in one batched call per step), and
--workload qmesh the batching form (64 q-points with log-uneven spheres, NG
200-3000, on the slab cell at Gamma; one step = E_c of all 64 in one batched
call, timed against a loop of single-q calls), and --workload grad the
differentiation form (E_c(q) and its gradient with respect to eigenvalues,
coefficients and projections of all 16 + 800 states of the O2 box, FP64);
--workload spin, unfold, realfreq and metalq0 measure the two-channel
(spin-polarised) O2 box, sets unfolded from the irreducible zone by a symmetry
operation, chi0 at real frequencies, and the metal slab's q -> 0 head.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chi0 build TFLOP/s + ms/q-point for E_c at 1e-6 Ha, split-precision vs FP64"
PEAK_TFLOPS = {"split_bf16": 2500.0, "split_fp16": 2500.0, "fp64": 78.6}
HERK_KERNELS = {1: ("k_herk_split", "k_herk_split.hip"), 4: ("k_herk_split4", "k_herk_split2.hip"),
                5: ("k_herk_split5", "k_herk_split2.hip")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def npairs(s, t):
    return int(np.sum(s.f[:, None] - t.f[None, :] > 1e-8))


def measured_traffic(kernel, src, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary for this workload, if
    that summary was taken on the current source of the kernel (sha256 recorded in it); None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.md")
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


def executed_mfma_flops(variant, NG, P, nw):
    """MFMA flops the split kernel issues for one q and P pairs: its lower-triangle tiles incl. the diagonal,
    K padded to 32 per chunk (ignored here: chunks are large), 12 real 16-bit products per complex
    multiply-add (4 real products x 3 split terms)."""
    if variant >= 4:
        nr = (NG + 63) // 64
        elems = sum(i // 2 + 1 for i in range(nr)) * 64 * 128
    else:
        nT = (NG + 63) // 64
        elems = nT * (nT + 1) / 2 * 64 * 64
    return elems * nw * P * 12 * 2


# ------------------------------------------------------------------------------------------ CPU baseline
def _oracle_sample(path):
    """Child process: the FP64 oracle's chi0 build of the sample saved at `path`; prints one JSON line."""
    import oracle
    z = np.load(path)
    A, grid, q, ecut = z["A"], tuple(int(x) for x in z["grid"]), z["q"], float(z["ecut"])
    C, P, eps, f = z["C"], z["P"], z["eps"], z["f"]
    omega, wk, vol = z["omega"], float(z["wk"]), float(abs(np.linalg.det(z["A"])))
    times = []
    for _ in range(int(z["repeats"])):
        t0 = time.perf_counter()
        gm = oracle.gsphere(A, q, ecut)
        pairs = oracle.pair_list(f, f)
        phi = oracle.orbitals(C, z["miller"], grid)
        rho = oracle.pseudo_pair_density(phi, phi, pairs, gm, grid)
        rho += oracle.paw_correction(P, P, pairs, z["Q"], z["offsets"])
        a = oracle.transition_weights(eps, eps, f, f, pairs, wk, vol, omega)
        chi = oracle.chi0_grouped(rho, a)
        times.append(time.perf_counter() - t0)
    flops = 4.0 * len(gm) ** 2 * pairs[0].size * omega.size
    print(json.dumps({"times": times, "flops": flops, "pairs": int(pairs[0].size), "bands": int(C.shape[0]),
                      "NG": int(len(gm)), "chi0_max": float(np.abs(chi).max())}), flush=True)


def _oracle_grad_sample(path):
    """Child process: the FP64 oracle's E_c(q) and gradient (torch autograd on the CPU) of the sample saved
    at `path`; prints one JSON line."""
    import oracle
    import oracle.grad as G
    z = np.load(path)
    A, grid, q, ecut = z["A"], tuple(int(x) for x in z["grid"]), z["q"], float(z["ecut"])

    class S:
        pass
    s = S()
    s.C, s.P, s.eps, s.f, s.miller = z["C"], z["P"], z["eps"], z["f"], z["miller"]
    s.kpt, s.weight = z["kpt"], float(z["wk"])
    omega, ow = z["omega"], z["omega_weight"]
    times = []
    for _ in range(int(z["repeats"])):
        t0 = time.perf_counter()
        gm = oracle.gsphere(A, q, ecut)
        E, g = G.ec_and_grad(A, grid, s, s, gm, z["Q"], z["offsets"], q, omega, ow, False, (1.0, 0.0, 0.0), z["D"])
        times.append(time.perf_counter() - t0)
    P = int(oracle.pair_list(s.f, s.f)[0].size)
    flops = 12.0 * len(gm) ** 2 * P * omega.size
    print(json.dumps({"times": times, "flops": flops, "pairs": P, "bands": int(s.C.shape[0]), "NG": int(len(gm)),
                      "ec": E}), flush=True)


def cpu_baseline(wl, iq, band_stride, label, grad=False):
    """The FP64 oracle timed on the host on a band subset of k-point 0 (every band_stride-th band and all
    the transitions among them): median of 3 runs with every core, and one run in a child process pinned to
    one CPU with one BLAS thread. grad: E_c(q) and its gradient (the oracle's autograd reference) instead of
    the chi0 build."""
    import tempfile
    import synth
    s = wl.kpoints[0]
    qp = wl.qpoints[iq]
    keep = np.arange(0, s.nbands, band_stride)
    import paper_1307_8052_amd as rpa
    gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
    fd, path = tempfile.mkstemp(suffix=".npz")
    os.close(fd)
    base = dict(A=wl.A, grid=np.asarray(wl.grid), q=qp.q, ecut=qp.ecut, miller=s.miller, C=s.C[keep],
                P=s.P[keep], eps=s.eps[keep], f=s.f[keep], omega=wl.omega, wk=s.weight,
                Q=synth.paw_q_table(wl.paw, wl.A, qp.q, gm), offsets=wl.paw.offsets, kpt=s.kpt,
                omega_weight=wl.omega_weight, D=synth.paw_d_table(wl.paw))
    mode = "--oracle-grad-sample" if grad else "--oracle-sample"
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    try:
        np.savez(path, repeats=3, **base)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), mode, path],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(r.stderr[-2000:])
        allc = json.loads(r.stdout.strip().splitlines()[-1])
        one = None
        if hasattr(os, "sched_setaffinity"):
            np.savez(path, repeats=1, **base)
            cpu0 = sorted(os.sched_getaffinity(0))[0]
            env1 = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
            r1 = subprocess.run([sys.executable, os.path.abspath(__file__), mode, path],
                                capture_output=True, text=True, env=env1,
                                preexec_fn=lambda: os.sched_setaffinity(0, {cpu0}))
            if r1.returncode == 0:
                one = json.loads(r1.stdout.strip().splitlines()[-1])
    finally:
        os.unlink(path)
    med = float(np.median(allc["times"]))
    out = {"value": allc["flops"] / med / 1e12, "unit": "TFLOP/s", "cores": int(ncpu), "kind": "oracle",
           "sample": f"{label}: "
                     + ("E_c(q) and its gradient (torch autograd reference, eigenvalue log-determinant)"
                        if grad else "chi0 build (orbitals, pair densities, PAW, weights, grouped update)")
                     + f" of the {allc['pairs']} transitions among {allc['bands']} bands (every {band_stride}th "
                     f"band of k-point 0), NG = {allc['NG']}, {wl.omega.size} frequencies; median of "
                     f"{len(allc['times'])} runs {med:.1f} s",
           "seconds_median": med, "seconds_runs": allc["times"]}
    if one:
        out["one_core"] = {"value": one["flops"] / one["times"][0] / 1e12, "unit": "TFLOP/s", "cores": 1,
                           "seconds": one["times"][0]}
    return out


# ------------------------------------------------------------------------------------------ slab
def slab_inputs(rpa, wl, dev):
    import synth
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    ks = [rpa.States.from_synth(s, wl.paw, dev) for s in wl.kpoints]
    qp = wl.qpoints[0]
    gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
    qs = rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight, device=dev)
    return ks, qs, fr


def k_step(ctx, ks, qs, fr, chi, i, prec):
    """chi0 contribution of k-point i mod 8: overwrite at the first k of a pass, add for the others."""
    k = i % len(ks)
    if k == 0:
        out = ctx.chi0([ks[0]], [ks[0]], qs, fr, prec)
        chi.copy_(out)
        del out
    else:
        ctx.chi0_add([ks[k]], [ks[k]], qs, fr, chi, prec)


def run_slab(args, torch, rpa, synth):
    dev = "cuda:0"
    t = time.perf_counter()
    wl = synth.config2(device=dev)
    log(f"metal-slab workload generated in {time.perf_counter() - t:.1f} s")
    ks, qs, fr = slab_inputs(rpa, wl, dev)
    nk, nw, NG = len(ks), fr.nw, qs.NG
    P = [npairs(s, s) for s in wl.kpoints]
    flops_k = [4.0 * NG * NG * p * nw for p in P]
    log(f"NG = {NG}, pairs per k = {P}")
    ctx = rpa.Context(wl.A, wl.grid, device=0)
    prec = args.precision
    variant = ctx.tune_get(NG, prec)
    chi = torch.empty((nw, NG, NG), dtype=torch.complex128, device=dev)

    # the chi0 build for one k reuses the call's internal buffers: build them at full size with the
    # first rpa_chi0, so that no step allocates
    for i in range(args.warmup):
        k_step(ctx, ks, qs, fr, chi, i, prec)
        torch.cuda.synchronize()
    ctx.check()

    # timed steps: one k-point each, a pass over the 8 k-points every 8 steps
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        k_step(ctx, ks, qs, fr, chi, i, prec)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.check()
    prof = ctx.profile_get()
    ctx.profile(False)
    flops_timed = sum(flops_k[i % nk] for i in range(args.steps))
    value = flops_timed / dt / 1e12
    ms_step = dt / args.steps * 1e3
    log(f"split: {ms_step:.1f} ms per k-step, {value:.1f} TFLOP/s")
    log("stage ms (timed region): " + ", ".join(f"{k}={v[0]:.1f}/{v[1]}" for k, v in prof.items()))
    # complete the last pass untimed, so that chi holds the q-point's whole chi0 (one pass over the k-points)
    for i in range(args.steps, -(-args.steps // nk) * nk):
        k_step(ctx, ks, qs, fr, chi, i, prec)

    # E_c stage on the complete chi0 (second call timed)
    ec_full, F_full = ctx.ec_from_chi0(qs, fr, chi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ec_full, F_full = ctx.ec_from_chi0(qs, fr, chi)
    torch.cuda.synchronize()
    ms_ec = (time.perf_counter() - t0) * 1e3
    ctx.check()
    ec_split_full = float(ec_full.cpu()[0])
    ms_q = nk * ms_step + ms_ec
    log(f"E_c(q) split, all {nk} k-points: {ec_split_full:.12f} Ha; E_c stage {ms_ec:.1f} ms; {ms_q:.0f} ms/q")

    # FP64 on the first n64 k-points, split on the same ones, E_c of both partial sums
    n64 = max(0, min(args.fp64_kpoints, nk))
    fp64 = None
    if n64:
        chi64 = torch.empty_like(chi)
        ms64 = []
        ctx.profile(True)
        for i in range(n64):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k_step(ctx, ks, qs, fr, chi64, i, "fp64")
            torch.cuda.synchronize()
            ms64.append((time.perf_counter() - t0) * 1e3)
            log(f"fp64 k-step {i}: {ms64[-1]:.0f} ms")
        ctx.check()
        prof64 = ctx.profile_get()
        ctx.profile(False)
        e64, F64 = ctx.ec_from_chi0(qs, fr, chi64)
        ctx.check()
        ec64 = float(e64.cpu()[0])
        if n64 == nk:
            ecs = ec_split_full
        else:
            for i in range(n64):
                k_step(ctx, ks, qs, fr, chi, i, prec)
            es, _ = ctx.ec_from_chi0(qs, fr, chi)
            ctx.check()
            ecs = float(es.cpu()[0])
        del chi64
        ms_step64 = float(np.mean(ms64))
        herk64_ms, _ = prof64["herk"]
        herk64_flops = sum(flops_k[:n64])
        fp64 = {"value": sum(flops_k[:n64]) / (sum(ms64) * 1e-3) / 1e12, "unit": "TFLOP/s",
                "ms_per_k_step": ms_step64, "ms_per_q": nk * ms_step64 + ms_ec, "kpoints_timed": n64,
                "herk_tflops": herk64_flops / (herk64_ms * 1e-3) / 1e12,
                "herk_frac_of_fp64_peak": herk64_flops / (herk64_ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
                "stage_ms_per_k": {k: v[0] / n64 for k, v in prof64.items() if v[1]},
                "ec_partial": ec64, "ec_split_partial": ecs, "ec_split_minus_fp64_ha": ecs - ec64}
        log(f"fp64: {ms_step64:.0f} ms per k-step; E_c over k-points 0..{n64 - 1}: fp64 {ec64:.12f} "
            f"split {ecs:.12f} diff {ecs - ec64:.3e} Ha")

    # roofline of the split rank-k kernel over the timed steps
    stage_ms = {k: v[0] / args.steps for k, v in prof.items() if v[1]}
    dominant = max(stage_ms, key=stage_ms.get)
    herk_ms, herk_n = prof["herk"]
    achieved = flops_timed / (herk_ms * 1e-3) / 1e12
    executed = sum(executed_mfma_flops(variant, NG, P[i % nk], nw) for i in range(args.steps))
    peak = PEAK_TFLOPS[prec]
    kname, ksrc = HERK_KERNELS[variant]
    roofline = {"kernel": f"{kname} (grouped complex rank-k update of chi0, split {prec[6:]} hi/lo)",
                "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(kname, ksrc, "slab"), "avg_launch_ms": herk_ms / max(herk_n, 1),
                "launches": herk_n, "algorithmic_flops_per_launch": flops_timed / max(herk_n, 1),
                "executed_mfma_tflops": executed / (herk_ms * 1e-3) / 1e12,
                "executed_mfma_frac": executed / (herk_ms * 1e-3) / 1e12 / peak,
                "dominant_stage": dominant}
    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{prec[6:]}x3 MFMA / f32 FFT / f64 log-det",
        "data": "synthetic",
        "config": {"workload": "metal slab: 9x9x36 bohr, 40x40x160 grid, 8 k-points, 120+3000 Fermi-smeared "
                               "states per k (T = 0.01 Ha), 20x18 PAW projectors, NG = %d, 16 imaginary "
                               "frequencies; one step = one k-point's chi0 contribution" % NG,
                   "precision": prec, "NG": NG, "pairs_per_k": P, "nw": nw, "kpoints": nk},
        "ms_per_q": ms_q, "ms_ec_stage": ms_ec,
        "ec_split": ec_split_full,
        "ec_split_minus_fp64_ha": fp64 and fp64["ec_split_minus_fp64_ha"],
        "speedup_vs_fp64": fp64 and fp64["ms_per_q"] / ms_q,
        "stage_ms": stage_ms,
        "fp64": fp64,
        "roofline": roofline,
    }
    ctx.close()
    return out, wl


# ------------------------------------------------------------------------------------------ O2 box
def run_o2box(args, torch, rpa, synth):
    dev = "cuda:0"
    wl = synth.config1()
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    ks = [rpa.States.from_synth(s, wl.paw, dev) for s in wl.kpoints]
    qspecs = []
    for qp in wl.qpoints:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        qspecs.append(rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), optical=qp.optical,
                                qhat=qp.qhat, Dpaw=synth.paw_d_table(wl.paw), weight=qp.weight, device=dev))
    P = npairs(wl.kpoints[0], wl.kpoints[0])
    NGs = [q.NG for q in qspecs]
    nw = fr.nw
    flops_step = sum(4.0 * ng * ng * P * nw for ng in NGs)
    ctx = rpa.Context(wl.A, wl.grid, device=0)

    def steps(prec, n, profile=False):
        out = None
        if n <= 0:
            return 0.0, None, None
        torch.cuda.synchronize()
        if profile:
            ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(n):
            out = ctx.ec_batched(ks, ks, qspecs, fr, prec, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.check()
        prof = ctx.profile_get() if profile else None
        ctx.profile(False)
        return dt, [float(x) for x in out[0].cpu().numpy()[:len(qspecs)]], prof

    prec = args.precision
    variant = ctx.tune_get(NGs[0], prec)
    steps(prec, args.warmup)
    dt, ec_split, prof = steps(prec, args.steps, True)
    steps("fp64", 1)
    dt64, ec64, prof64 = steps("fp64", args.steps, True)
    ms_step, ms_step64 = dt / args.steps * 1e3, dt64 / args.steps * 1e3
    herk_ms, herk_n = prof["herk"]
    achieved = flops_step * args.steps / (herk_ms * 1e-3) / 1e12
    executed = sum(executed_mfma_flops(variant, ng, P, nw) for ng in NGs) * args.steps
    kname, ksrc = HERK_KERNELS[variant]
    peak = PEAK_TFLOPS[prec]
    out = {
        "metric": METRIC, "value": flops_step * args.steps / dt / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"{prec[6:]}x3 MFMA / f32 FFT / f64 log-det",
        "data": "synthetic",
        "config": {"workload": "O2-in-box: 12x12x13 bohr, 48^3 grid, Gamma, 16+800 states, 2x13 PAW projectors, "
                               "3 q-points (optical, 0.1, 0.2 x 2pi/12), 16 imaginary frequencies; one step = "
                               "E_c of the three q-points", "precision": prec, "NG": NGs, "pairs_per_q": P,
                   "nw": nw},
        "ms_per_q": ms_step / len(NGs), "ec_split": ec_split, "ec_fp64": ec64,
        "ec_split_minus_fp64_ha": [a - b for a, b in zip(ec_split, ec64)],
        "speedup_vs_fp64": ms_step64 / ms_step,
        "stage_ms": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
        "fp64": {"value": flops_step * args.steps / dt64 / 1e12, "unit": "TFLOP/s", "ms_per_step": ms_step64,
                 "ms_per_q": ms_step64 / len(NGs),
                 "stage_ms": {k: v[0] / args.steps for k, v in prof64.items() if v[1]}},
        "roofline": {"kernel": f"{kname} (grouped complex rank-k update of chi0, split {prec[6:]} hi/lo)",
                     "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(kname, ksrc, "o2box"),
                     "avg_launch_ms": herk_ms / max(herk_n, 1), "launches": herk_n,
                     "algorithmic_flops_per_launch": flops_step * args.steps / max(herk_n, 1),
                     "executed_mfma_tflops": executed / (herk_ms * 1e-3) / 1e12,
                     "executed_mfma_frac": executed / (herk_ms * 1e-3) / 1e12 / peak},
    }
    ctx.close()
    return out, wl


# --------------------------------------------------------------------------------------- q mesh
def run_qmesh(args, torch, rpa, synth):
    """The batching form: 64 q-points of a 4x4x4 mesh with log-uneven spheres (NG 200-3000) on the slab cell
    at Gamma, E_c of all of them in one batched call (per-class chi0 storage and factorisation) against a
    loop of single-q calls on the same inputs."""
    dev = "cuda:0"
    t = time.perf_counter()
    wl = synth.config3(n_occ=args.qmesh_bands[0], n_unocc=args.qmesh_bands[1], device=dev)
    log(f"q-mesh workload generated in {time.perf_counter() - t:.1f} s")
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    ks = [rpa.States.from_synth(s, wl.paw, dev) for s in wl.kpoints]
    qspecs = []
    for qp in wl.qpoints:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        qspecs.append(rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight,
                                device=dev))
    P = npairs(wl.kpoints[0], wl.kpoints[0])
    NGs = [q.NG for q in qspecs]
    nw = fr.nw
    flops = sum(4.0 * ng * ng * P * nw for ng in NGs)
    log(f"{len(NGs)} q-points, NG {min(NGs)}-{max(NGs)}, {P} pairs, {flops:.3e} useful chi0 flops per pass")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = rpa.Context(wl.A, wl.grid, device=0)
    prec = args.precision

    def batched(n):
        out = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            out = ctx.ec_batched(ks, ks, qspecs, fr, prec, out=out)
        torch.cuda.synchronize()
        ctx.check()
        return time.perf_counter() - t0, out[0].cpu().numpy()

    def loop(n):
        res = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            res = [ctx.ec(ks, ks, q, fr, prec)[0] for q in qspecs]
        torch.cuda.synchronize()
        ctx.check()
        return time.perf_counter() - t0, np.array([float(r.cpu()[0]) for r in res])

    batched(args.warmup)
    dt_b, ec_b = batched(args.steps)
    # stage times of one more batched pass (HIP events around each kernel group; outside the timed region)
    ctx.profile(True)
    batched(1)
    prof = ctx.profile_get()
    ctx.profile(False)
    # device memory held by the context after the batched call (chi0 sized per class of sphere sizes),
    # against chi0 alone padded to the largest sphere for every q
    used_b = free0 - torch.cuda.mem_get_info()[0]
    ldmax = -(-max(NGs) // 64) * 64
    padded_chi = len(NGs) * nw * ldmax * ldmax * 16
    log(f"batched: {dt_b / args.steps * 1e3:.1f} ms per pass of {len(NGs)} q")
    loop(args.warmup)
    dt_l, ec_l = loop(args.steps)
    log(f"per-q loop: {dt_l / args.steps * 1e3:.1f} ms per pass")
    ms_b, ms_l = dt_b / args.steps * 1e3, dt_l / args.steps * 1e3
    diff = float(np.max(np.abs(ec_b[:len(NGs)] - ec_l)))
    out = {
        "metric": METRIC, "value": flops * args.steps / dt_b / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"{prec[6:]}x3 MFMA / f32 FFT / f64 log-det",
        "data": "synthetic",
        "config": {"workload": f"q mesh: 9x9x36 bohr, 40x40x160 grid, Gamma, {args.qmesh_bands[0]}+"
                               f"{args.qmesh_bands[1]} states, 20x18 PAW projectors, 64 q-points of a 4x4x4 mesh, "
                               f"NG {min(NGs)}-{max(NGs)} (log-uneven), 16 imaginary frequencies; one step = E_c of "
                               f"all 64 q-points in one batched call", "precision": prec, "NG": NGs,
                   "pairs_per_q": P, "nw": nw},
        "ms_per_q": ms_b / len(NGs), "ms_per_step_per_q_loop": ms_l, "batched_speedup_vs_loop": ms_l / ms_b,
        "stage_ms_one_pass": {k: v[0] for k, v in prof.items() if v[1]},
        "stage_groups_one_pass": {k: v[1] for k, v in prof.items() if v[1]},
        "ec_batched_minus_loop_max_ha": diff, "ec_weighted_sum": float(ec_b[len(NGs)]),
        "device_bytes_after_batched_call": used_b, "chi0_bytes_if_padded_to_largest_sphere": padded_chi,
        "roofline": dict(_herk_roofline(prof, flops, prec, 1),
                         measured_on="the profiled batched pass after the timed ones (HIP events on the launch "
                                     "stream around each rank-k launch)"),
    }
    ctx.close()
    return out, wl


# --------------------------------------------------------------------------------------- gradient
def run_grad(args, torch, rpa, synth):
    """The differentiation form at O2-in-box size: E_c(q) and its gradient with respect to the eigenvalues,
    the plane-wave coefficients and the PAW projections of all 16 + 800 states at q = 0.1 x 2pi/12 (NG
    1500, 16 frequencies, FP64). One step = one rpa_ec_backward call: the FP64 forward pass (chi0, Cholesky),
    (1 - K)^-1 and W(omega), then per pair chunk the recomputed pair densities, the products W(omega) rho,
    the PAW, optical and FFT adjoints, and the coefficient transforms. Timed beside the FP64 forward call."""
    dev = "cuda:0"
    wl = synth.config1(which_q=(1,))
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    ks = [rpa.States.from_synth(s, wl.paw, dev) for s in wl.kpoints]
    qp = wl.qpoints[0]
    gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
    qs = rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), optical=qp.optical, qhat=qp.qhat,
                   Dpaw=synth.paw_d_table(wl.paw), weight=qp.weight, device=dev)
    P = npairs(wl.kpoints[0], wl.kpoints[0])
    NG, nw = qs.NG, fr.nw
    flops_chi, flops_wrho = 4.0 * NG * NG * P * nw, 8.0 * NG * NG * P * nw
    ctx = rpa.Context(wl.A, wl.grid, device=0)

    def grads(n, profile=False):
        ec = g = None
        torch.cuda.synchronize()
        if profile:
            ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(n):
            ec, g = ctx.ec_backward(ks[0], ks[0], qs, fr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.check()
        prof = ctx.profile_get() if profile else None
        ctx.profile(False)
        return dt, ec, g, prof

    def forward(n):
        e = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            e, _ = ctx.ec(ks, ks, qs, fr, "fp64")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e

    grads(args.warmup)
    dt, ec, g, prof = grads(args.steps, True)
    forward(1)
    dtf, ef = forward(args.steps)
    ms, msf = dt / args.steps * 1e3, dtf / args.steps * 1e3
    gemm_ms, gemm_n = prof["adjoint_gemm"]
    achieved = flops_wrho * args.steps / (gemm_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": (flops_chi + flops_wrho) * args.steps / dt / 1e12, "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "gradient of E_c(q) at O2-in-box size: 12x12x13 bohr, 48^3 grid, Gamma, 16+800 "
                               "states, 2x13 PAW projectors, q = 0.1 x 2pi/12, 16 imaginary frequencies; one step "
                               "= E_c(q) and dE_c/d(eps, C, P) of all states (FP64 forward and adjoint)",
                   "NG": NG, "pairs": P, "nw": nw},
        "value_counts": "chi0 (4 NG^2 P nw) + the adjoint's W(omega) rho products (8 NG^2 P nw) per gradient",
        "ms_per_gradient": ms, "ms_forward_fp64": msf, "gradient_over_forward": ms / msf,
        "ec_backward": float(ec.cpu()[0]), "ec_forward": float(ef.cpu()[0]),
        "grad_norms": {k: float(v.abs().square().sum().sqrt()) for k, v in g.items()},
        "stage_ms": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
        "roofline": {"kernel": "k_gemm_c64 (the adjoint's products W(omega) rho, complex FP64 MFMA)",
                     "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["fp64"], "traffic": None,
                     "avg_launch_ms": gemm_ms / max(gemm_n, 1), "launches": gemm_n,
                     "algorithmic_flops_per_launch": flops_wrho * args.steps / max(gemm_n, 1)},
    }
    ctx.close()
    return out, wl


# --------------------------------------------------------------------------------------- next rows
def _herk_roofline(prof, flops, prec, steps):
    herk_ms, herk_n = prof["herk"]
    achieved = flops * steps / (herk_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    return {"kernel": "grouped complex rank-k update of chi0 (" + ("FP64" if prec == "fp64" else
                                                                    f"split {prec[6:]} hi/lo") + ")",
            "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None, "avg_launch_ms": herk_ms / max(herk_n, 1), "launches": herk_n}


def _timed(ctx, torch, fn, n, profile=False):
    r = None
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(n):
        r = fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.check()
    prof = ctx.profile_get() if profile else None
    ctx.profile(False)
    return dt, r, prof


def run_spin(args, torch, rpa, synth):
    """Spin polarisation (Sec. 2.2: the spin index of Eq. chi0): the O2 box as a triplet, two channels of
    16 + 1 and 16 - 1 occupied states (f in [0, 1]) out of 816, q = 0.1 x 2pi/12; one step = E_c(q) from
    chi0 summed over both channels (one call with two state-set pairs)."""
    dev = "cuda:0"
    wl = synth.config1(which_q=(1,), spin_moment=2)
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    ks = [rpa.States.from_synth(s, wl.paw, dev) for s in wl.kpoints]
    qp = wl.qpoints[0]
    gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
    qs = rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight, device=dev)
    P = [npairs(s, s) for s in wl.kpoints]
    NG, nw = qs.NG, fr.nw
    flops = sum(4.0 * NG * NG * p * nw for p in P)
    ctx = rpa.Context(wl.A, wl.grid, device=0)
    prec = args.precision
    _timed(ctx, torch, lambda: ctx.ec(ks, ks, qs, fr, prec), args.warmup)
    dt, (ec, _), prof = _timed(ctx, torch, lambda: ctx.ec(ks, ks, qs, fr, prec), args.steps, True)
    _timed(ctx, torch, lambda: ctx.ec(ks, ks, qs, fr, "fp64"), 1)
    dt64, (ec64, _), _ = _timed(ctx, torch, lambda: ctx.ec(ks, ks, qs, fr, "fp64"), args.steps)
    out = {
        "metric": METRIC, "value": flops * args.steps / dt / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"{prec[6:]}x3 MFMA / f32 FFT / f64 log-det",
        "data": "synthetic",
        "config": {"workload": "spin-polarised O2 box: 12x12x13 bohr, 48^3 grid, two spin channels of 816 states "
                               "(17 and 15 occupied, f in [0, 1]), 2x13 PAW projectors, q = 0.1 x 2pi/12, 16 "
                               "imaginary frequencies; one step = E_c(q) summed over both channels",
                   "precision": prec, "NG": NG, "pairs_per_channel": P, "nw": nw},
        "ec_split": float(ec.cpu()[0]), "ec_fp64": float(ec64.cpu()[0]),
        "ec_split_minus_fp64_ha": float(ec.cpu()[0]) - float(ec64.cpu()[0]),
        "ms_per_step_fp64": dt64 / args.steps * 1e3, "speedup_vs_fp64": dt64 / dt,
        "stage_ms": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
        "roofline": _herk_roofline(prof, flops, prec, args.steps),
    }
    ctx.close()
    return out, wl


def run_unfold(args, torch, rpa, synth):
    """Symmetry unfolding (Eq. kmap, Eq. trans_wfs): a simple-cubic crystal (7 bohr, 48^3 grid, seven atoms
    with s + p projectors) whose k and k+q sets (16 + 400 states) come from the irreducible zone by a
    three-fold axis with time reversal; one step = E_c(q) from the unfolded sets (transformed plane-wave
    labels, conjugated coefficients, rotated projections) against the same call on the irreducible sets as
    they are (no operation), which differs only by the unfolding."""
    dev = "cuda:0"
    L = 7.0
    U = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]])
    tr, g0 = 1, (0, 0, 0)
    A = L * np.eye(3)
    B = 2 * np.pi * np.linalg.inv(A).T
    T = synth.cartesian_op(U, A)
    qf = (0.09, -0.05, 0.07)
    qv = np.asarray(qf) * 2 * np.pi / L
    k1 = np.array([0.11, 0.047, 0.023]) * 2 * np.pi / L
    k = -T @ k1
    k2 = -(T.T @ (k + qv))
    w = synth.symmetric_cubic([k1, k2], grid=(48, 48, 48), n_occ=16, n_unocc=400, target_ng=900, q=qf)
    amap, shift = synth.atom_images(U, w.atoms)
    D = synth.sp_rotation_blocks(U, A, len(w.atoms))
    fr = rpa.Freq(w.omega, w.omega_weight)
    s1, s2 = w.sets

    def lib(s, kpt, sym):
        op = rpa.SymOp(U, tr, g0, s.kpt, amap, shift, D) if sym else None
        return rpa.States(s.C, s.miller, s.eps, s.f, s.P, w.paw.offsets, kpt=kpt if sym else s.kpt,
                          weight=s.weight, device=dev, sym=op)
    a, b = lib(s1, k, True), lib(s2, k + qv, True)
    a0, b0 = lib(s1, None, False), lib(s2, None, False)
    gm = rpa.gsphere(w.A, w.grid, w.qpoint.q, w.qpoint.ecut)
    qs = rpa.QSpec(w.qpoint.q, gm, synth.paw_q_table(w.paw, w.A, w.qpoint.q, gm), weight=1.0, device=dev)
    P = npairs(s1, s2)
    NG, nw = qs.NG, fr.nw
    flops = 4.0 * NG * NG * P * nw
    ctx = rpa.Context(w.A, w.grid, device=0)
    prec = args.precision
    _timed(ctx, torch, lambda: ctx.ec([a], [b], qs, fr, prec), args.warmup)
    dt, (ec, _), prof = _timed(ctx, torch, lambda: ctx.ec([a], [b], qs, fr, prec), args.steps, True)
    _timed(ctx, torch, lambda: ctx.ec([a0], [b0], qs, fr, prec), 1)
    dt0, _, _ = _timed(ctx, torch, lambda: ctx.ec([a0], [b0], qs, fr, prec), args.steps)
    ms, ms0 = dt / args.steps * 1e3, dt0 / args.steps * 1e3
    out = {
        "metric": METRIC, "value": flops * args.steps / dt / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"{prec[6:]}x3 MFMA / f32 FFT / f64 log-det",
        "data": "synthetic",
        "config": {"workload": "symmetry unfolding: simple-cubic crystal 7 bohr, 48^3 grid, 7 atoms x 4 "
                               "projectors, k and k+q sets of 16+400 states unfolded from the irreducible zone by "
                               "a three-fold axis with time reversal, 16 imaginary frequencies; one step = E_c(q) "
                               "from the unfolded sets", "precision": prec, "NG": NG, "pairs": P, "nw": nw},
        "ec_unfolded": float(ec.cpu()[0]), "ms_per_step_without_unfolding": ms0,
        "unfolding_ms_per_step": ms - ms0,
        "stage_ms": {k2_: v[0] / args.steps for k2_, v in prof.items() if v[1]},
        "roofline": _herk_roofline(prof, flops, prec, args.steps),
    }
    ctx.close()
    return out, w


def run_realfreq(args, torch, rpa, synth):
    """Real frequencies (Sec. 5 outlook: chi0 for TDDFT, GW and BSE): chi0(q, w + i eta) of the O2 box at
    q = 0.1 x 2pi/12 for 16 frequencies in [0, 1] Ha with eta = 0.01 Ha (two Hermitian updates, Re a and
    Im a); one step = one rpa_chi0_real call, timed beside rpa_chi0 on the imaginary axis."""
    dev = "cuda:0"
    wl = synth.config1(which_q=(1,))
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    ks = [rpa.States.from_synth(s, wl.paw, dev) for s in wl.kpoints]
    qp = wl.qpoints[0]
    gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
    qs = rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight, device=dev)
    P = npairs(wl.kpoints[0], wl.kpoints[0])
    NG = qs.NG
    om = np.linspace(0.0, 1.0, 16)
    eta = 0.01
    flops = 2 * 4.0 * NG * NG * P * om.size
    ctx = rpa.Context(wl.A, wl.grid, device=0)
    prec = args.precision
    _timed(ctx, torch, lambda: ctx.chi0_real(ks, ks, qs, om, eta, prec), args.warmup)
    dt, _, prof = _timed(ctx, torch, lambda: ctx.chi0_real(ks, ks, qs, om, eta, prec), args.steps, True)
    _timed(ctx, torch, lambda: ctx.chi0(ks, ks, qs, fr, prec), 1)
    dti, _, _ = _timed(ctx, torch, lambda: ctx.chi0(ks, ks, qs, fr, prec), args.steps)
    out = {
        "metric": METRIC, "value": flops * args.steps / dt / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"{prec[6:]}x3 MFMA / f32 FFT",
        "data": "synthetic",
        "config": {"workload": "real frequencies: O2 box (12x12x13 bohr, 48^3 grid, 16+800 states, 2x13 PAW "
                               "projectors), q = 0.1 x 2pi/12, 16 frequencies w in [0, 1] Ha, eta = 0.01 Ha; one "
                               "step = chi0(q, w + i eta) of all frequencies", "precision": prec, "NG": NG,
                   "pairs": P, "nw": int(om.size)},
        "value_counts": "two Hermitian updates per frequency (Re a and Im a): 8 NG^2 P nw",
        "ms_per_step_imaginary_axis_chi0": dti / args.steps * 1e3,
        "stage_ms": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
        "roofline": _herk_roofline(prof, flops, prec, args.steps),
    }
    ctx.close()
    return out, wl


def run_metalq0(args, torch, rpa, synth):
    """The metallic q -> 0 head (Sec. 2.2 with Fermi-smeared bands): one k-point of the metal slab (120 +
    3000 states, T = 0.01 Ha) at the optical q-point (q -> 0 along x, the optical row of every pair and the
    intraband head from -df/de) against the same k-point at q = 0.1 x 2pi/9; one step = that k-point's chi0
    contribution."""
    dev = "cuda:0"
    wl = synth.config2(device=dev)
    ks, qs1, fr = slab_inputs(rpa, wl, dev)
    q0 = np.zeros(3)
    gm0 = rpa.gsphere(wl.A, wl.grid, q0, wl.qpoints[0].ecut)
    qs0 = rpa.QSpec(q0, gm0, synth.paw_q_table(wl.paw, wl.A, q0, gm0), optical=True, qhat=(1.0, 0.0, 0.0),
                    Dpaw=synth.paw_d_table(wl.paw), weight=1.0, device=dev)
    P = npairs(wl.kpoints[0], wl.kpoints[0])
    NG, nw = qs0.NG, fr.nw
    flops = 4.0 * NG * NG * P * nw
    ctx = rpa.Context(wl.A, wl.grid, device=0)
    prec = args.precision
    step0 = lambda: ctx.chi0([ks[0]], [ks[0]], qs0, fr, prec)
    step1 = lambda: ctx.chi0([ks[0]], [ks[0]], qs1, fr, prec)
    _timed(ctx, torch, step0, args.warmup)
    dt, chi, prof = _timed(ctx, torch, step0, args.steps, True)
    del chi
    _timed(ctx, torch, step1, 1)
    dt1, chi1, _ = _timed(ctx, torch, step1, args.steps)
    del chi1
    out = {
        "metric": METRIC, "value": flops * args.steps / dt / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"{prec[6:]}x3 MFMA / f32 FFT",
        "data": "synthetic",
        "config": {"workload": "metallic q -> 0: metal slab (9x9x36 bohr, 40x40x160 grid, 120+3000 Fermi-smeared "
                               "states, T = 0.01 Ha, 20x18 PAW projectors), k-point 0 at the optical q-point "
                               "(qhat = x, intraband head from -df/de), 16 imaginary frequencies; one step = that "
                               "k-point's chi0", "precision": prec, "NG": NG, "pairs": P, "nw": nw},
        "ms_per_step_at_q_0.1": dt1 / args.steps * 1e3,
        "stage_ms": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
        "roofline": _herk_roofline(prof, flops, prec, args.steps),
    }
    ctx.close()
    return out, wl


def main():
    if len(sys.argv) > 2 and sys.argv[1] == "--oracle-sample":
        _oracle_sample(sys.argv[2])
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--oracle-grad-sample":
        _oracle_grad_sample(sys.argv[2])
        return
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8, help="timed steps (slab: one k-point each)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="slab", choices=["slab", "o2box", "qmesh", "grad", "spin", "unfold",
                                                           "realfreq", "metalq0"])
    ap.add_argument("--qmesh-bands", type=int, nargs=2, default=(8, 60), metavar=("OCC", "UNOCC"),
                    help="qmesh: occupied and empty states at Gamma (the full form is 60 1500)")
    ap.add_argument("--precision", default="split_bf16", choices=["split_bf16", "split_fp16"])
    ap.add_argument("--fp64-kpoints", type=int, default=8,
                    help="slab: k-points run through the FP64 path for its timing and the E_c comparison "
                         "(8: the whole q-point)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); the path "
              f"shards over pair chunks or q-points with one reduce-scatter of chi0, which this program does not "
              f"launch.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1307_8052_amd as rpa

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "slab":
        out, wl = run_slab(args, torch, rpa, synth)
        band_stride, label = 80, "metal slab"
    elif args.workload == "qmesh":
        out, wl = run_qmesh(args, torch, rpa, synth)
        band_stride, label = 4, "q mesh q-point 0"
    elif args.workload == "grad":
        out, wl = run_grad(args, torch, rpa, synth)
        band_stride, label = 16, "gradient at O2-in-box size, q = 0.1"
    elif args.workload in ("spin", "unfold", "realfreq", "metalq0"):
        run = {"spin": run_spin, "unfold": run_unfold, "realfreq": run_realfreq,
               "metalq0": run_metalq0}[args.workload]
        out, wl = run(args, torch, rpa, synth)
        band_stride, label = 4, "spin-polarised O2 box, up channel, q = 0.1"
        # the oracle baseline of these lines: the spin channel's chi0 build (the unfolded and real-frequency
        # lines report their comparison calls instead)
        if args.workload != "spin":
            args.no_cpu_baseline = True
    else:
        out, wl = run_o2box(args, torch, rpa, synth)
        band_stride, label = 4, "O2-in-box q-point 0"
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl, 0, band_stride, label, grad=args.workload == "grad")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
