"""Benchmark: dual messenger Wiener filter solves on one MI355X.

One step = one complete solve (input screening, alpha, every cooling level of
xi with its iterations of the fused transform pair, Cauchy stopping) of the
paper-scale workload: HEALPix Nside 1024 (12,582,912 pixels), lmax 2048,
damped spectrum, ecliptic-modulated noise (sigma0 45 uK), 20% of the sky
masked, eps_final 1e-6, FP64.  Inputs are synthetic and resident in HBM
before the timed region.

Prints one JSON line.  Besides solves/s it reports the full-band transform pair
rate (one iteration at xi = alpha, l_iter = lmax), the roofline position of
the dominant kernel measured with HIP events around each of its launches on
the launch stream, and the CPU oracle on a bounded sample.  Further records:
configuration 3 with the Legendre contractions in FP32 and split-BF16x3 on the
matrix cores; the solves and pair rates of configurations 1 and 2 (Nside 16
and 256) with the oracle beside them; the batched workload (96 maps of
Nside 128, 256 and 512, one plan per Nside, the three solved from one graph)
in the three precision forms; and the learned warm start against the cold
start on 16 unseen Nside-512 maps.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X, 256 CU x 2.4 GHz x 128 FP64 flop/clk/CU
HBM_PEAK_GBS = 8000.0
METRIC = "Nside-1024 WF solves/s at 1e-6 residual; SHT pairs/s; plain vs mixed+learned"


def legendre_flops(nside: int, ell: int) -> float:
    """Algorithmic flops of one Legendre launch (one direction) at band limit ell:
    8 per (m, l, ring pair) triple = 4 for the recurrence, 4 for the complex contraction."""
    if ell < 0:
        return 0.0
    return 8.0 * (2 * nside) * (ell + 1) * (ell + 2) / 2.0


def make_inputs(nside, dev):
    import numpy as np
    import torch

    import dmwf_inputs as inp
    from paper_1702_08852_amd import Plan

    p = inp.make_problem("cfg3", nside=nside)
    plan = Plan(nside, p.lmax, device=dev)
    sig = plan.alm2map(torch.tensor(p.alm_true, device=dev))
    d = sig + torch.tensor(p.sigma * p.white, device=dev)
    mask = torch.tensor(p.mask, device=dev)
    d[mask] = 0.0
    w = torch.tensor(p.ninv, device=dev)
    cl = torch.tensor(p.cl, device=dev)
    torch.cuda.synchronize()
    return p, plan, cl, d.contiguous(), w, np


def cpu_baseline(nside, lmax, iters_per_solve, fraction):
    """Oracle FP64 transform pair at full band on a bounded sample, scaled.

    The oracle evaluates every iteration at full band (f_l = 0 masks modes above
    l_iter), so its solve costs iterations x one pair.  Sample: the synthesis on
    every k-th ring and the adjoint on every k-th m, scaled by the exact work
    ratio of the direct sums (Legendre terms plus phi terms).
    """
    import numpy as np

    import dmwf_inputs as inp
    import oracle

    k = max(1, int(round(1.0 / fraction)))
    cores = oracle.max_threads()
    z, st, nph, p0, start = oracle.rings(nside)
    nr = len(z)
    nalm = oracle.n_alm(lmax)
    rings = list(range(1, nr + 1, k))
    ms = list(range(0, lmax + 1, k))
    a = inp.random_alm(lmax, 4242)
    mp = inp.random_map(nside, 4243)
    # work units of the oracle's direct sums
    syn_all = nr * nalm + int(nph.sum()) * lmax
    syn_smp = len(rings) * nalm + int(sum(nph[r - 1] for r in rings)) * lmax
    ana_all = (lmax + 1) * int(nph.sum()) + nr * nalm
    ana_smp = len(ms) * int(nph.sum()) + nr * sum(lmax - m + 1 for m in ms)
    t0 = time.perf_counter()
    oracle.alm2map_rings(a, nside, lmax, rings, nthreads=cores)
    t1 = time.perf_counter()
    oracle.adjoint_m(mp, nside, lmax, ms, nthreads=cores)
    t2 = time.perf_counter()
    pair_s = (t1 - t0) * syn_all / syn_smp + (t2 - t1) * ana_all / ana_smp
    # the same oracle on one thread, on every 64th ring and m, scaled the same way
    r1 = list(range(1, nr + 1, 64))
    m1 = list(range(0, lmax + 1, 64))
    s1 = len(r1) * nalm + int(sum(nph[r - 1] for r in r1)) * lmax
    a1 = len(m1) * int(nph.sum()) + nr * sum(lmax - m + 1 for m in m1)
    t3 = time.perf_counter()
    oracle.alm2map_rings(a, nside, lmax, r1, nthreads=1)
    t4 = time.perf_counter()
    oracle.adjoint_m(mp, nside, lmax, m1, nthreads=1)
    t5 = time.perf_counter()
    oracle.adjoint_m(mp, nside, lmax, [0], nthreads=cores)  # the thread count back for later calls
    pair_1t = (t4 - t3) * syn_all / s1 + (t5 - t4) * ana_all / a1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": 1.0 / (pair_s * iters_per_solve),
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "extrapolated": True,
        "cpu_model": model,
        "one_thread": {"pair_seconds": pair_1t, "solves_per_s": 1.0 / (pair_1t * iters_per_solve),
                       "sample": (f"every 64th ring (synthesis) and m (adjoint) on one thread, "
                                  f"{t5 - t3:.1f} s measured, scaled by the work ratio")},
        "sample": ((f"one full-band FP64 oracle pair (synthesis on all rings, adjoint on all m) "
                    if k == 1 else
                    f"FP64 oracle synthesis on every {k}th ring and adjoint on every {k}th m, scaled "
                    f"by the exact work ratio to one full-band pair, ")
                   + f"at Nside {nside}, lmax {lmax}: {t2 - t0:.1f} s measured, {pair_s:.1f} s per "
                   f"pair, times the {iters_per_solve} iterations of the GPU solve"),
        "pair_seconds": pair_s,
    }


TRAFFIC_FILE = "profiles/hbm_traffic_fp64_nside1024_iteration.md"
TRAFFIC_KERNELS = {"legendre_analysis": "k_leg_ana", "legendre_synthesis": "k_leg_syn",
                   "ring_iter": "k_ring_fft", "harmonic_diag": "k_diag"}


def measured_traffic(kernel):
    """HBM bytes per launch of a kernel class from the committed counter summary.

    The summary holds lines 'traffic_json: {...}' with the calibrated bytes per
    launch of each kernel and the SHA-256 of its source file at the time the
    counters were taken; if the source has changed since, the figure no longer
    describes the kernel and None is returned.
    """
    import hashlib

    name = TRAFFIC_KERNELS.get(kernel)
    summ = os.path.join(ROOT, TRAFFIC_FILE)
    if name is None or not os.path.exists(summ):
        return None
    for line in open(summ):
        if not line.startswith("traffic_json:"):
            continue
        rec = json.loads(line.split(":", 1)[1])
        if rec.get("kernel") != name:
            continue
        src = os.path.join(ROOT, rec["source"])
        if not os.path.exists(src):
            return None
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("source_sha256"):
            return None
        return rec["bytes_per_launch"]
    return None


def copy_calibration(dev):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (reads and writes 2^30 bytes per launch)."""
    import torch

    n = (1 << 30) // 8
    src = torch.rand(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)  # an elementwise kernel, not a runtime blit
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 1 << 30, "launches": 5}))


def batch_inputs(nside, dev):
    """One Nside group of the batched workload: its members' C_l, data and
    N^-1 stacked on the device (each member draws its own mask and noise)."""
    import numpy as np
    import torch

    import dmwf_inputs as inp
    from paper_1702_08852_amd import Plan

    idx = inp.batch_members(nside)
    probs = [inp.make_problem("cfg4", nside=nside, index=k) for k in idx]
    lmax = probs[0].lmax
    syn = Plan(nside, lmax, nmaps=len(idx), device=dev)
    sig = syn.alm2map(torch.tensor(np.stack([q.alm_true for q in probs]), device=dev))
    noise = torch.tensor(np.stack([q.sigma * q.white for q in probs]), device=dev)
    mask = torch.tensor(np.stack([q.mask for q in probs]), device=dev)
    d = (sig + noise).masked_fill(mask, 0.0).contiguous()
    w = torch.tensor(np.stack([q.ninv for q in probs]), device=dev)
    cl = torch.tensor(np.stack([q.cl for q in probs]), device=dev)
    del syn
    return {"nside": nside, "lmax": lmax, "maps": len(idx), "cl": cl, "d": d, "w": w}


def pair_rate(pl, cl_, d_, w_, a_, pairs, with_kernels=True):
    """Full-band iteration time of a plan: iterations at xi = alpha replayed
    from a converged state as the solve loop runs them (graph replays), two
    lengths, the difference per extra iteration; the per-kernel split from
    the same replays launched one by one with kernel timing on."""
    import torch

    def run(n, prof):
        pl.profile(prof)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl.solve(cl_, d_, w_, eps_final=1e-6, start_final=True, alm=a_.clone(), replay=[n])
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) * 1e3
        pr = pl.profile_read() if prof else None
        pl.profile(False)
        return t, pr
    n0, n1 = 5, 5 + pairs
    run(n0, False)
    t0, t1 = run(n0, False)[0], run(n1, False)[0]
    kern = None
    if with_kernels:
        p0, p1 = run(n0, True)[1], run(n1, True)[1]
        kern = {k: (p1[k][1] - p0[k][1]) / pairs for k in p1 if p1[k][0]}
    return (t1 - t0) / pairs, kern


def bench_configs(dev, with_cpu):
    """Configurations 1 and 2 (Nside 16, lmax 32, eps 1e-8; Nside 256, lmax 512,
    eps 1e-6): one full solve each as a user runs it (graph replays, no kernel
    timing) and the full-band pair rate, with the oracle beside them: the full
    oracle solve at Nside 16, one oracle pair times the GPU's iteration count
    at Nside 256 (extrapolated)."""
    import numpy as np
    import torch

    import dmwf_inputs as inp
    import oracle
    from oracle import dm
    from paper_1702_08852_amd import Plan

    out = {}
    for name in ("cfg1", "cfg2"):
        p = inp.make_problem(name)
        nside, lmax = p.nside, p.lmax
        plan = Plan(nside, lmax, device=dev)
        sig = plan.alm2map(torch.tensor(p.alm_true, device=dev))
        d = (sig + torch.tensor(p.sigma * p.white, device=dev)).masked_fill(
            torch.tensor(p.mask, device=dev), 0.0).contiguous()
        w = torch.tensor(p.ninv, device=dev)
        cl = torch.tensor(p.cl, device=dev)
        plan.solve(cl, d, w, eps_final=p.eps_final, max_iter=20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        alm, _, st = plan.solve(cl, d, w, eps_final=p.eps_final, eps_coarse=1e-4)
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t0

        def run(n):
            torch.cuda.synchronize()
            t = time.perf_counter()
            plan.solve(cl, d, w, eps_final=p.eps_final, start_final=True, alm=alm.clone(),
                       replay=[n])
            torch.cuda.synchronize()
            return time.perf_counter() - t

        run(5)
        pair_ms = (run(205) - run(5)) / 200 * 1e3
        rec = {"nside": nside, "lmax": lmax, "eps_final": p.eps_final, "solve_s": solve_s,
               "iterations": st.n_iter, "levels": st.n_levels,
               "wf_residual": plan.wf_residual(cl, d, w, alm), "ms_per_pair": pair_ms,
               "pairs_per_s": 1e3 / pair_ms,
               "gate": "Cauchy ratio < eps_final at xi = alpha (Algorithm 2's stopping rule)",
               "residual_target": p.eps_final}
        rec["residual_target_met"] = bool(rec["wf_residual"] <= p.eps_final)
        if not rec["residual_target_met"]:
            # Continue the last level (xi = alpha) from the solution with a
            # tenfold tighter Cauchy tolerance until the FP64 residual meets
            # the figure the configuration names (at most four rounds).
            a_c, eps_c, iters, t_c = alm, p.eps_final, 0, 0.0
            resid = rec["wf_residual"]
            rounds = 0
            while resid > p.eps_final and rounds < 4:
                eps_c /= 10.0
                rounds += 1
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                a_c, _, st_c = plan.solve(cl, d, w, eps_final=eps_c, start_final=True,
                                          alm=a_c.clone())
                torch.cuda.synchronize()
                t_c += time.perf_counter() - t0
                iters += st_c.n_iter
                resid = plan.wf_residual(cl, d, w, a_c)
            rec["residual_continuation"] = {
                "how": "last level continued from the solution, Cauchy tolerance / 10 per round",
                "rounds": rounds, "final_eps": eps_c, "extra_iterations": iters,
                "extra_seconds": t_c, "wf_residual": resid,
                "residual_target_met": bool(resid <= p.eps_final)}
        if with_cpu:
            T = oracle.SphereTransforms(nside, lmax)
            dh, wh = d.cpu().numpy(), w.cpu().numpy()
            if name == "cfg1":
                t0 = time.perf_counter()
                ref = dm.solve(T, dh, wh, p.cl, eps_final=p.eps_final, eps_coarse=1e-4)
                cpu_s = time.perf_counter() - t0
                rec["cpu_oracle"] = {"solve_s": cpu_s, "iterations": ref.n_iter,
                                     "kind": "full oracle solve", "cores": oracle.max_threads()}
            else:
                t0 = time.perf_counter()
                T.adjoint(T.synth(p.alm_true))
                pair_s = time.perf_counter() - t0
                rec["cpu_oracle"] = {"solve_s": pair_s * st.n_iter, "pair_s": pair_s,
                                     "kind": "one oracle pair times the GPU iteration count "
                                             "(extrapolated)", "cores": oracle.max_threads()}
        out[name] = rec
        del plan
    return out


# FP64 residual the batched workload names for every map
BATCH_RESIDUAL = 1e-6


def bench_batch(dev, pairs):
    """The batched workload: 96 maps of Nside {128: 48, 256: 32, 512: 16}, lmax
    2 Nside, each with its own mask and noise.  One plan per Nside group; all
    three solved together by dmwf_solve_plans (one HIP graph replayed for every
    iteration of every group, device-side stops per map), in each precision
    form of the Legendre contractions: FP64, FP32 on the matrix cores and
    split-BF16x3 on the matrix cores (the reduced forms hand every map's last
    level over to FP64, so all three stop on the same FP64 Cauchy test).
    Reported per form: maps/s, iterations, the FP64 residual of every map and,
    for the reduced forms, the distance to the FP64 form's solution; per group
    the full-band iteration time of the batch."""
    import numpy as np
    import torch

    import dmwf_inputs as inp
    from paper_1702_08852_amd import BF16X3_GEMM, FP32_GEMM, FP64, Plan, solve_plans

    inputs = [batch_inputs(ns, dev) for ns, _ in inp.BATCH_GROUPS]
    nm_all = sum(g["maps"] for g in inputs)
    forms = {}
    ref = None
    for prec, name in ((FP64, "fp64"), (FP32_GEMM, "fp32_gemm"), (BF16X3_GEMM, "bf16x3_gemm")):
        plans = [Plan(g["nside"], g["lmax"], nmaps=g["maps"], device=dev, precision=prec)
                 for g in inputs]
        tiles = [pl.autotune()[0] for pl in plans]
        args = ([g["cl"] for g in inputs], [g["d"] for g in inputs], [g["w"] for g in inputs])
        solve_plans(plans, *args, eps_final=1e-6, max_iter=20)  # warm-up: graph, tables
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = solve_plans(plans, *args, eps_final=1e-6, eps_coarse=1e-4)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        groups = []
        for g, pl, tile, (alm, smap, sts) in zip(inputs, plans, tiles, res):
            resid = pl.wf_residual(g["cl"], g["d"], g["w"], alm)
            rec = {"nside": g["nside"], "maps": g["maps"],
                   "iterations_mean": float(np.mean([x.n_iter for x in sts])),
                   "iterations_max": int(max(x.n_iter for x in sts)),
                   "reduced_iterations_mean": float(np.mean([x.iters_reduced for x in sts])),
                   "converged": all(x.status == 0 for x in sts),
                   "wf_residual_max": float(max(resid)),
                   "wf_residual_median": float(np.median(resid)),
                   "maps_meeting_residual_target": int(sum(r <= BATCH_RESIDUAL for r in resid)),
                   "legendre_tiles": list(tile)}
            it_ms, kern = pair_rate(pl, g["cl"], g["d"], g["w"], alm, pairs)
            rec["batch_iteration_ms"] = it_ms
            rec["batch_kernel_ms_per_iteration"] = kern
            rec["pair_ms_per_map"] = it_ms / g["maps"]
            if prec == FP64:
                one = Plan(g["nside"], g["lmax"], nmaps=1, device=dev)
                single, _ = pair_rate(one, g["cl"][0].contiguous(), g["d"][0].contiguous(),
                                      g["w"][0].contiguous(), alm[0].contiguous(), pairs,
                                      with_kernels=False)
                rec["single_map_pair_ms"] = single
                rec["batch_gain_per_map"] = single / (it_ms / g["maps"])
                rec["frac_of_fp64_peak"] = (2 * legendre_flops(g["nside"], g["lmax"]) * g["maps"]
                                            / (it_ms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS)
                del one
            groups.append(rec)
        rec = {"seconds": secs, "maps_per_s": nm_all / secs, "groups": groups,
               "wf_residual_max": max(x["wf_residual_max"] for x in groups),
               "maps_meeting_residual_target": sum(x["maps_meeting_residual_target"]
                                                   for x in groups)}
        alms = [r[0] for r in res]
        if ref is None:
            ref = [a.clone() for a in alms]
        else:
            errs = [float((torch.linalg.vector_norm(a[k] - r[k]) / torch.linalg.vector_norm(r[k])).item())
                    for a, r in zip(alms, ref) for k in range(a.shape[0])]
            rec["rel_l2_to_fp64_solution_max"] = max(errs)
            rec["rel_l2_to_fp64_solution_mean"] = float(np.mean(errs))
        forms[name] = rec
        print(f"batch {name}: {nm_all} maps in {secs:.2f} s", file=sys.stderr, flush=True)
        del plans, res, alms
        torch.cuda.empty_cache()
    return {"workload": ("batched: 96 maps, Nside {128: 48, 256: 32, 512: 16}, lmax 2 Nside, "
                         "damped C_l, own |b| cut U[5,20] deg + U{50..500} holes of 1 deg and "
                         "sigma0 U[10,60] uK x lognormal(0, 0.25) per map, eps_final 1e-6"),
            "maps": nm_all,
            "measured_as": ("three plans (one per Nside) solved by dmwf_solve_plans: one HIP graph "
                            "holds an iteration of every plan and is replayed; per-map device "
                            "control; the host waits once per batch of iterations"),
            "gate": "Cauchy ratio < eps_final at xi = alpha, judged on an FP64 iteration",
            "residual_target": BATCH_RESIDUAL,
            "residual_note": ("the solves stop on the Cauchy ratio; maps_meeting_residual_target "
                              "counts the maps whose FP64 residual also meets the figure the "
                              "workload names"),
            "seconds": forms["fp64"]["seconds"], "maps_per_s": forms["fp64"]["maps_per_s"],
            "forms": forms}


def precision_legs(nside, lmax, cl, d, w, alm64, smap64, pairs, eps_final, eps_coarse):
    """Configuration 3 with the Legendre contractions in the reduced forms
    (FP32 and split-BF16x3 on the matrix cores; recurrence, Cauchy sums and
    residual in FP64).  The solve hands the last level over to FP64, so it
    stops on the same FP64 Cauchy test as the FP64 solve; reported: time,
    iterations (reduced and all), the FP64 residual, the distance to the FP64
    solution, and the full-band iteration time in the reduced form."""
    import torch

    from paper_1702_08852_amd import BF16X3_GEMM, FP32_GEMM, Plan

    out = {}
    for prec, name in ((FP32_GEMM, "fp32_gemm"), (BF16X3_GEMM, "bf16x3_gemm")):
        pl = Plan(nside, lmax, device=d.device, precision=prec)
        pl.solve(cl, d, w, eps_final=eps_final, max_iter=10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        alm, smap, st = pl.solve(cl, d, w, eps_final=eps_final, eps_coarse=eps_coarse,
                                 want_residual=True)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        it_ms, kern = pair_rate(pl, cl, d, w, alm, pairs)
        rl2 = lambda x, y: float((torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y)).item())
        out[name] = {"solve_s": secs, "solves_per_s": 1.0 / secs, "iterations": st.n_iter,
                     "reduced_iterations": st.iters_reduced, "levels": st.n_levels,
                     "final_cauchy": st.final_cauchy, "wf_residual": st.wf_residual,
                     "rel_l2_alm_to_fp64_solution": rl2(alm, alm64),
                     "rel_l2_map_to_fp64_solution": rl2(smap, smap64),
                     "reduced_pair_ms": it_ms, "reduced_kernel_ms_per_pair": kern}
        print(f"config 3 {name}: {secs:.2f} s, {st.n_iter} iterations ({st.iters_reduced} "
              f"reduced)", file=sys.stderr, flush=True)
        del pl
        torch.cuda.empty_cache()
    return out


def learned_warm_start(dev):
    """The learned warm start on its evaluation workload (16 unseen Nside-512
    maps of configuration 2's shape, eps_final 1e-6): cold solves against
    solves entering from the network's estimate at the last level and at the
    first level of the cooling schedule.  The network is the committed one,
    trained by the library's own kernels on 2000 Nside-256 solves (its
    training record is in profiles/)."""
    from paper_1702_08852_amd import warmstart

    path = warmstart.DEFAULT_WEIGHTS
    if not os.path.exists(path):
        return None
    net = warmstart.load_net(path, dev)
    log = lambda msg: print(f"warm start {msg}", file=sys.stderr, flush=True)
    rec = warmstart.evaluate(net, dev, log=log)
    rec["network"] = "24 -> 128 -> 128 -> 2, FP32, per (l, m) mode"
    train = os.path.join(ROOT, "profiles", "warmstart_training_nside256_2000maps.md")
    if os.path.exists(train):
        for line in open(train):
            if line.startswith("training_json:"):
                rec["training_record"] = json.loads(line.split(":", 1)[1])
    return rec


def probe(dev, nside, maps, precision, iters):
    """A short fixed workload for profiler runs: `iters` full-band iterations
    at xi = alpha (replayed, graph launches) of one plan of `maps` maps of
    configuration 3's recipe at this Nside (the batched workload's recipe for
    several maps), from a zero start."""
    import numpy as np
    import torch

    import dmwf_inputs as inp
    from paper_1702_08852_amd import BF16X3_GEMM, FP32_GEMM, FP64, Plan

    prec = {"fp64": FP64, "fp32": FP32_GEMM, "bf16x3": BF16X3_GEMM}[precision]
    if maps == 1:
        probs = [inp.make_problem("cfg3", nside=nside)]
    else:
        probs = [inp.make_problem("cfg4", nside=nside, index=k) for k in range(maps)]
    lmax = probs[0].lmax
    plan = Plan(nside, lmax, nmaps=maps, device=dev, precision=prec)
    if maps > 1:
        plan.autotune()
    st = lambda xs: torch.tensor(np.stack(xs) if maps > 1 else xs[0], device=dev).contiguous()
    sig = plan.alm2map(st([q.alm_true for q in probs]))
    d = (sig + st([q.sigma * q.white for q in probs])).masked_fill(st([q.mask for q in probs]), 0.0)
    w, cl = st([q.ninv for q in probs]), st([q.cl for q in probs])
    a0 = torch.zeros_like(plan._alm())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, sts = plan.solve(cl, d.contiguous(), w, eps_final=1e-6, start_final=True, alm=a0,
                           replay=[iters])
    torch.cuda.synchronize()
    print(json.dumps({"probe": {"nside": nside, "lmax": lmax, "maps": maps,
                                "precision": precision, "iterations": iters,
                                "seconds": time.perf_counter() - t0}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nside", type=int, default=1024)
    ap.add_argument("--pairs", type=int, default=100,
                    help="full-band iterations timed separately (replayed at xi = alpha)")
    ap.add_argument("--cpu-fraction", type=float, default=1.0,
                    help="fraction of rings (synthesis) and of m (adjoint) the oracle evaluates")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched measurements (96-map workload, four-map pair rate)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip configurations 1 and 2 (Nside 16 and 256)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip configuration 3's reduced-precision forms")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm start's evaluation")
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the batched workload and print its record")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--probe-iterations", type=int, default=0,
                    help="only run this many full-band iterations (xi = alpha) of the plan "
                         "shape given by --nside, --maps and --precision, for profiler runs")
    ap.add_argument("--maps", type=int, default=1, help="maps of the --probe-iterations plan")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32", "bf16x3"),
                    help="Legendre contraction of the --probe-iterations plan")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this library "
              "has no multi-GPU path (no collectives, no sharding).", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(dev)
        return
    if args.probe_iterations > 0:
        probe(dev, args.nside, args.maps, args.precision, args.probe_iterations)
        return
    if args.batch_only:
        print(json.dumps({"batched": bench_batch(dev, 20)}))
        return
    nside = args.nside
    p, plan, cl, d, w, np = make_inputs(nside, dev)
    lmax = p.lmax
    eps_final, eps_coarse = 1e-6, 1e-4

    def solve():
        return plan.solve(cl, d, w, eps_final=eps_final, eps_coarse=eps_coarse)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    # one solve without any kernel timing (iterations replayed whole from the
    # solve loop's graph), beside the timed steps below
    t0 = time.perf_counter()
    solve()
    torch.cuda.synchronize()
    graph_solve_s = time.perf_counter() - t0

    # timed steps: the dominant kernel (the Legendre analysis) between HIP
    # events on its launch stream, the rest of every iteration replayed from
    # the solve loop's graph
    plan.profile(2)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        alm, smap, st = solve()
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_read()
    plan.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    st = stats[-1]

    # algorithmic flops of the Legendre launches over the timed region
    leg_flops = 0.0
    for s in stats:
        for it, ell in zip(s.iters_per_level, s.lmax_per_level):
            leg_flops += it * legendre_flops(nside, ell)
    cand = {k: v for k, v in prof.items() if v[0] > 0}
    dom = max(cand, key=lambda k: cand[k][1])
    cnt, tot_ms = prof[dom]
    if dom in ("legendre_analysis", "legendre_synthesis"):
        achieved = leg_flops / (tot_ms * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved,
                "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VALU_PEAK_TFLOPS, "traffic": measured_traffic(dom),
                "launches": cnt, "avg_launch_ms": tot_ms / cnt,
                "priced_on": "the full T(l_iter) of every launch (8 flops per triple)"}
        # the same time priced on the work the kernel does: the triples after
        # each ring's recurrence start (polar terms below 2^-100 skipped), and
        # the lane-steps it issues (wave-wide starts, whole blocks)
        key = "analysis_issued" if dom == "legendre_analysis" else "synthesis_issued"
        work = {ell: plan.legendre_work(ell) for s in stats for ell in set(s.lmax_per_level)}
        started = issued = 0
        for s in stats:
            for it, ell in zip(s.iters_per_level, s.lmax_per_level):
                started += it * work[ell]["started"]
                issued += it * work[ell][key]
        roof["frac_started_work"] = 8.0 * started / (tot_ms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS
        roof["frac_issued_work"] = 8.0 * issued / (tot_ms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS
    else:
        npix = 12 * nside * nside
        achieved = 32.0 * npix * cnt / (tot_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "launches": cnt, "avg_launch_ms": tot_ms / cnt}

    # Full-band transform pair (l_iter = lmax): iterations at xi = alpha as the
    # solve loop runs them, from the converged state, replayed for a fixed
    # count.  Two replay lengths, the difference divided by the extra
    # iterations: the warm-start set-up of each call cancels.
    alpha = st.alpha

    def replay_run(n, prof):
        a0 = alm.clone()
        torch.cuda.synchronize()
        plan.profile(prof)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.solve(cl, d, w, eps_final=eps_final, start_final=True, alm=a0, replay=[n])
        e1.record()
        torch.cuda.synchronize()
        prof_ = plan.profile_read() if prof else None
        plan.profile(False)
        return e0.elapsed_time(e1), prof_

    # timed as the solve loop runs (graph replays); the per-kernel split from
    # the same replays with kernel timing on (launch by launch)
    n_short, n_long = 10, 10 + args.pairs
    ms_short, _ = replay_run(n_short, False)
    ms_long, _ = replay_run(n_long, False)
    _, prof_short = replay_run(n_short, True)
    _, prof_long = replay_run(n_long, True)
    pair_ms = (ms_long - ms_short) / args.pairs
    pprof = {k: (prof_long[k][0] - prof_short[k][0], prof_long[k][1] - prof_short[k][1])
             for k in prof_long}
    # the same iteration through the single-call entry point dmwf_dm_iterate,
    # which also recomputes l_iter and the m bounds on every call
    a_t = alm.clone()
    s_t = torch.zeros(12 * nside * nside, dtype=torch.float64, device=dev)
    c2 = torch.zeros(2, dtype=torch.float64, device=dev)
    plan.dm_iterate(alpha, alpha, cl, d, w, a_t, s_t, c2, first=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        plan.dm_iterate(alpha, alpha, cl, d, w, a_t, s_t, c2, first=False)
    e1.record()
    torch.cuda.synchronize()
    dm_iterate_ms = e0.elapsed_time(e1) / 10
    f_full = legendre_flops(nside, lmax)
    wfull = plan.legendre_work(lmax)
    leg = {}
    for k, key in (("legendre_analysis", "analysis_issued"),
                   ("legendre_synthesis", "synthesis_issued")):
        c_, t_ = pprof[k]
        if c_:
            sec = t_ / c_ * 1e-3
            leg[k] = {"avg_launch_ms": t_ / c_,
                      "achieved_tflops": f_full / sec / 1e12,
                      "frac": f_full / sec / 1e12 / FP64_VALU_PEAK_TFLOPS,
                      "frac_started_work": 8.0 * wfull["started"] / sec / 1e12 / FP64_VALU_PEAK_TFLOPS,
                      "frac_issued_work": 8.0 * wfull[key] / sec / 1e12 / FP64_VALU_PEAK_TFLOPS}
    pair_frac = 2 * f_full / (pair_ms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS

    resid = plan.wf_residual(cl, d, w, alm)
    iters = st.n_iter

    batched4 = None
    if not args.no_batch:
        # the same full-band iteration for four copies of this map in one plan
        # (one launch per stage for all four, autotuned tiles)
        from paper_1702_08852_amd import Plan
        nb = 4
        bplan = Plan(nside, lmax, nmaps=nb, device=dev)
        btile, _ = bplan.autotune()
        bcl, bd, bw = (x.unsqueeze(0).repeat(nb, *([1] * x.dim())).contiguous() for x in (cl, d, w))
        balm = alm.unsqueeze(0).repeat(nb, 1, 1).contiguous()

        def breplay(n):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            bplan.solve(bcl, bd, bw, eps_final=eps_final, start_final=True, alm=balm.clone(),
                        replay=[n])
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1)

        breplay(5)
        b_it_ms = (breplay(5 + 20) - breplay(5)) / 20
        batched4 = {"ms_per_iteration": b_it_ms, "ms_per_map_pair": b_it_ms / nb,
                    "gain_per_map": pair_ms / (b_it_ms / nb), "tiles": list(btile)}
        del bplan, bcl, bd, bw, balm
        torch.cuda.empty_cache()
    out = {
        "metric": METRIC,
        "value": 1e3 / ms_per_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"configuration 3: plain FP64 dual messenger, HEALPix Nside {nside} "
                         f"({12 * nside * nside} px), lmax {lmax}, damped C_l, sigma0 45 uK "
                         f"ecliptic hits, {100 * p.meta['masked_fraction']:.2f}% masked, "
                         f"beta 0.75, eps_coarse {eps_coarse:g}, eps_final {eps_final:g}"),
            "nside": nside, "lmax": lmax, "maps": 1,
        },
        "roofline": roof,
        "sht_pair": {"pairs_per_s": 1e3 / pair_ms, "ms_per_pair": pair_ms,
                     "lmax": lmax, "frac_of_fp64_peak": pair_frac, "legendre": leg,
                     "kernel_ms_per_pair": {k: v[1] / args.pairs
                                            for k, v in pprof.items() if v[0]},
                     "measured_as": (f"solve-loop iterations at xi = alpha replayed from the "
                                     f"converged state: ({n_long} - {n_short}) iterations, "
                                     f"graph replays; kernel split from the same replays "
                                     f"launched one by one with kernel timing"),
                     "dm_iterate_call_ms": dm_iterate_ms,
                     "batched_4_maps": batched4},
        "solve": {"untimed_solve_s": graph_solve_s,
                  "timed_steps_launch": ("Legendre analysis launched between HIP events, the rest "
                                         "of every iteration replayed from the solve loop's graph"),
                  "iterations": iters, "levels": st.n_levels, "alpha": st.alpha,
                  "final_cauchy": st.final_cauchy, "wf_residual": resid,
                  "gate": ("Cauchy ratio ||s_i - s_{i-1}|| / ||s_i|| < eps_final at xi = alpha "
                           "(Algorithm 2's stopping rule); the FP64 residual ||Ax - y|| / ||y|| "
                           "is reported beside it, not used to stop"),
                  "residual_target": eps_final, "residual_target_met": bool(resid <= eps_final),
                  "iters_per_level": st.iters_per_level, "lmax_per_level": st.lmax_per_level,
                  "kernel_ms_per_solve": {k: v[1] / args.steps for k, v in prof.items() if v[0]}},
    }
    del plan
    torch.cuda.empty_cache()
    if not args.no_precision:
        out["precision_forms"] = precision_legs(nside, lmax, cl, d, w, alm, smap, 20, eps_final,
                                                eps_coarse)
    if not args.no_configs:
        out["configs"] = bench_configs(dev, not args.no_cpu)
    if not args.no_batch:
        out["batched"] = bench_batch(dev, 20)
    if not args.no_learned:
        out["learned_warm_start"] = learned_warm_start(dev)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(nside, lmax, iters, args.cpu_fraction)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
