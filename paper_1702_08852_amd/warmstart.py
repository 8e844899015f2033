"""Learned warm start: training data from the method's own solves, training
and evaluation of the network (argument marshalling and orchestration only;
every transform, solve, feature, forward and backward pass runs in the HIP
library through the C ABI).

    python -m paper_1702_08852_amd.warmstart train [--maps 2000] [--out FILE]
    python -m paper_1702_08852_amd.warmstart evaluate [--weights FILE]

Training maps: the warm-start recipe (configuration 2's shape: damped C_l,
30 uK / sqrt(hits) ecliptic noise, |b| < 15 deg plus 200 holes of 1 deg, own
holes and draws per map) at Nside 256, solved by the plain FP64 dual messenger
to eps_final 1e-5; each map gives `per_map` random modes (l >= 2) as
(features, whitened Wiener filter a_lm) pairs.  Evaluation: unseen maps of the
same recipe at Nside 512, solved to eps_final 1e-6 from a cold start and from
the network's estimate (entering at the last level, and at the first level
of the cooling schedule).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import dmwf

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "warmstart_weights.npy")


def _inputs():
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import dmwf_inputs
    return dmwf_inputs


def batch_problem(nside, indices, dev):
    """A plan over the listed warm-start maps and their (C_l, d, N^-1) on the
    device; the data map is the GPU synthesis of the drawn a_lm plus noise."""
    inp = _inputs()
    probs = [inp.make_problem("cfg5", nside=nside, index=k) for k in indices]
    lmax = probs[0].lmax
    nm = len(probs)
    plan = dmwf.Plan(nside, lmax, nmaps=nm, device=dev)
    st = lambda xs: torch.tensor(np.stack(xs), device=dev).contiguous()
    sig = plan.alm2map(st([q.alm_true for q in probs]).reshape(plan._alm().shape))
    noise = st([q.sigma * q.white for q in probs]).reshape(sig.shape)
    mask = st([q.mask for q in probs]).reshape(sig.shape)
    d = (sig + noise).masked_fill(mask, 0.0).contiguous()
    w = st([q.ninv for q in probs]).reshape(sig.shape)
    cl = st([q.cl for q in probs]).reshape((nm, lmax + 1) if nm > 1 else (lmax + 1,))
    return plan, lmax, cl, d, w


def valid_slots(lmax):
    """a_lm slots with l >= 2 (the modes the network predicts)."""
    out = []
    for m in range(lmax + 1):
        base = m * (2 * lmax + 1 - m) // 2
        out.extend(base + l for l in range(max(m, 2), lmax + 1))
    return np.array(out, dtype=np.int32)


def generate(nside, first, count, per_map, eps, dev, batch=100, seed=0, log=None):
    """Training pairs from `count` solves: features X [N][24], targets T [N][2]
    (device FP32), plus the iteration counts of the solves."""
    slots_all = torch.tensor(valid_slots(2 * nside), device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    xs, ts, iters = [], [], []
    for b0 in range(first, first + count, batch):
        idx = list(range(b0, min(b0 + batch, first + count)))
        plan, lmax, cl, d, w = batch_problem(nside, idx, dev)
        alm, _, sts = plan.solve(cl, d, w, eps_final=eps, eps_coarse=1e-4)
        sts = sts if isinstance(sts, list) else [sts]
        iters += [s.n_iter for s in sts]
        dlm = plan.adjoint(d, scale_by_pixel_area=True)
        nm = len(idx)
        for k in range(nm):
            sel = slots_all[torch.randint(0, slots_all.numel(), (per_map,), generator=gen,
                                          device=dev)].contiguous()
            wk = w[k] if nm > 1 else w
            nw, fsky = dmwf.noise_stats(wk.contiguous())
            x, t = dmwf.nn_features(lmax, (dlm[k] if nm > 1 else dlm).contiguous(),
                                    (cl[k] if nm > 1 else cl).contiguous(), nw, fsky, slots=sel,
                                    target=(alm[k] if nm > 1 else alm).contiguous())
            xs.append(x)
            ts.append(t)
        if log:
            log(f"generated maps {idx[0]}..{idx[-1]}: mean {np.mean(iters[-nm:]):.0f} iterations")
        del plan, alm, dlm, d, w, cl
        torch.cuda.empty_cache()
    return torch.cat(xs), torch.cat(ts), iters


def train(X, T, dev, steps=3000, batch=8192, lr=1e-3, seed=1, log=None, holdout=0.05):
    """Adam on minibatches of the pairs (the network's own kernels); a held-out
    share of the pairs measures generalisation.  Returns the network and a
    record of the losses."""
    inp = _inputs()
    n = X.shape[0]
    nh = int(n * holdout)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    perm = torch.randperm(n, generator=gen, device=dev)
    hold, fit = perm[:nh], perm[nh:]
    net = dmwf.Net(max_batch=max(batch, 65536), device=dev)
    net.set_params(torch.tensor(inp.nn_init_params(seed), device=dev))
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    hist = []

    def held_loss():
        tot, cnt = 0.0, 0
        for i0 in range(0, nh, 65536):
            sel = hold[i0:i0 + 65536]
            _, lv = net.gradient(X[sel].contiguous(), T[sel].contiguous())
            tot += float(lv.cpu()[0]) * sel.numel()
            cnt += sel.numel()
        return tot / max(cnt, 1)

    # the variance of the targets: the loss of predicting zero
    base = float((T[hold] ** 2).sum(dim=1).mean().cpu()) if nh else float((T ** 2).sum(1).mean())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        sel = fit[torch.randint(0, fit.numel(), (batch,), generator=gen, device=dev)]
        # cosine decay of the step size
        lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps))
        net.train_step(X[sel].contiguous(), T[sel].contiguous(), max(lr_t, 1e-6), loss)
        if step % 500 == 0 or step == steps - 1:
            rec = {"step": step, "train_loss": float(loss.cpu()[0]), "held_out_loss": held_loss()}
            hist.append(rec)
            if log:
                log(f"step {step}: {rec}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return net, {"pairs": n, "held_out_pairs": nh, "steps": steps, "batch": batch, "lr": lr,
                 "seconds": secs, "zero_predictor_loss": base, "history": hist,
                 "held_out_relative_error": math.sqrt(hist[-1]["held_out_loss"] / base)}


def evaluate(net, dev, nside=None, first=None, count=None, eps=1e-6, log=None, max_iter=60000):
    """Cold start against the network's warm start on unseen maps: iterations
    and wall time of the solves (one plan for all the maps; per map, the
    iterations each map needed), the distance of the estimate to the solution,
    and the FP64 residuals the solves reach.  Warm-started solves are capped at
    twice the cold start's largest iteration count."""
    inp = _inputs()
    nside = inp.WARM_EVAL_NSIDE if nside is None else nside
    first = inp.WARM_EVAL_FIRST if first is None else first
    count = inp.WARM_EVAL_MAPS if count is None else count
    plan, lmax, cl, d, w = batch_problem(nside, list(range(first, first + count)), dev)
    plan.autotune()

    def timed(name, cap=max_iter, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.solve(cl, d, w, eps_final=eps, eps_coarse=1e-4, max_iter=cap, **kw)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        if log:
            log(f"{name}: {secs:.2f} s, iterations {[s.n_iter for s in r[2]]}")
        return secs, r

    plan.solve(cl, d, w, eps_final=eps, max_iter=10)  # warm-up
    cold_s, (a_cold, _, st_cold) = timed("cold")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dlm = plan.adjoint(d, scale_by_pixel_area=True)
    a0 = torch.empty_like(a_cold)
    for k in range(count):
        nw, fsky = dmwf.noise_stats(w[k].contiguous())
        a0[k] = net.warm_start(lmax, dlm[k].contiguous(), cl[k].contiguous(), nw, fsky)
    torch.cuda.synchronize()
    infer_s = time.perf_counter() - t0
    if log:
        log(f"inference: {infer_s:.3f} s for {count} maps")
    est_err = [float((torch.linalg.vector_norm(a0[k] - a_cold[k]) /
                      torch.linalg.vector_norm(a_cold[k])).cpu()) for k in range(count)]
    out = {"nside": nside, "lmax": lmax, "maps": count, "eps_final": eps,
           "inference_seconds": infer_s,
           "estimate_rel_l2_to_solution_mean": float(np.mean(est_err)),
           "cold": {"seconds": cold_s, "iterations_mean": float(np.mean([s.n_iter for s in st_cold])),
                    "iterations_max": int(max(s.n_iter for s in st_cold)),
                    "wf_residual_max": float(max(plan.wf_residual(cl, d, w, a_cold)))}}
    for name, kw in (("warm_last_level", {"start_final": True}),
                     ("warm_first_level", {"warm_start": True})):
        # a warm start that needs more than twice the cold start's iterations
        # is stopped there and reported as not converged
        secs, (a_w, _, st_w) = timed(name, cap=2 * out["cold"]["iterations_max"], alm=a0.clone(),
                                     **kw)
        out[name] = {"seconds": secs + infer_s,
                     "iterations_mean": float(np.mean([s.n_iter for s in st_w])),
                     "iterations_max": int(max(s.n_iter for s in st_w)),
                     "converged": all(s.status == 0 for s in st_w),
                     "wf_residual_max": float(max(plan.wf_residual(cl, d, w, a_w))),
                     "rel_l2_to_cold_solution_max": max(
                         float((torch.linalg.vector_norm(a_w[k] - a_cold[k]) /
                                torch.linalg.vector_norm(a_cold[k])).cpu()) for k in range(count)),
                     "iterations_saved_mean": out["cold"]["iterations_mean"] -
                     float(np.mean([s.n_iter for s in st_w])),
                     "speedup": cold_s / (secs + infer_s)}
        if log:
            log(f"{name}: {out[name]}")
    return out


def load_net(path, dev):
    p = np.load(path, allow_pickle=False)
    net = dmwf.Net(max_batch=65536, device=dev)
    net.set_params(torch.tensor(p.astype(np.float32), device=dev))
    return net


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1702_08852_amd.warmstart")
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--maps", type=int, default=None)
    tr.add_argument("--per-map", type=int, default=2048)
    tr.add_argument("--steps", type=int, default=3000)
    tr.add_argument("--eps", type=float, default=1e-5)
    tr.add_argument("--out", default=DEFAULT_WEIGHTS)
    tr.add_argument("--record", default=None, help="JSON file for the training record")
    tr.add_argument("--evaluate", action="store_true")
    ev = sub.add_parser("evaluate")
    ev.add_argument("--weights", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    inp = _inputs()
    dev = torch.device("cuda:0")
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    if args.cmd == "train":
        maps = inp.WARM_TRAIN_MAPS if args.maps is None else args.maps
        t0 = time.perf_counter()
        X, T, iters = generate(inp.WARM_TRAIN_NSIDE, 0, maps, args.per_map, args.eps, dev, log=log)
        gen_s = time.perf_counter() - t0
        net, rec = train(X, T, dev, steps=args.steps, log=log)
        rec.update({"maps": maps, "nside": inp.WARM_TRAIN_NSIDE, "eps_final": args.eps,
                    "generation_seconds": gen_s, "solve_iterations_mean": float(np.mean(iters))})
        np.save(args.out, net.params().cpu().numpy())
        if args.evaluate:
            rec["evaluation"] = evaluate(net, dev, log=log)
        if args.record:
            with open(args.record, "w") as f:
                json.dump(rec, f, indent=1)
        print(json.dumps(rec))
    else:
        print(json.dumps(evaluate(load_net(args.weights, dev), dev, log=log)))


if __name__ == "__main__":
    main()
