#!/usr/bin/env python3
"""Benchmark of the fold likelihood hot path on one MI355X.

Headline workload (value): the large uneven batch of 16384 pseudo-experiments, a seeded mix of
  A  energy-family models: 3-5 species on 500 true cells, Gaussian response, 100-200 bins;
  B  Borexino-like models: 6-16 species on 1000-4000 true cells, gamma response with light
     yield, Birks quenching and resolution (a, b, c), 200-900 bins;
  C  the pulse-shape model: 12 species, 900 energy x 50 pulse-shape bins x 1-3 datasets.
One step is one batched -ln L + gradient evaluation of every toy (cells, fold, Poisson
reduction, adjoint, gradient), inputs resident in device memory; value = toys x steps / wall
time, after the batch scheduler's autotuner has picked the work layout.

Also reported: the dominant kernel of that step against the FP64 vector roofline (timed live
with HIP events on its stream; algorithmic flops from the banded-mesh pair counts), toy fits per
second of the mix, each class as a batch of its own, the 4096-toy Borexino-scale toy study
(evaluations, kernels, fits, fits one at a time by the host driver), the single 1-D fit, the
single Borexino-scale fit and the pulse-shape model with adjoint versus central finite-difference
gradients, and the CPU oracle on the host cores (a bounded per-class sample of the mix).
"""
import argparse
import json
import os
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NLL+grad evals/sec and toy fits/sec at |dNLL|/NLL<=1e-11 (adjoint vs finite-diff)"
FP64_PEAK_TFLOPS = 78.6
# Algorithmic FP64 work per banded-mesh pair (a window bin inside a cell's support), for one
# direction: 26.5 operations, half of the 53 per pair for the forward fold plus the adjoint
# with an exponential counted at ~20 (the cost model of the analytic fit, Eq.2, priced per
# pair).  The per-species kernels of the pulse-shape toys add one multiply-add (2 operations)
# per species the pair's cell carries: the weighting in the fold, the seed contraction in the
# adjoint.
ALGO_FLOPS_PER_PAIR = 26.5
# The same, counted from the kernels' own gfx950 instruction mix with an FMA as 2 (fold: tile-
# relative exponent 2 FMA, table-driven exponential 5 FMA + SUB + MUL + LDEXP, accumulation
# 1 FMA; adjoint: 3 accumulating FMAs; the clamped tiles add a MAX): context only.
INSTR_FLOPS_PER_PAIR = {"fold": 19, "adj": 23}
KERNEL_NAMES = {"fold": "k_fold1", "adj": "k_adj<1>", "folds": "k_fold_s", "adj_s": "k_adj_s"}


def kernel_names(adj_waves):
    """The pair kernels' names; the 1-D adjoint is the template the batch's layout runs."""
    return dict(KERNEL_NAMES, adj=f"k_adj<{adj_waves}>")
# HBM bytes per launch of the pair kernels on the 16384-toy mixed batch (the headline step; both
# 1-D adjoint layouts the autotuner chooses between), from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE;
# KiB per dispatch) scaled by what the same counters read for a plain 512 MiB device copy
# (FETCH_SIZE x 2.00, WRITE_SIZE x 1.00).  They hold only for the kernel sources named by the
# sha (taken on sources that build to the same library byte for byte): any change to those
# sources reports traffic as null.
TRAFFIC = {"sources_sha256": "cc0e859ce3cb040b256f17f9714b75003478ff57a68098b013f524e53f93fa6d",
           "workload": "mix16384", "kernels": {"k_fold1": 1342681031, "k_adj<1>": 2430168712,
                                                "k_adj<4>": 2360077300, "k_fold_s": 598661994,
                                                "k_adj_s": 799931802}}


def strip_c_comments(text):
    """C/C++ source without its // and /* */ comments (string and character literals kept),
    with every run of whitespace outside literals reduced to one newline (if it held one) or
    one space, so that edits to comments alone leave it unchanged."""
    out, i, n = [], 0, len(text)
    ws = ""  # pending whitespace outside literals

    def flush():
        nonlocal ws
        if ws:
            out.append("\n" if "\n" in ws else " ")
            ws = ""

    while i < n:
        c = text[i]
        if c in "\"'":
            flush()
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            ws += " "
        elif c.isspace():
            ws += c
            i += 1
        else:
            flush()
            out.append(c)
            i += 1
    return "".join(out).strip()


def sources_sha256():
    """sha256 of the kernel sources (paper_1812_05686_amd/csrc: .hip, .h, .cpp) with comments
    removed: the key under which HBM traffic measured for a build is reused."""
    import hashlib
    d = os.path.join(ROOT, "paper_1812_05686_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(d, name), encoding="utf-8") as f:
                h.update(strip_c_comments(f.read()).encode())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """Host CPU as the oracle baseline ran on: logical CPUs, the ones this process may use,
    and the model / sockets lscpu reports."""
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core"):
                info[k.strip()] = v.strip()
    except Exception as e:  # lscpu missing: keep the counts
        info["lscpu"] = repr(e)
    return info


def kernel_rooflines(kt, counts, adj_waves=1):
    """Achieved TFLOP/s and fraction of the FP64 vector peak of the pair kernels, from their
    average launch time (HIP events) and the algorithmic work of one launch: banded pairs x
    26.5 (+ 2 per species of the pair's cell for the per-species kernels)."""
    fold_p, adj_p, full, band, band2, band2s = counts
    band1 = band - band2
    work = {"fold": (band1, band1 * ALGO_FLOPS_PER_PAIR), "adj": (band1, band1 * ALGO_FLOPS_PER_PAIR),
            "folds": (band2, band2 * ALGO_FLOPS_PER_PAIR + 2.0 * band2s),
            "adj_s": (band2, band2 * ALGO_FLOPS_PER_PAIR + 2.0 * band2s)}
    out = {}
    for k, (pairs, flops) in work.items():
        ms, n = kt.get(k, (0.0, 0))
        if not n or pairs <= 0:
            continue
        avg = ms / n
        tf = flops / (avg * 1e-3) / 1e12
        out[k] = {"kernel": kernel_names(adj_waves)[k], "avg_launch_ms": round(avg, 4), "pairs_per_launch": pairs,
                  "flops_per_launch": flops, "achieved_tflops": round(tf, 3),
                  "frac": round(tf / FP64_PEAK_TFLOPS, 4)}
    return out


def timed_steps(batch, theta, nll, grad, st, steps, warmup, torch):
    for _ in range(warmup):
        batch.nll_grad(theta, nll, grad, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.nll_grad(theta, nll, grad, st)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def profiled_kernels(batch, theta, nll, grad, st, reps, torch):
    batch.set_profiling(True)
    batch.kernel_times(reset=True)
    for _ in range(reps):
        batch.nll_grad(theta, nll, grad, st)
    kt = batch.kernel_times(reset=True)
    batch.set_profiling(False)
    torch.cuda.synchronize()
    return kt


def buffers(n, stride, torch):
    return (torch.empty(n, dtype=torch.float64, device="cuda"),
            torch.empty(n, stride, dtype=torch.float64, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda"))


def theta_of(toys, stride, which="theta_true"):
    th = np.zeros((len(toys), stride))
    for t, m in enumerate(toys):
        th[t, : m.n_params] = getattr(m, which)
    return th


def cpu_baseline_mix(toys, classes, gpu_nll, gpu_grad, seconds, threads):
    """The oracle's -ln L + gradient on the host, one toy per thread, per class of the mix for a
    bounded time each; the mix's rate is its toy count over the time the measured per-class
    rates need for one evaluation of every toy.  The evaluated toys double as a parity sample
    against the GPU values at the same points."""
    import oracle
    oracle.build(force=False)
    per_class, parity = {}, {"toys": 0, "max_rel_dnll": 0.0, "max_grad_err": 0.0}
    share = {"A": 0.15, "B": 0.35, "C": 0.5}
    for c in sorted(set(classes)):
        idx = [t for t in range(len(toys)) if classes[t] == c][:threads]
        orcs = [oracle.Oracle(toys[t]) for t in idx]
        counts = [0] * len(idx)
        first = [None] * len(idx)
        stop = time.perf_counter() + seconds * share.get(c, 0.3)

        def work(i):
            while True:
                r = orcs[i].nll_grad(toys[idx[i]].theta_true)
                if first[i] is None:
                    first[i] = r
                counts[i] += 1
                if time.perf_counter() >= stop:
                    break

        t0 = time.perf_counter()
        th = [threading.Thread(target=work, args=(i,)) for i in range(len(idx))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        el = time.perf_counter() - t0
        per_class[c] = {"evals_per_s": round(sum(counts) / el, 3), "evals": sum(counts), "seconds": round(el, 2),
                        "threads": len(idx)}
        for i, t in enumerate(idx):
            m = toys[t]
            ov, og, _ = first[i]
            parity["toys"] += 1
            parity["max_rel_dnll"] = max(parity["max_rel_dnll"], abs(gpu_nll[t] - ov) / abs(ov))
            parity["max_grad_err"] = max(parity["max_grad_err"], float(np.max(
                np.abs(gpu_grad[t, : m.n_params] - og) * m.fd_scale / np.maximum(np.abs(og) * m.fd_scale, 1.0))))
    n_of = {c: classes.count(c) for c in per_class}
    t_mix = sum(n_of[c] / per_class[c]["evals_per_s"] for c in per_class)
    parity["pass"] = bool(parity["max_rel_dnll"] <= 1e-11 and parity["max_grad_err"] <= 1e-8)
    return len(toys) / t_mix, per_class, parity


def one_thread_rate(toy, seconds):
    import oracle
    o = oracle.Oracle(toy)
    n, t0 = 0, time.perf_counter()
    while True:
        o.nll_grad(toy.theta_true)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    return n / (time.perf_counter() - t0), n


def mixed_batch(gs, gsgen, torch, args):
    """The headline: the 16384-toy uneven mix as one batch."""
    t0 = time.perf_counter()
    toys = gsgen.config4(args.mixed_toys)
    gen_s = time.perf_counter() - t0
    classes = [m.name.split("/")[1] for m in toys]
    batch = gs.Batch(toys)
    theta = torch.tensor(theta_of(toys, batch.stride), dtype=torch.float64, device="cuda")
    nll, grad, st = buffers(len(toys), batch.stride, torch)
    if args.mix_layout:
        batch.set_layout(*(int(x) for x in args.mix_layout.split(",")))
        tune = dict(batch.layout(), forced=True)
    else:
        tune = batch.autotune(theta, reps=2)
    log(f"bench: mix autotune {tune}")
    el = timed_steps(batch, theta, nll, grad, st, args.steps, args.warmup, torch)
    kt = profiled_kernels(batch, theta, nll, grad, st, max(2, args.steps // 4), torch)
    counts = batch.mesh_counts()
    roof = kernel_rooflines(kt, counts, batch.layout()["adj_waves"])
    out = {"toys": len(toys), "classes": {c: classes.count(c) for c in sorted(set(classes))},
           "evals_per_s": len(toys) * args.steps / el, "ms_per_step": el * 1e3 / args.steps,
           "generator_s": round(gen_s, 1), "status_nonzero": int((st != 0).sum().item()), "autotune": tune,
           "kernel_ms": {k: round(v[0] / v[1], 4) for k, v in kt.items() if v[1]}, "kernels": roof,
           "mesh": dict(zip(("fold_pairs", "adj_pairs", "full_mesh", "banded", "banded_2d", "banded_2d_species"),
                            counts)),
           "fixed_params_per_toy": round(float(np.mean([int((~m.free).sum()) if m.free is not None else 0
                                                        for m in toys])), 2)}
    gpu_nll, gpu_grad = nll.cpu().numpy(), grad.cpu().numpy()
    if not args.no_fits:
        th0 = torch.tensor(theta_of(toys, batch.stride, "theta0"), dtype=torch.float64, device="cuda")
        free, scales = batch.free_masks(toys), batch.scales(toys)
        batch.fit(th0, scales, free=free)  # warm: builds the captured graph
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = batch.fit(th0, scales, free=free)
        torch.cuda.synchronize()
        el = time.perf_counter() - ta
        stt = r["status"].cpu().numpy()
        out["fits"] = {"fits_per_s": round(len(toys) / el, 1), "seconds": round(el, 3),
                       "converged": int(np.sum(stt & 32 != 0)),
                       "per_class_converged": {c: int(sum(1 for t in range(len(toys)) if classes[t] == c and stt[t] & 32))
                                               for c in out["classes"]}}
    # each class of the mix as a batch of its own (same toys)
    per_class = {}
    for c in sorted(set(classes)):
        idx = [t for t in range(len(toys)) if classes[t] == c]
        sub = [toys[t] for t in idx]
        b_c = gs.Batch(sub)
        th_c = theta[idx, : b_c.stride].contiguous()
        n_c, g_c, s_c = buffers(len(sub), b_c.stride, torch)
        el_c = timed_steps(b_c, th_c, n_c, g_c, s_c, args.steps, args.warmup, torch)
        kt_c = profiled_kernels(b_c, th_c, n_c, g_c, s_c, 2, torch)
        per_class[c] = {"toys": len(sub), "evals_per_s": round(len(sub) * args.steps / el_c, 1),
                        "ms_per_step": round(el_c * 1e3 / args.steps, 3),
                        "status_nonzero": int((s_c != 0).sum().item()),
                        "kernel_ms": {k: round(v[0] / v[1], 4) for k, v in kt_c.items() if v[1]},
                        "kernels": kernel_rooflines(kt_c, b_c.mesh_counts(), b_c.layout()["adj_waves"])}
        del b_c
    out["per_class"] = per_class
    return out, toys, classes, gpu_nll, gpu_grad


def toy_study(gs, gsgen, torch, args):
    """The 4096-toy Borexino-scale study: evaluations, kernels, fits."""
    base = gsgen.config1()
    toys = gsgen.config3(args.toys, base=base)
    batch = gs.Batch(toys)
    theta = torch.tensor(np.stack([t.theta_true for t in toys]), dtype=torch.float64, device="cuda")
    nll, grad, st = buffers(len(toys), batch.stride, torch)
    tune = batch.autotune(theta, reps=3)
    el = timed_steps(batch, theta, nll, grad, st, args.steps, args.warmup, torch)
    kt = profiled_kernels(batch, theta, nll, grad, st, args.steps, torch)
    counts = batch.mesh_counts()
    roof = kernel_rooflines(kt, counts, batch.layout()["adj_waves"])
    for k in ("fold", "adj"):
        if k in roof:
            roof[k]["instr_flops_per_pair"] = INSTR_FLOPS_PER_PAIR[k]
            roof[k]["executed_over_banded"] = round(counts[0 if k == "fold" else 1] / counts[3], 4)
    traffic = None  # the stored counters are of the mixed batch, not of this study
    fixed = [int((~t.free).sum()) for t in toys]
    out = {"toys": len(toys), "evals_per_s": round(len(toys) * args.steps / el, 1),
           "ms_per_step": round(el * 1e3 / args.steps, 4), "autotune": tune,
           "mean_window_bins": round(float(np.mean([t.win_hi - t.win_lo for t in toys])), 1),
           "fixed_params_per_toy": round(float(np.mean(fixed)), 2), "params_per_toy": int(toys[0].n_params),
           "full_mesh_pairs": counts[2], "banded_pairs": counts[3], "kernels": roof, "hbm_bytes_per_launch": traffic,
           "status_nonzero": int((st != 0).sum().item())}
    if args.no_fits:
        return out
    th0 = torch.tensor(np.stack([t.theta0 for t in toys]), dtype=torch.float64, device="cuda")
    free = batch.free_masks(toys)
    batch.fit(th0, base.fd_scale, free=free)  # warm: builds the captured graph
    torch.cuda.synchronize()
    ta = time.perf_counter()
    r = batch.fit(th0, base.fd_scale, free=free)
    torch.cuda.synchronize()
    el = time.perf_counter() - ta
    stt, it = r["status"].cpu().numpy(), r["iters"].cpu().numpy()
    act, tms = batch.fit_trace()
    out["fits"] = {"fits_per_s": round(len(toys) / el, 2), "seconds": round(el, 4),
                   "converged": int(np.sum(stt & 32 != 0)), "mean_iters": round(float(it.mean()), 2),
                   "max_iters": int(it.max()), "graph_launches": int(len(act)),
                   "ms_until_90pct_done": round(float(tms[np.argmax(act <= 0.1 * len(toys))]), 2) if len(act) else None}
    # the same toys fitted one at a time by the host driver over single-model evaluations,
    # with central-difference gradients (the plain path) and with the adjoint
    n_one = 16
    models = [gs.Model(t) for t in toys[:n_one]]
    models[0].fit(toys[0].theta0, base.fd_scale, free=toys[0].free_mask(), hesse=False)  # warm
    bnll = r["nll"].cpu().numpy()
    one = {"toys": n_one}
    for name, fd in (("adjoint", False), ("finite_diff", True)):
        ta = time.perf_counter()
        res = [mdl.fit(t.theta0, base.fd_scale, use_fd=fd, free=t.free_mask(), hesse=False)
               for mdl, t in zip(models, toys[:n_one])]
        el = time.perf_counter() - ta
        one[name] = {"fits_per_s": round(n_one / el, 2), "seconds": round(el, 3),
                     "converged": int(sum(bool(q["ok"]) for q in res)),
                     "max_rel_dnll_vs_batched": float(max(abs(q["nll"] - bnll[i]) / abs(bnll[i])
                                                          for i, q in enumerate(res)))}
    out["fits_one_at_a_time_host"] = one
    return out


def single_model(gs, torch, m, reps=200, fits=True):
    """One model: device-resident evaluation latency (a batch of one), per-kernel times, and
    one fit with the adjoint versus central finite differences (host driver)."""
    b = gs.Batch([m])
    th = torch.tensor(theta_of([m], b.stride), dtype=torch.float64, device="cuda")
    n1, g1, s1 = buffers(1, b.stride, torch)
    el = timed_steps(b, th, n1, g1, s1, reps, 10, torch)
    kt = profiled_kernels(b, th, n1, g1, s1, 20, torch)
    out = {"us_per_eval": round(el * 1e6 / reps, 2), "evals_per_s": round(reps / el, 1),
           "kernel_us": {k: round(v[0] * 1e3 / v[1], 2) for k, v in kt.items() if v[1]},
           "kernels": kernel_rooflines(kt, b.mesh_counts(), b.layout()["adj_waves"])}
    if fits:  # the same fit on the device BFGS (graph of evaluation + step launches), as a batch of one
        th0 = torch.tensor(theta_of([m], b.stride, "theta0"), dtype=torch.float64, device="cuda")
        free, sc = b.free_masks([m]), b.scales([m])
        b.fit(th0, sc, free=free)  # warm: builds the captured graph
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = b.fit(th0, sc, free=free)
        torch.cuda.synchronize()
        el = time.perf_counter() - ta
        out["device_fit"] = dict(fits_per_s=round(1.0 / el, 3), seconds=round(el, 5), iters=int(r["iters"][0]),
                                 converged=bool(int(r["status"][0]) & 32), nll=float(r["nll"][0]))
    del b
    if fits:
        model = gs.Model(m)
        for name, fd in (("adjoint", False), ("finite_diff", True)):
            model.fit(m.theta0, m.fd_scale, use_fd=fd, hesse=False)  # warm
            ta = time.perf_counter()
            r = model.fit(m.theta0, m.fd_scale, use_fd=fd, hesse=False)
            el = time.perf_counter() - ta
            out[name] = dict(fits_per_s=round(1.0 / el, 3), seconds=round(el, 5), iters=r["iters"],
                             n_eval=r["n_eval"], converged=r["ok"], nll=r["nll"])
        out["speedup_adjoint_over_fd"] = round(out["finite_diff"]["seconds"] / out["adjoint"]["seconds"], 2)
        model.close()
    return out


def discovery_study(gs, gsgen, torch, n_toys):
    """The profile-likelihood discovery test (section 4.2, Eq.5) over null pseudo-experiments of
    the Gaussian-signal model: two batched fits per toy (signal free; signal fixed at 0)."""
    from scipy import stats
    toys = gsgen.discovery_toys(n_toys)
    batch = gs.Batch(toys)
    th0 = torch.tensor(theta_of(toys, batch.stride, "theta0"), dtype=torch.float64, device="cuda")
    sc, free = batch.scales(toys), batch.free_masks(toys)
    gs.discovery(batch, th0, sc, [0] * len(toys), free=free)  # warm: captures the fit graphs
    torch.cuda.synchronize()
    ta = time.perf_counter()
    r = gs.discovery(batch, th0, sc, [0] * len(toys), free=free)
    torch.cuda.synchronize()
    el = time.perf_counter() - ta
    t = r["t"].cpu().numpy()
    ok = np.isfinite(t)
    return {"toys": len(toys), "tests_per_s": round(len(toys) / el, 1), "seconds": round(el, 4),
            "fits_per_s": round(2 * len(toys) / el, 1), "both_converged": int(ok.sum()),
            "t_mean": round(float(t[ok].mean()), 4),
            "ks_pvalue_vs_chi2_1": float(stats.kstest(np.maximum(t[ok], 0.0), stats.chi2(1).cdf).pvalue)}


def template_study(gs, gsgen, torch, args):
    """The Monte Carlo template fit (section 3.2, Eq.1): toys of the pulse-shape model's
    templates flattened to 45,000 bins, 12 rates each; mu = templates x rates, no fold.  The
    kernel streams each toy's counts once: its roofline is HBM bandwidth."""
    base = gsgen.template_model(flat2d=True)
    toys = gsgen.template_toys(args.template_toys, base)
    batch = gs.Batch(toys)
    theta = torch.tensor(theta_of(toys, batch.stride), dtype=torch.float64, device="cuda")
    nll, grad, st = buffers(len(toys), batch.stride, torch)
    el = timed_steps(batch, theta, nll, grad, st, args.steps, args.warmup, torch)
    kt = profiled_kernels(batch, theta, nll, grad, st, args.steps, torch)
    ms, n = kt["tmpl"]
    avg = ms / n
    bins = sum(m.win_hi - m.win_lo for m in toys)
    S = base.n_species
    # algorithmic bytes per evaluation: each toy's counts (FP64) once, the shared templates once
    byts = 8.0 * bins + 8.0 * S * base.n_reco
    gbs = byts / (avg * 1e-3) / 1e9
    out = {"toys": len(toys), "bins_per_toy": base.n_reco, "species": S,
           "evals_per_s": round(len(toys) * args.steps / el, 1), "ms_per_step": round(el * 1e3 / args.steps, 4),
           "kernel": {"kernel": "k_tmpl", "avg_launch_ms": round(avg, 4), "bytes_per_launch": byts,
                      "achieved_gbs": round(gbs, 1), "peak_gbs": 8000.0, "frac": round(gbs / 8000.0, 4),
                      "bound": "hbm"},
           "kernel_ms": {k: round(v[0] / v[1], 4) for k, v in kt.items() if v[1]},
           "status_nonzero": int((st != 0).sum().item())}
    if not args.no_fits:
        th0 = torch.tensor(theta_of(toys, batch.stride, "theta0"), dtype=torch.float64, device="cuda")
        batch.fit(th0, base.fd_scale)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = batch.fit(th0, base.fd_scale)
        torch.cuda.synchronize()
        el = time.perf_counter() - ta
        out["fits"] = {"fits_per_s": round(len(toys) / el, 1), "seconds": round(el, 4),
                       "converged": int(np.sum(r["status"].cpu().numpy() & 32 != 0))}
    return out


FAMILY_CASES = (("gengamma_p1.6", "GENGAMMA_PE", 1.6, 0), ("scaled_poisson", "SPOIS_PE", 0.0, 0),
                 ("mod_gauss_f0.35", "EMG_PE", 0.35, 0), ("gamma_exact_bins", "GAMMA_PE", 0.0, 1),
                 ("gauss_exact_bins", "GAUSS_PE", 0.0, 1), ("gengamma_p1.6_exact_bins", "GENGAMMA_PE", 1.6, 1),
                 ("mod_gauss_f0.35_exact_bins", "EMG_PE", 0.35, 1))


def families_study(gs, gsgen, torch, args):
    """The further response families and exact bin contents (section 2.3, section 2.5) on the
    Borexino-scale model (4000 cells x 900 bins): the direct per-pair path's evaluation latency,
    its fold and adjoint kernels per banded pair, and one fit each way; then 256 toys of the
    generalized-gamma model in one batch."""
    out = {}
    for key, fam, shape, exact in FAMILY_CASES:
        m = gsgen.family_model(getattr(gsgen, fam), shape, exact_bins=exact)
        r = single_model(gs, torch, m, reps=50, fits=not args.no_fits)
        b = gs.Batch([m])
        band1 = b.mesh_counts()[3]
        del b
        for k in ("fold", "adj"):
            if k in r["kernel_us"]:
                r[f"{k}_ns_per_pair"] = round(r["kernel_us"][k] * 1e3 / max(band1, 1), 4)
        r["banded_pairs"] = band1
        r.pop("kernels", None)  # the FP64 pair count of the fast path does not apply here
        out[key] = r
        log(f"bench: family {key} {json.dumps(r)}")
    base = gsgen.family_model(gsgen.GENGAMMA_PE, 1.6)
    toys = gsgen.config3(256, base=base)
    batch = gs.Batch(toys)
    theta = torch.tensor(theta_of(toys, batch.stride), dtype=torch.float64, device="cuda")
    nll, grad, st = buffers(len(toys), batch.stride, torch)
    el = timed_steps(batch, theta, nll, grad, st, max(4, args.steps // 4), 2, torch)
    kt = profiled_kernels(batch, theta, nll, grad, st, 4, torch)
    band1 = batch.mesh_counts()[3]
    out["gengamma_256_toys"] = {"evals_per_s": round(len(toys) * max(4, args.steps // 4) / el, 1),
                                "kernel_ms": {k: round(v[0] / v[1], 4) for k, v in kt.items() if v[1]},
                                "banded_pairs": band1, "status_nonzero": int((st != 0).sum().item())}
    log(f"bench: family batch {json.dumps(out['gengamma_256_toys'])}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--toys", type=int, default=4096, help="pseudo-experiments of the Borexino-scale toy study")
    ap.add_argument("--mixed-toys", type=int, default=16384, help="toys of the uneven mix (the headline)")
    ap.add_argument("--template-toys", type=int, default=4096, help="toys of the Monte Carlo template study")
    ap.add_argument("--discovery-toys", type=int, default=4096, help="null toys of the discovery test")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fits", action="store_true")
    ap.add_argument("--no-study", action="store_true", help="skip the 4096-toy study and the single models")
    ap.add_argument("--mix-layout", type=str, default="", metavar="TW,GC,IT,AW",
                    help="put this work layout in force for the mix instead of autotuning it (one of its candidates: "
                         "split-K target, cells per gradient block, rounds per 2-D block, waves per 1-D adjoint item)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": args.copy_calibration, "ok": bool(dst[-1].item() == n - 1)}))
        return

    import gsgen
    import paper_1812_05686_amd as gs

    log(f"bench: {args.mixed_toys}-toy uneven mix (headline)")
    mix, toys, classes, gpu_nll, gpu_grad = mixed_batch(gs, gsgen, torch, args)
    log(f"bench: mix {json.dumps(mix)}")
    dom = max(mix["kernels"], key=lambda k: mix["kernels"][k]["avg_launch_ms"])
    dk = mix["kernels"][dom]
    traffic = None
    if TRAFFIC["sources_sha256"] == sources_sha256() and mix["toys"] == 16384:
        traffic = TRAFFIC["kernels"].get(dk["kernel"])
    roofline = {"bound": "alu", "kernel": dk["kernel"], "achieved": dk["achieved_tflops"], "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": dk["frac"], "traffic": traffic,
                "flops_per_launch": dk["flops_per_launch"], "pairs_per_launch": dk["pairs_per_launch"],
                "algo_flops_per_pair": ALGO_FLOPS_PER_PAIR, "avg_launch_ms": dk["avg_launch_ms"],
                "other_kernels": {v["kernel"]: {"frac": v["frac"], "avg_launch_ms": v["avg_launch_ms"]}
                                  for k, v in mix["kernels"].items() if k != dom}}

    study = singles = None
    if not args.no_study:
        log("bench: 4096-toy Borexino-scale study")
        study = toy_study(gs, gsgen, torch, args)
        log(f"bench: study {json.dumps(study)}")
        singles = {}
        for key, fn in (("c0_energy_family", gsgen.config0), ("c1_borexino_scale", gsgen.config1),
                        ("c2_pulse_shape", gsgen.config2),
                        ("c2_multivariate_10_slices", lambda: gsgen.multivariate_model(gsgen.config2(), 90)),
                        ("template_900_bins", gsgen.template_model)):
            singles[key] = single_model(gs, torch, fn(), fits=not args.no_fits)
            log(f"bench: {key} {json.dumps(singles[key])}")
        log("bench: Monte Carlo template study")
        templates = template_study(gs, gsgen, torch, args)
        log(f"bench: templates {json.dumps(templates)}")
        discovery = None
        if not args.no_fits:
            log("bench: discovery test")
            discovery = discovery_study(gs, gsgen, torch, args.discovery_toys)
            log(f"bench: discovery {json.dumps(discovery)}")
        singles["template_study"] = templates
        singles["discovery_test"] = discovery
        log("bench: response families and exact bins")
        singles["response_families"] = families_study(gs, gsgen, torch, args)

    cpu = parity = None
    if not args.no_cpu:
        aff = len(os.sched_getaffinity(0))
        threads = max(1, min(16, aff))  # a one-GPU machine's CPU share is 16
        rate, per_class, parity = cpu_baseline_mix(toys, classes, gpu_nll, gpu_grad, args.cpu_seconds, threads)
        b_toy = next(m for m, c in zip(toys, classes) if c == "B")
        r1, n1 = one_thread_rate(b_toy, max(2.0, args.cpu_seconds / 4))
        cpu = {"value": round(rate, 3), "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": (f"oracle -ln L+gradient of the mix's toys at their true parameters, one toy per thread, "
                          f"{threads} threads: per class " + ", ".join(
                              f"{c} {v['evals']} evaluations in {v['seconds']} s" for c, v in per_class.items()) +
                          "; the mix's rate = toys / sum over classes of (toys of the class / class rate)"),
               "per_class": per_class, "one_thread_class_B": {"value": round(r1, 3), "evals": n1},
               "host": host_info()}
        log(f"bench: cpu {cpu}; parity {parity}")

    fixed = mix["fixed_params_per_toy"]
    out = {"metric": METRIC, "value": round(mix["evals_per_s"], 1), "unit": "evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(mix["ms_per_step"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": (f"{mix['toys']} pseudo-experiments in one batch, a seeded uneven mix: "
                                   f"{mix['classes'].get('A', 0)} energy-family toys (3-5 species, 500 cells, 100-200 "
                                   f"bins), {mix['classes'].get('B', 0)} Borexino-like toys (6-16 species, 1000-4000 "
                                   f"cells, gamma response, 200-900 bins), {mix['classes'].get('C', 0)} pulse-shape "
                                   f"toys (12 species, 900 x 50 bins x 1-3 datasets); one batched -lnL+gradient of "
                                   f"every toy per step; parameters a toy's window cannot determine are fixed "
                                   f"({fixed} per toy on average)"),
                      "toys": mix["toys"], "classes": mix["classes"],
                      "toy_study_4096": None if study is None else {
                          "evals_per_s": study["evals_per_s"], "ms_per_step": study["ms_per_step"],
                          "fixed_params_per_toy": study["fixed_params_per_toy"],
                          "params_per_toy": study["params_per_toy"]}},
           "roofline": roofline, "cpu_baseline": cpu, "parity_sample": parity,
           "toy_fits": mix.get("fits"), "mixed_batch": mix, "toy_study": study, "single_models": singles}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
