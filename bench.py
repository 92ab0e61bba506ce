#!/usr/bin/env python3
"""Benchmark of the fold likelihood hot path on one MI355X.

Workload: 4096 pseudo-experiments of the Borexino-scale model (12 species: 4 lines, 6
betas, 2 exponentials; 4000 true cells of 0.75 keV plus 4 lines; 900 reco bins of 1.6 pe;
gamma response with light yield, Birks quenching and resolution a, b, c; 17 parameters,
3 pulls), each with its own Poisson data, rates drawn +-20% around nominal and its own fit
window of 200-900 bins.  One step is one batched -ln L + gradient evaluation of all toys
(cells, fold, Poisson reduction, adjoint, gradient) with every input already resident in
device memory; value = toys * steps / wall time.

Also reported: toy fits per second (device BFGS over the same toys in captured graphs),
the dominant kernel against the FP64 vector roofline (timed live with HIP events on its
stream), single-evaluation latency, one Borexino-scale fit with the adjoint gradient
versus central finite differences, and the CPU oracle on the host cores (sampled).
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NLL+grad evals/sec and toy fits/sec at |dNLL|/NLL<=1e-11 (adjoint vs finite-diff)"
FP64_PEAK_TFLOPS = 78.6
# FP64 operations per evaluated (bin, cell) pair of the gamma-response kernels, counted from
# their gfx950 instruction mix with an FMA as 2: the block-relative exponent (2 FMA), the
# exponential (MAX, 11 FMA, ADD, LDEXP) and the accumulation (1 FMA in the fold, 3 in the
# adjoint): 31 and 35.  The double-double reference exponent formed once per cell and bin
# block (tile) is set-up work and is not counted.
FLOPS_PER_PAIR = {"fold": 31, "adj": 35}
# HBM bytes per launch on the default workload (4096 toys), from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) scaled by what the same counters read for a
# plain 512 MiB device copy (FETCH_SIZE x 2.00, WRITE_SIZE x 1.00).  They hold only for the
# kernel sources they were taken on: any change to those sources reports traffic as null.
# Source: profiles/hbm_bytes_k_fold1_k_adj_borexino_4096toys.md.
TRAFFIC = {"sources_sha256": "a29e2632daf14d6c3656bd1017f632e34e1cea0ca6fdc33810aee63fbbb61525",
           "toys": 4096, "kernels": {"k_fold1": 1071554480, "k_adj": 1756266072}}


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


def cpu_baseline(toys, seconds, threads):
    """Oracle -ln L + gradient on the host, one toy per thread, for about `seconds`."""
    import oracle
    oracle.build(force=False)
    orcs = [oracle.Oracle(t) for t in toys[:threads]]
    counts = [0] * threads
    out = [None] * threads
    stop = time.perf_counter() + seconds

    def work(i):
        while True:
            out[i] = orcs[i].nll_grad(toys[i].theta_true)
            counts[i] += 1
            if time.perf_counter() >= stop:
                break

    t0 = time.perf_counter()
    th = [threading.Thread(target=work, args=(i,)) for i in range(threads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    el = time.perf_counter() - t0
    return sum(counts) / el, sum(counts), el, out


def mixed_batch(gs, gsgen, torch, n_toys, steps, warmup, with_oracle):
    """The large uneven batch: energy-family, Borexino-like and pulse-shape toys together.
    Batched -ln L + gradient evaluations per second, toy fits per second, and the oracle's
    error on two toys of every class."""
    t0 = time.perf_counter()
    toys = gsgen.config4(n_toys)
    gen_s = time.perf_counter() - t0
    batch = gs.Batch(toys)
    th = np.zeros((len(toys), batch.stride))
    for t, m in enumerate(toys):
        th[t, : m.n_params] = m.theta_true
    theta = torch.tensor(th, dtype=torch.float64, device="cuda")
    nll = torch.empty(len(toys), dtype=torch.float64, device="cuda")
    grad = torch.empty(len(toys), batch.stride, dtype=torch.float64, device="cuda")
    st = torch.empty(len(toys), dtype=torch.int32, device="cuda")
    for _ in range(warmup):
        batch.nll_grad(theta, nll, grad, st)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(steps):
        batch.nll_grad(theta, nll, grad, st)
    torch.cuda.synchronize()
    el = time.perf_counter() - ta
    batch.set_profiling(True)
    batch.kernel_times(reset=True)
    for _ in range(max(1, steps // 4)):
        batch.nll_grad(theta, nll, grad, st)
    kt = batch.kernel_times(reset=True)
    batch.set_profiling(False)
    classes = [m.name.split("/")[1] for m in toys]
    out = {"toys": len(toys), "classes": {c: classes.count(c) for c in sorted(set(classes))},
           "evals_per_s": round(len(toys) * steps / el, 1), "ms_per_step": round(el * 1e3 / steps, 3),
           "generator_s": round(gen_s, 1), "status_nonzero": int((st != 0).sum().item()),
           "kernel_ms": {k: round(v[0] / v[1], 3) for k, v in kt.items() if v[1]}}
    th0 = np.zeros_like(th)
    for t, m in enumerate(toys):
        th0[t, : m.n_params] = m.theta0
    th0 = torch.tensor(th0, dtype=torch.float64, device="cuda")
    free, scales = batch.free_masks(toys), batch.scales(toys)
    batch.fit(th0, scales, free=free)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    r = batch.fit(th0, scales, free=free)
    torch.cuda.synchronize()
    el = time.perf_counter() - ta
    stt = r["status"].cpu().numpy()
    out["fits_per_s"] = round(len(toys) / el, 1)
    out["fits_seconds"] = round(el, 3)
    out["fits_converged"] = int(np.sum(stt & 32 != 0))
    # each class of the mix as a batch of its own (same toys): batched evaluations per second
    per_class = {}
    for c in sorted(set(classes)):
        idx = [t for t in range(len(toys)) if classes[t] == c]
        sub = [toys[t] for t in idx]
        b_c = gs.Batch(sub)
        th_c = theta[idx, : b_c.stride].contiguous()
        n_c = torch.empty(len(sub), dtype=torch.float64, device="cuda")
        g_c = torch.empty(len(sub), b_c.stride, dtype=torch.float64, device="cuda")
        s_c = torch.empty(len(sub), dtype=torch.int32, device="cuda")
        for _ in range(warmup):
            b_c.nll_grad(th_c, n_c, g_c, s_c)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(steps):
            b_c.nll_grad(th_c, n_c, g_c, s_c)
        torch.cuda.synchronize()
        el_c = time.perf_counter() - ta
        per_class[c] = {"toys": len(sub), "evals_per_s": round(len(sub) * steps / el_c, 1),
                        "ms_per_step": round(el_c * 1e3 / steps, 3), "status_nonzero": int((s_c != 0).sum().item())}
        del b_c
    out["per_class"] = per_class
    if with_oracle:
        import oracle
        oracle.build(force=False)
        gn, gg = nll.cpu().numpy(), grad.cpu().numpy()
        seen, worst_nll, worst_grad = {}, 0.0, 0.0
        for t, m in enumerate(toys):
            c = classes[t]
            if seen.get(c, 0) >= 2:
                continue
            seen[c] = seen.get(c, 0) + 1
            ov, og, _ = oracle.Oracle(m).nll_grad(m.theta_true)
            worst_nll = max(worst_nll, abs(gn[t] - ov) / abs(ov))
            worst_grad = max(worst_grad, float(np.max(np.abs(gg[t, : m.n_params] - og) * m.fd_scale /
                                                      np.maximum(np.abs(og) * m.fd_scale, 1.0))))
        out["oracle_sample"] = {"toys": sum(seen.values()), "max_rel_dnll": worst_nll, "max_grad_err": worst_grad,
                                "pass": bool(worst_nll <= 1e-11 and worst_grad <= 1e-8)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--toys", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fits", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 16384-toy mixed batch")
    ap.add_argument("--mixed-toys", type=int, default=16384)
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

    base = gsgen.config1()
    toys = gsgen.config3(args.toys, base=base)
    log(f"bench: {len(toys)} pseudo-experiments of the Borexino-scale model, ragged windows")
    batch = gs.Batch(toys)
    stride = batch.stride
    theta = torch.tensor(np.stack([t.theta_true for t in toys]), dtype=torch.float64, device="cuda")
    nll = torch.empty(len(toys), dtype=torch.float64, device="cuda")
    grad = torch.empty(len(toys), stride, dtype=torch.float64, device="cuda")
    st = torch.empty(len(toys), dtype=torch.int32, device="cuda")
    # the batch scheduler's autotuner picks the work layout the timed steps use
    tune = batch.autotune(theta, reps=3)
    log(f"bench: autotune {tune}")
    for _ in range(args.warmup):
        batch.nll_grad(theta, nll, grad, st)
    torch.cuda.synchronize()
    batch.set_profiling(True)
    batch.kernel_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.nll_grad(theta, nll, grad, st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = batch.kernel_times(reset=True)
    batch.set_profiling(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = len(toys) * args.steps / (t1 - t0)
    log(f"bench: {ms_step:.3f} ms/step, {value:.1f} evals/s; kernels " +
        ", ".join(f"{k}={v[0] / max(v[1], 1):.3f}ms" for k, v in kt.items() if v[1]))
    gpu_nll = nll.cpu().numpy()
    gpu_grad = grad.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)

    fold_pairs, adj_pairs, full_pairs, band_pairs = batch.mesh_pairs()
    # the unit of work is a banded-mesh pair: a (window bin, cell) pair whose bin lies in
    # the cell's support; pairs a kernel evaluates beyond those are its own overhead
    executed = {"fold": fold_pairs, "adj": adj_pairs}
    per_kernel = {}
    for k in ("fold", "adj"):
        ms, n = kt[k]
        avg = ms / n
        per_kernel[k] = dict(avg_ms=avg, tflops=band_pairs * FLOPS_PER_PAIR[k] / (avg * 1e-3) / 1e12,
                             executed_over_banded=executed[k] / band_pairs)
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_ms"])
    ach = per_kernel[dom]["tflops"]
    kname = "k_fold1" if dom == "fold" else "k_adj"
    traffic = None
    if (TRAFFIC["sources_sha256"] == sources_sha256() and len(toys) == TRAFFIC["toys"]
            and kname in TRAFFIC["kernels"]):
        traffic = TRAFFIC["kernels"][kname]
    roofline = {"bound": "alu", "kernel": kname, "achieved": round(ach, 3),
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4),
                "traffic": traffic, "flops_per_pair": FLOPS_PER_PAIR[dom], "pairs_per_launch": band_pairs,
                "executed_pairs": executed[dom], "full_mesh_pairs": full_pairs,
                "banded_over_full": round(band_pairs / full_pairs, 4),
                "avg_launch_ms": round(per_kernel[dom]["avg_ms"], 4),
                "other": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in per_kernel.items() if k != dom}}
    pairs = full_pairs

    # single-evaluation latency on one device-resident problem
    single = gs.Batch([toys[0]])
    th1 = theta[:1].clone()
    n1, g1, s1 = (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty(1, stride, dtype=torch.float64,
                                                                               device="cuda"),
                  torch.empty(1, dtype=torch.int32, device="cuda"))
    for _ in range(10):
        single.nll_grad(th1, n1, g1, s1)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    reps = 200
    for _ in range(reps):
        single.nll_grad(th1, n1, g1, s1)
    torch.cuda.synchronize()
    single_us = (time.perf_counter() - ta) * 1e6 / reps

    toy_fits = None
    if not args.no_fits:
        th0 = torch.tensor(np.stack([t.theta0 for t in toys]), dtype=torch.float64, device="cuda")
        free = batch.free_masks(toys)
        batch.fit(th0, base.fd_scale, free=free)  # warm: builds the captured graph
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = batch.fit(th0, base.fd_scale, free=free)
        torch.cuda.synchronize()
        el = time.perf_counter() - ta
        stt = r["status"].cpu().numpy()
        it = r["iters"].cpu().numpy()
        act, tms = batch.fit_trace()
        toy_fits = {"fits_per_s": round(len(toys) / el, 2), "seconds": round(el, 4), "toys": len(toys),
                    "fixed_rates": int(sum(int((~t.free).sum()) for t in toys)),
                    "converged": int(np.sum(stt & 32 != 0)), "mean_iters": round(float(it.mean()), 2),
                    "max_iters": int(it.max()), "graph_launches": int(len(act)),
                    "ms_until_90pct_done": round(float(tms[np.argmax(act <= 0.1 * len(toys))]), 2) if len(act) else None}
        log(f"bench: toy fits {toy_fits}")
        # the same toys fitted one at a time by the host BFGS over single-model evaluations,
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
        toy_fits["one_at_a_time_host"] = one
        log(f"bench: toy fits one at a time {one}")

    fits = None
    if not args.no_fits:
        model = gs.Model(base)
        fits = {}
        for name, fd in (("adjoint", False), ("finite_diff", True)):
            model.fit(base.theta0, base.fd_scale, use_fd=fd)  # warm
            ta = time.perf_counter()
            r = model.fit(base.theta0, base.fd_scale, use_fd=fd, hesse=False)
            el = time.perf_counter() - ta
            fits[name] = dict(fits_per_s=round(1.0 / el, 3), seconds=round(el, 4), iters=r["iters"],
                              n_eval=r["n_eval"], converged=r["ok"], nll=r["nll"])
        fits["speedup_adjoint_over_fd"] = round(fits["finite_diff"]["seconds"] / fits["adjoint"]["seconds"], 2)
        log(f"bench: fits {fits}")

    # the multi-observable model: 12 species x 900 energy x 50 pulse-shape bins x 3 datasets
    two_d = None
    if not args.no_fits:
        c2 = gsgen.config2()
        m2 = gs.Model(c2)
        for _ in range(5):
            m2.nll_grad(c2.theta0)
        ta = time.perf_counter()
        for _ in range(50):
            m2.nll_grad(c2.theta0)
        us2 = (time.perf_counter() - ta) * 1e6 / 50
        two_d = {"bins": int(c2.counts.size), "us_per_eval": round(us2, 2)}
        for name, fd in (("adjoint", False), ("finite_diff", True)):
            m2.fit(c2.theta0, c2.fd_scale, use_fd=fd, hesse=False)
            ta = time.perf_counter()
            r = m2.fit(c2.theta0, c2.fd_scale, use_fd=fd, hesse=False)
            el = time.perf_counter() - ta
            two_d[name] = dict(seconds=round(el, 4), iters=r["iters"], n_eval=r["n_eval"], converged=r["ok"],
                               nll=r["nll"])
        log(f"bench: 2-D model {two_d}")

    mixed = None
    if not args.no_mixed:
        mixed = mixed_batch(gs, gsgen, torch, args.mixed_toys, args.steps, args.warmup, not args.no_cpu)
        log(f"bench: mixed {mixed}")

    cpu = None
    parity = None
    if not args.no_cpu:
        threads = max(1, min(16, os.cpu_count() or 1))
        rate, n_done, el, outs = cpu_baseline(toys, args.cpu_seconds, threads)
        rate1, n1, el1, _ = cpu_baseline(toys, max(2.0, args.cpu_seconds / 3), 1)
        cpu = {"value": round(rate, 4), "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": f"{n_done} oracle -ln L+gradient evaluations of the first {threads} pseudo-experiments "
                         f"(one per thread) in {el:.1f} s",
               "one_thread": {"value": round(rate1, 4), "unit": "evals/s",
                              "sample": f"{n1} evaluations of the first pseudo-experiment in {el1:.1f} s"}}
        rel = max(abs(gpu_nll[i] - outs[i][0]) / abs(outs[i][0]) for i in range(threads))
        gerr = max(np.max(np.abs(gpu_grad[i, :17] - outs[i][1]) * base.fd_scale /
                          np.maximum(np.abs(outs[i][1]) * base.fd_scale, 1.0)) for i in range(threads))
        parity = {"toys_checked": threads, "max_rel_dnll": float(rel), "max_grad_err": float(gerr),
                  "pass": bool(rel <= 1e-11 and gerr <= 1e-8)}
        log(f"bench: cpu {cpu}; parity {parity}")

    out = {"metric": METRIC, "value": round(value, 3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "4096 pseudo-experiments of the Borexino-scale model (12 species, 4000+4 "
                                  "true cells, 900 reco bins, gamma response, 17 params), own rates and "
                                  "200-900-bin windows; one batched -lnL+gradient per step",
                      "toys": len(toys), "mean_window_bins": round(float(np.mean([t.win_hi - t.win_lo for t in toys])), 1),
                      "full_mesh_pairs_per_step": pairs},
           "roofline": roofline, "cpu_baseline": cpu, "parity_sample": parity, "autotune": tune, "toy_fits": toy_fits,
           "single_eval": {"us_per_eval": round(single_us, 2), "evals_per_s": round(1e6 / single_us, 1)},
           "single_fit_borexino_scale": fits, "two_d_model": two_d, "mixed_batch": mixed}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
