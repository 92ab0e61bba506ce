"""Writes fit_goldens.json: oracle fits (analytic gradient, Hesse sigma) of the benchmark
workloads, for the GPU fit-parity test.

Only the oracle (oracle/) and the seeded input generator (gsgen/) are used: no value here
comes from the GPU library.  Each entry holds the recipe that rebuilds its model from gsgen
(config and toy index), the start point, free mask and parameter scales of the fit, and the
oracle's fitted parameters, Hesse sigma (central differences of the analytic gradient,
inverted), -ln L at the minimum, status and iteration count.

Cases: the 1-D energy-family model (config 0), the Borexino-scale model (config 1), the
pulse-shape model with three datasets (config 2), eight seeded pseudo-experiments of the
ragged-window toy study (config 3, with their free-parameter masks) and the first toy of each
class of the uneven mix (config 4).  Run from the repository root:

    python tests/golden/make_fit_goldens.py

It takes a few minutes on 8 host cores (one fit per thread).
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gsgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fit_goldens.json")
C3_POOL = 64      # toys 0..63 of the toy study; 8 drawn from them with a fixed seed
C4_TOYS = 48      # the first toy of each class among the first 48 of the mix


def cases():
    """(key, recipe, model, theta0, free mask, scale) of every golden fit."""
    out = []
    for key, fn in (("c0", gsgen.config0), ("c1", gsgen.config1), ("c2", gsgen.config2)):
        m = fn()
        out.append((key, {"config": key}, m, m.theta0, m.free_mask(), m.fd_scale))
    base = gsgen.config1()
    toys = gsgen.config3(C3_POOL, base=base)
    for t in sorted(np.random.default_rng(1812).choice(C3_POOL, 8, replace=False).tolist()):
        m = toys[t]
        out.append((f"c3/{t}", {"config": "c3", "toy": t, "pool": C3_POOL}, m, m.theta0, m.free_mask(),
                    base.fd_scale))
    mix = gsgen.config4(C4_TOYS)
    seen = set()
    for t, m in enumerate(mix):
        cls = m.name.split("/")[1]
        if cls in seen:
            continue
        seen.add(cls)
        out.append((f"c4/{cls}/{t}", {"config": "c4", "toy": t, "pool": C4_TOYS}, m, m.theta0, m.free_mask(),
                    m.fd_scale))
    return out


def fit_one(item):
    key, recipe, m, th0, free, scale = item
    t0 = time.perf_counter()
    r = oracle.Oracle(m).fit(th0, free=free, scale=scale, hesse=True)
    el = time.perf_counter() - t0
    print(f"{key}: ok={r['ok']} nll={r['nll']:.12g} iters={r['iters']} n_eval={r['n_eval']} {el:.1f}s", flush=True)
    return key, dict(recipe=recipe, theta0=np.asarray(th0, float).tolist(), free=np.asarray(free, int).tolist(),
                     scale=np.asarray(scale, float).tolist(), theta_hat=r["theta"].tolist(),
                     sigma=r["sigma"].tolist(), nll=r["nll"], status=int(r["status"]), iters=int(r["iters"]),
                     ok=bool(r["ok"]), oracle_seconds=round(el, 1))


def main():
    oracle.build(force=False)
    items = cases()
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = dict(ex.map(fit_one, items))
    doc = {"about": "oracle fits (analytic gradient, BFGS to EDM < 1e-9, Hesse sigma) of seeded synthetic "
                    "workloads; written by tests/golden/make_fit_goldens.py from oracle/ and gsgen/ only",
           "edm_tol": 1e-9, "max_iter": 500,
           "cases": {k: res[k] for k, *_ in items}}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
