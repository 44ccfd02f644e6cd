"""Serving measurement: Poisson arrivals of sampling requests of mixed
dimension, run with continuous admission on the worker pool.

The request mix is the serving workload's: D log-uniform on [34, 1038],
the model a fair coin between GP-logistic (P = 2) and the multiple-kernel
propensity model (P = 14), per-request seed = request id.  Its run lengths
(200..2000 moves of 10 leapfrogs) put the offered load far above what one
GPU sustains at 20 requests/s, so the measurement runs the same mix with the
move counts scaled by --moves-scale (work per request is linear in the move
count, so a sustainable rate r at scale s is r*s at full length) and sweeps
the arrival rate upwards, stopping at the first rate whose backlog does not
clear, to find the largest rate whose queue stays bounded.

    python -m paper_2511_06407_amd.serve_bench --rates 0.5,1,2,4,8,16,20 --window 15

prints one JSON line per rate.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import serving as sv


def run_rate(rate, window_s, moves, n_workers, n_slots, budget_gb, seed, n_leapfrog=10,
             precision=None):
    reqs = sv.make_requests(rate, window_s, moves=moves, seed=seed)
    if not reqs:
        return None
    ex = sv.PoolExecutor(n_workers=n_workers, n_leapfrog=n_leapfrog, precision=precision)
    sch = sv.Scheduler(ex, hbm_budget_bytes=budget_gb * 1e9, n_slots=n_slots)
    t0 = time.perf_counter()
    sch.run(reqs)
    wall = time.perf_counter() - t0
    ex.close()
    out = sv.summarize(reqs, wall, sch.queue_depth)
    svc = np.array([r.done_s - r.admit_s for r in reqs])
    out.update({"rate_per_s": rate, "window_s": window_s, "moves": list(moves),
                "n_leapfrog": n_leapfrog, "workers": n_workers, "slots": n_slots,
                "p50_service_s": float(np.percentile(svc, 50)),
                "p99_service_s": float(np.percentile(svc, 99)),
                "max_running": sch.max_running, "max_hbm_gb": sch.max_in_use / 1e9,
                "drain_s": wall - window_s,
                "D_mean": float(np.mean([r.D for r in reqs]))})
    # sustained: the backlog left when arrivals stop clears within a quarter
    # of the window plus the longest single service (above capacity the
    # backlog grows as (rate - capacity) x window)
    out["sustained"] = bool(out["drain_s"] < 0.25 * window_s + float(svc.max()))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--rates", default="0.5,1,2,4,8,16,20", help="ascending")
    ap.add_argument("--window", type=float, default=15.0, help="seconds of arrivals per rate")
    ap.add_argument("--moves-scale", type=float, default=0.01)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    lo = max(1, int(round(200 * a.moves_scale)))
    hi = max(lo, int(round(2000 * a.moves_scale)))
    best = None
    for rate in [float(x) for x in a.rates.split(",")]:
        print(f"[serve] rate {rate}/s window {a.window} s moves {lo}..{hi}", file=sys.stderr,
              flush=True)
        out = run_rate(rate, a.window, (lo, hi), a.workers, a.slots, a.budget_gb, a.seed)
        if out is None:
            continue
        out["moves_scale"] = a.moves_scale
        print(json.dumps(out), flush=True)
        if not out["sustained"]:
            break              # rates are swept upwards: stop at the first overload
        best = rate
    print(json.dumps({"sustainable_rate_per_s": best, "moves_scale": a.moves_scale,
                      "full_length_equivalent_per_s": None if best is None else best * a.moves_scale}),
          flush=True)


if __name__ == "__main__":
    main()
