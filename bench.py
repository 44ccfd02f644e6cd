"""Benchmark: softabs RMHMC throughput at D = 1038 (N = 1024 latent values,
14 kernel hyperparameters).

One step = one generalized leapfrog (Eq. leapfrog of the paper) inside the
RMHMC chain of Algorithm 1, run entirely on the device: K Hessian assemblies
and warm-started Jacobi eigendecompositions for the implicit position update,
the contraction precompute at the new point, K + 2 structured third-derivative
contractions for the two momentum half steps, and per move of C leapfrogs the
momentum draw and the Metropolis-Hastings test.  The timed steps continue the
chain of the warmup steps; an ESS chain continues after them.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

Prints one JSON line.  Only one GPU is used; --gpus above 1 is refused.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64_tflops": 78.6, "f32_tflops": 157.3, "hbm_gbs": 8000.0}
# The dominant kernel by time is the Jacobi round kernel (subproblem solves of
# round r+1 beside the Psi update of round r).  Its algorithmic intensity,
# about 4.5 flop/byte, is below the FP64 ridge point of 78.6 TFLOP/s over
# 8 TB/s (~10 flop/byte), so its roofline is HBM.  The FP64 MFMA GEMMs, which
# carry most of the flops, are reported beside it.
DOMINANT = "jacobi_round"
DOMINANT_KERNEL = "jacobi_round_kernel<1>"   # warm-started (one inner sweep)
GEMM = "gemm_f64"
TRAFFIC_FILE = "profiles/jacobi_round_kernel_dynamic_propensity_mkl_d1038_traffic.json"
TRAFFIC_SOURCES = ("paper_2511_06407_amd/csrc/eig.hip",)


# The paper's own timing for its basis-model workloads, on other hardware:
# context only.  Its convergence runs took about 14,000 s (d = 34) and
# 60,000 s (d = 484) on one A100 driven by one Xeon core (Sec. 3.1); taken
# as the full 9,600 moves of 100 leapfrogs each (Sec. 2.5) that is the rate
# below (a derived figure: the paper prints no per-leapfrog rate).
PAPER_CONTEXT = {
    "basis_logistic_d34": {"leapfrog_per_s": 68.6, "hardware": "A100 PCIe 80GB + 1 Xeon core",
                           "derivation": "960,000 leapfrogs in ~14,000 s (Sec. 3.1, Sec. 2.5)"},
    "basis_logistic_d484": {"leapfrog_per_s": 16.0, "hardware": "A100 PCIe 80GB + 1 Xeon core",
                            "derivation": "960,000 leapfrogs in ~60,000 s (Sec. 3.1, Sec. 2.5)"},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="propensity_mkl_d1038")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="skip the per-kernel event timing (use under a profiler)")
    ap.add_argument("--ess-moves", type=int, default=40,
                    help="moves of the ESS chain run after the timed steps (0: none)")
    ap.add_argument("--ess-burnin", type=int, default=-1,
                    help="burn-in moves of the ESS chain (default: a quarter)")
    ap.add_argument("--eps", type=float, default=0.0, help="step size (default: the workload's)")
    ap.add_argument("--leapfrogs", type=int, default=0,
                    help="leapfrogs per move C (default: the workload's)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--calib-copy-mb", type=float, default=0.0,
                    help="run one device-to-device copy of this many MB before the timed "
                         "steps (a kernel of known traffic for scaling PMC byte counters)")
    ap.add_argument("--mode", choices=["leapfrog", "tempered", "serve"], default="leapfrog",
                    help="leapfrog: one chain at D=1038 (default); tempered: 64 power-posterior "
                         "chains of uneven D on the worker pool; serve: Poisson request stream")
    ap.add_argument("--chains", type=int, default=64)
    ap.add_argument("--moves", type=int, default=4, help="moves per chain (tempered mode)")
    ap.add_argument("--workers", type=int, default=8, help="streams (graph) or workers (pool)")
    ap.add_argument("--engine", choices=["graph", "pool"], default="pool",
                    help="tempered mode: graph-captured batch or eager worker pool")
    ap.add_argument("--rate", type=float, default=4.0, help="requests/s (serving)")
    ap.add_argument("--duration", type=float, default=10.0,
                    help="arrival window in s (serving; 0 leaves the serving block out)")
    ap.add_argument("--moves-scale", type=float, default=0.01,
                    help="fraction of the serving mix's 200..2000 moves per request")
    ap.add_argument("--hbm-gb", type=float, default=200.0, help="admission budget (serve)")
    return ap.parse_args()


def run_tempered_mode(args):
    from paper_2511_06407_amd.tempered import run_tempered
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)  # noqa: E731
    from paper_2511_06407_amd import rmhmc
    out = run_tempered(n_chains=args.chains, n_moves=args.moves, n_leapfrog=10, n_fixed_point=6,
                       eps=0.01, n_workers=args.workers, seed=args.seed, log=log,
                       engine=args.engine,
                       precision=rmhmc.MIXED if args.precision == "mixed" else rmhmc.FP64)
    dims = [c["D"] for c in out["chains"]]
    return {"metric": "tempered chains: aggregate chain-leapfrogs/s", "value": out["chain_leapfrogs_per_s"],
            "unit": "chain-leapfrogs/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f64" if args.precision == "fp64" else "f32+f64",
            "data": "synthetic", "wall_s": out["wall_s"], "setup_s": out["setup_s"],
            "config": {"workload": f"{args.chains} power-posterior chains, beta_k=(k/{args.chains - 1})^5, "
                                   "D from {66,130,258,514}", "moves": args.moves, "n_leapfrog": 10,
                       "workers": args.workers, "engine": args.engine, "dims": dims},
            "shapes": {str(c["D"]): c["shape"] for c in out["chains"]},
            "fail_noconv": sum(c["fail_noconv"] for c in out["chains"]),
            "accept": [c["accepted"] for c in out["chains"]],
            "failures": sum(c["failures"] for c in out["chains"])}


def serving_block(rate, window_s, moves_scale, workers, hbm_gb, seed, precision="fp64"):
    """Requests of the serving mix (D log-uniform on [34, 1038], GP-logistic
    or multiple-kernel) arriving as a Poisson stream, with the move counts
    scaled by moves_scale; latencies and the backlog as measured."""
    from paper_2511_06407_amd.serve_bench import run_rate
    lo = max(1, int(round(200 * moves_scale)))
    hi = max(lo, int(round(2000 * moves_scale)))
    from paper_2511_06407_amd import rmhmc
    out = run_rate(rate, window_s, (lo, hi), workers, 32, hbm_gb, seed,
                   precision=rmhmc.MIXED if precision == "mixed" else rmhmc.FP64)
    out["moves_scale"] = moves_scale
    out["precision"] = precision
    out["note"] = ("requests of the serving mix with 1/{:g} of its move counts; a sustainable "
                   "rate r here is r x {:g} requests/s at full length".format(1 / moves_scale,
                                                                              moves_scale))
    return out


def run_serve_mode(args):
    summ = serving_block(args.rate, args.duration, args.moves_scale, args.workers, args.hbm_gb,
                         args.seed, args.precision)
    return {"metric": "serving: p50/p99 request latency", "value": summ["p99_latency_s"],
            "unit": "s (p99 latency)", "n_gpus": 1, "higher_is_better": False,
            "dtype": "f64" if args.precision == "fp64" else "f32+f64",
            "data": "synthetic", **summ,
            "config": {"workload": "Poisson arrivals, D log-uniform in [34,1038], GP-logistic or "
                                   "multiple-kernel", "rate_per_s": args.rate,
                       "duration_s": args.duration, "moves_scale": args.moves_scale,
                       "workers": args.workers, "hbm_budget_gb": args.hbm_gb}}


def file_hash(*paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_src_hash):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, only if it was taken on the current kernel source."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_src_hash:
        return None
    return d.get("bytes_per_launch")


def lscpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, cfg):
    """The FP64 reference timed on the host cores on a bounded sample: one
    whole generalized leapfrog (K Hessians and eigendecompositions, K + 2
    contractions) from the chain's start point, first with all BLAS threads,
    then with one (the paper drove its GPU from one core).  The start point's
    own metric, which a chain carries over from the previous leapfrog, is
    set up outside the timed region."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import hamiltonian as oham
    from oracle.chain import momentum
    from oracle.integrator import glf_step
    from oracle import basis as obasis, softabs as osoft
    from paper_2511_06407_amd import workloads as wl
    T = obasis.BasisTarget(spec) if isinstance(spec, wl.BasisSpec) else oham.GPTarget(spec)
    amap = osoft.SqrtMap(1.0 / cfg.alpha) if cfg.sqrt_map else cfg.alpha
    q = wl.start_point(spec)
    z = np.random.default_rng(0).standard_normal(spec.D)

    def sample():
        st = oham.State(T, q, amap)
        p = momentum(st, z)
        t0 = time.perf_counter()
        glf_step(st, p, cfg.eps, cfg.n_fixed_point)
        return time.perf_counter() - t0

    cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    t_all = sample()
    with threadpool_limits(limits=1):
        t_one = sample()
    return {"value": 1.0 / t_all, "unit": "leapfrog steps/s", "cores": int(cores),
            "kind": "oracle", "cpu_model": lscpu_model(),
            "value_1_thread": 1.0 / t_one,
            "sample": (f"1 generalized leapfrog (K={cfg.n_fixed_point}) from the start point of the "
                       f"{spec.D}-dim workload: {t_all:.1f} s on {cores} threads, "
                       f"{t_one:.1f} s on 1 thread"),
            "seconds": t_all + t_one}


def algorithmic_flops(N, P, D, K):
    """Flops of one generalized leapfrog by textbook counts: Cholesky N^3/3,
    inverse 2N^3/3, GEMM 2mnk, 4.3 D^3 per eigendecomposition with vectors;
    K metric evaluations ((1 + 2P) N^3 + 4.3 D^3 each), K + 1 W1 builds
    (4 D^3), one W2 build (2 D^3), K + 2 contractions (2 N^3 each) and the
    per-point trace tensor (min(2P(K + 2), P(P + 1)) N^3)."""
    return (K * ((1 + 2 * P) * N ** 3 + 4.3 * D ** 3) + (K + 1) * 4 * D ** 3 + 2 * D ** 3
            + (K + 2) * 2 * N ** 3 + min(2 * P * (K + 2), P * (P + 1)) * N ** 3)


def basis_flops(N, F, D, K):
    """The same count for the basis model: K metric evaluations (the
    likelihood Hessian Phi' diag(l'') Phi, 2 N (F + 1)^2, and 4.3 D^3), K + 1
    W1 builds, one W2 build and K + 2 contractions (Phi W, 2 N (F + 1)^2)."""
    Fa = F + 1
    return (K * (2 * N * Fa ** 2 + 4.3 * D ** 3) + (K + 1) * 4 * D ** 3 + 2 * D ** 3
            + (K + 2) * 2 * N * Fa ** 2)


def softabs_kind(cfg):
    from paper_2511_06407_amd import rmhmc
    return rmhmc.SOFTABS_SQRT if cfg.sqrt_map else rmhmc.SOFTABS_COTH


def run_chain_steps(model, cfg, q0_dev, n_steps, seed, stream_id, burn=False):
    """n_steps leapfrogs of the device chain from q0: moves of C leapfrogs and
    one shorter move for the remainder.  Returns (seconds, last sample, stats
    list, (samples, logpost, accepted) of the full moves)."""
    import torch
    C = cfg.n_leapfrog
    parts = [(n_steps // C, C)] if n_steps >= C else []
    if n_steps % C:
        parts.append((1, n_steps % C))
    q = q0_dev
    stats, out = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (moves, lf) in enumerate(parts):
        s, l, a, st = model.chain(q, cfg.eps, lf, cfg.n_fixed_point, moves, seed=seed,
                                  stream_id=stream_id + i, alpha=cfg.alpha,
                                  softabs=softabs_kind(cfg))
        q = s[-1].clone()
        stats.append(st)
        if out is None:
            out = (s, l, a)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, q, stats, out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py: the sampler runs on one GPU; --gpus above 1 is not supported "
              "(chains and requests would be assigned to GPUs whole)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2511_06407_amd import rmhmc, workloads as wl

    if args.mode == "tempered":
        print(json.dumps(run_tempered_mode(args)), flush=True)
        return
    if args.mode == "serve":
        print(json.dumps(run_serve_mode(args)), flush=True)
        return
    spec, cfg = wl.workload(args.workload, args.seed)
    if args.eps > 0:
        cfg.eps = args.eps
    if args.leapfrogs > 0:
        cfg.n_leapfrog = args.leapfrogs
    basis = isinstance(spec, wl.BasisSpec)
    if basis:
        if args.precision != "fp64":
            sys.exit("bench.py: the basis model runs in FP64 only")
        model = rmhmc.BasisModel(spec)
    else:
        model = rmhmc.Model(spec, rmhmc.MIXED if args.precision == "mixed" else rmhmc.FP64)
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)  # noqa: E731
    q0 = torch.tensor(wl.start_point(spec), dtype=torch.float64, device="cuda")
    log(f"model ready D={spec.D} ({model.device_bytes / 2**30:.2f} GiB on the device)")
    q = q0
    if args.warmup > 0:
        tw, q, _, _ = run_chain_steps(model, cfg, q0, args.warmup, args.seed, 100)
        log(f"warmup {args.warmup} leapfrogs in {tw:.2f} s")
    if args.calib_copy_mb > 0:
        n = int(args.calib_copy_mb * 1e6 / 8)
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy of {8 * n} bytes done")
        del a, b
    elapsed, q, st_list, _ = run_chain_steps(model, cfg, q, args.steps, args.seed, 200)
    done = sum(st.leapfrogs for st in st_list)
    log(f"timed {args.steps} steps ({done} completed) in {elapsed:.3f} s")
    # a failed move is abandoned once the host sees it, so count the
    # leapfrogs that ran
    value = done / elapsed
    eig_calls = sum(st.eig_calls for st in st_list)
    sweeps = sum(st.sweeps for st in st_list)
    F = (basis_flops(spec.N, spec.n_features, spec.D, cfg.n_fixed_point) if basis
         else algorithmic_flops(spec.N, spec.P, spec.D, cfg.n_fixed_point))

    roofline = None
    roofline_gemm = None
    if not args.no_timing:
        # per-kernel HIP events on the launch stream, over further chain
        # leapfrogs kept out of the timed region above
        n_inst = min(args.steps, cfg.n_leapfrog)
        rmhmc.timing_enable((DOMINANT, GEMM))
        t_inst, q_inst, st_inst, _ = run_chain_steps(model, cfg, q, n_inst, args.seed, 300)
        log(f"instrumented {n_inst} steps in {t_inst:.3f} s")
        n, ms, flops, byts = rmhmc.timing_read(DOMINANT)
        gn, gms, gflops, _ = rmhmc.timing_read(GEMM)
        rmhmc.timing_enable(())
        # warm-started eigendecompositions only: each chain call starts with a
        # static solve (and a fallback is another), timed as their own family
        inst_eigs = sum(st.eig_calls - 1 - st.eig_fallbacks for st in st_inst)
        if n > 0 and ms > 0:
            # the unit of work of the eigensolver is one eigendecomposition,
            # 4.3 D^3 flops by the textbook count; a round launch does
            # eig_calls / launches of one
            per_launch = 4.3 * spec.D ** 3 * inst_eigs / n
            avg_s = ms * 1e-3 / n
            achieved = per_launch / avg_s / 1e12
            roofline = {"bound": "mfma", "kernel": DOMINANT_KERNEL,
                        "achieved": round(achieved, 4), "peak": PEAK["f64_tflops"],
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK["f64_tflops"], 5),
                        "traffic": traffic_from_profile(file_hash(*TRAFFIC_SOURCES)),
                        "algorithmic_flops_per_launch": per_launch,
                        "launches": n, "eigendecompositions": inst_eigs,
                        "avg_launch_us": round(avg_s * 1e6, 2),
                        "kernel_time_share": round(ms * 1e-3 / t_inst, 3),
                        "hbm_view": {"algorithmic_bytes_per_launch": byts / n,
                                     "achieved_gbs": round(byts / n / avg_s / 1e9, 1),
                                     "peak_gbs": PEAK["hbm_gbs"]}}
        if gn > 0 and gms > 0:
            ga = gflops / (gms * 1e-3) / 1e12
            roofline_gemm = {"bound": "mfma", "kernel": "gemm_kernel<double> (v_mfma_f64_16x16x4f64)",
                             "achieved": round(ga, 3), "peak": PEAK["f64_tflops"], "unit": "TFLOP/s",
                             "frac": round(ga / PEAK["f64_tflops"], 4), "launches": gn,
                             "avg_launch_us": round(gms * 1e3 / gn, 2),
                             "kernel_time_share": round(gms * 1e-3 / t_inst, 3)}
        q = q_inst

    ess_block = None
    if args.ess_moves > 0:
        from paper_2511_06407_amd.analysis import ess_summary
        nm = args.ess_moves
        burn = args.ess_burnin if args.ess_burnin >= 0 else nm // 4
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        samples, logpost, acc, stats = model.chain(q, cfg.eps, cfg.n_leapfrog, cfg.n_fixed_point,
                                                   nm, n_burnin=burn, seed=args.seed,
                                                   stream_id=400, alpha=cfg.alpha,
                                                   softabs=softabs_kind(cfg))
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        sm, lp = samples.cpu().numpy(), logpost.cpu().numpy()
        es = ess_summary(sm, lp)
        kept_time = (c1 - c0) * (nm - burn) / nm
        ess_block = {"moves": nm, "burn_in": burn, "eps": cfg.eps,
                     "leapfrogs_per_move": cfg.n_leapfrog, "seconds": c1 - c0,
                     "failures": stats.failures, "fail_not_pd": stats.fail_not_pd,
                     "fail_nonfinite": stats.fail_nonfinite, "fail_noconv": stats.fail_noconv,
                     "eig_fallbacks": stats.eig_fallbacks,
                     "accept_rate_kept": stats.accepted / max(nm - burn, 1),
                     "accept_rate_all": stats.accepted_all / nm,
                     "ess_min": es["min"], "ess_median": es["median"], "ess_logpost": es["logpost"],
                     "ess_min_per_sec": es["min"] / kept_time,
                     "ess_median_per_sec": es["median"] / kept_time,
                     "ess_logpost_per_sec": es["logpost"] / kept_time,
                     "chain_leapfrogs_per_sec": stats.leapfrogs / (c1 - c0),
                     "max_fixed_point_residual": [stats.max_res_p, stats.max_res_q],
                     "hyper_mean": [float(x) for x in sm[:, spec.D - spec.P:].mean(0)]}

    out = {"metric": "leapfrog steps/sec + ESS/sec at D=1036; p50/p99 request latency",
           "value": value, "unit": "leapfrog steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / max(done, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": args.workload, "D": spec.D, "N": spec.N, "P": spec.P,
                      "eps": cfg.eps, "n_leapfrog": cfg.n_leapfrog,
                      "n_fixed_point": cfg.n_fixed_point, "alpha": cfg.alpha,
                      "precision": args.precision, "parallelism": "single GPU",
                      "softabs": "sqrt" if cfg.sqrt_map else "coth"},
           "roofline": roofline, "roofline_gemm_f64": roofline_gemm,
           "whole_step": {"algorithmic_flops": F,
                          "achieved_tflops": round(F * value / 1e12, 3),
                          "frac_f64_peak": round(F * value / 1e12 / PEAK["f64_tflops"], 4)},
           "chain": {"leapfrogs_completed": done,
                     "accepted": sum(st.accepted for st in st_list),
                     "failures": sum(st.failures for st in st_list),
                     "eig_fallbacks": sum(st.eig_fallbacks for st in st_list),
                     "stats": [st.as_dict() for st in st_list]}}
    out["eig"] = {"eig_calls": eig_calls, "sweeps": sweeps,
                  "sweeps_per_eig": sweeps / max(eig_calls, 1),
                  "note": "in the timed chain (its first point is a static solve)"}
    if ess_block is not None:
        out["ess"] = ess_block
    if args.duration > 0:
        model.close()
        log(f"serving: {args.rate} requests/s for {args.duration} s")
        out["serving"] = serving_block(args.rate, args.duration, args.moves_scale, args.workers,
                                       args.hbm_gb, args.seed, args.precision)
        log(f"serving: p50 {out['serving']['p50_latency_s']:.2f} s "
            f"p99 {out['serving']['p99_latency_s']:.2f} s")
    if args.workload in PAPER_CONTEXT:
        out["paper_context"] = PAPER_CONTEXT[args.workload]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
